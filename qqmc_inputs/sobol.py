"""Sobol' point sets (the paper's generator, App. B) as inputs: direction
numbers and random digital shifts.

Nothing here is taken from a published table.  The construction follows
Sobol' (and the Bratley-Fox form of the recurrence):
  * dimension 1 is the van der Corput sequence in base 2 (every direction
    number m_k = 1);
  * dimension j >= 2 uses the (j-1)-th primitive polynomial over GF(2),
    x^s + a_1 x^{s-1} + ... + a_{s-1} x + 1, in order of degree and then of
    the coefficient bits, found here by testing the order of x;
  * its first s direction numbers m_1..m_s (m_k odd, m_k < 2^k) are chosen
    among seeded random candidates by the quality of the two-dimensional
    projections onto every earlier dimension (the criterion of Joe and Kuo:
    the t-values of those projections as (t, m, 2)-nets, summed over
    m = 1..M), the rest follow from the recurrence
      m_k = 2 a_1 m_{k-1} ^ 4 a_2 m_{k-2} ^ ... ^ 2^{s-1} a_{s-1} m_{k-s+1}
            ^ 2^s m_{k-s} ^ m_{k-s};
  * point i has coordinates x_j = (XOR over the set bits k of i of
    V_{j,k}) * 2^-32 with V_{j,k} = m_k 2^{32-k}; a random digital shift
    XORs a uniform 32-bit word into each coordinate (the randomisation that
    keeps the net property and gives an unbiased estimate per shift).
"""
from functools import lru_cache
from typing import List, Tuple

import numpy as np

BITS = 32


def _is_primitive(poly: int, s: int) -> bool:
    """poly: bit mask of x^s + ... + 1 (bit k = coefficient of x^k)."""
    if not (poly & 1) or (poly >> s) != 1:
        return False
    period = (1 << s) - 1
    r = 1                                   # x^0
    for k in range(1, period + 1):
        r <<= 1                             # multiply by x
        if r >> s & 1:
            r ^= poly
        if r == 1:
            return k == period
    return False


@lru_cache(maxsize=None)
def primitive_polynomials(count: int) -> Tuple[Tuple[int, int], ...]:
    """The first `count` primitive polynomials as (degree s, mask), by
    degree, then by the mask."""
    out: List[Tuple[int, int]] = []
    s = 1
    while len(out) < count:
        for mid in range(1 << (s - 1)):
            poly = (1 << s) | (mid << 1) | 1
            if _is_primitive(poly, s):
                out.append((s, poly))
                if len(out) == count:
                    break
        s += 1
    return tuple(out)


def _direction_numbers(s: int, poly: int, m_init: List[int]) -> List[int]:
    """m_1..m_BITS from the initial m_1..m_s and the recurrence."""
    m = list(m_init)
    a = [(poly >> (s - i)) & 1 for i in range(1, s)]   # a_1 .. a_{s-1}
    for k in range(s + 1, BITS + 1):
        v = m[k - s - 1] ^ (m[k - s - 1] << s)
        for i in range(1, s):
            if a[i - 1]:
                v ^= m[k - i - 1] << i
        m.append(v)
    return m


def _v_from_m(m: List[int]) -> np.ndarray:
    return np.array([(m[k - 1] << (BITS - k)) & 0xFFFFFFFF for k in range(1, BITS + 1)],
                    dtype=np.uint64).astype(np.uint32)


def _rows(v: np.ndarray, m: int) -> List[int]:
    """Generating-matrix rows r = 1..m (most significant output bit first)
    restricted to index bits 1..m, as bit masks over the columns."""
    rows = []
    for r in range(1, m + 1):
        mask = 0
        for k in range(1, m + 1):
            if (int(v[k - 1]) >> (BITS - r)) & 1:
                mask |= 1 << (k - 1)
        rows.append(mask)
    return rows


def _independent(vectors: List[int]) -> bool:
    basis: List[int] = []
    for x in vectors:
        for b in basis:
            x = min(x, x ^ b)
        if x == 0:
            return False
        basis.append(x)
    return True


def t_value_2d(v1: np.ndarray, v2: np.ndarray, m: int) -> int:
    """Quality t of the first 2^m points of a two-dimensional digital net:
    the smallest t with the first d1 rows of C1 and the first d2 rows of C2
    linearly independent for every d1 + d2 = m - t."""
    r1, r2 = _rows(v1, m), _rows(v2, m)
    for t in range(0, m + 1):
        d = m - t
        if all(_independent(r1[:d1] + r2[:d - d1]) for d1 in range(d + 1)):
            return t
    return m


@lru_cache(maxsize=None)
def _directions(n: int, seed: int, candidates: int, m_max: int) -> Tuple[Tuple[int, ...], ...]:
    from . import SplitMix64
    rng = SplitMix64(seed)
    vs = [_v_from_m([1] * BITS)]
    for s, poly in primitive_polynomials(max(n - 1, 0))[: n - 1]:
        best, best_score = None, None
        for _ in range(candidates):
            m_init = [1 | (int(rng.uniform() * (1 << k)) & ((1 << k) - 1)) for k in range(1, s + 1)]
            v = _v_from_m(_direction_numbers(s, poly, m_init))
            score = sum(t_value_2d(u, v, m) for u in vs for m in range(1, m_max + 1))
            if best_score is None or score < best_score:
                best, best_score = v, score
        vs.append(best)
    return tuple(tuple(int(x) for x in v) for v in vs)


def direction_numbers(n: int, seed: int = 2718, candidates: int = 32,
                      m_max: int = 12) -> np.ndarray:
    """(n, 32) uint32: V_{j,k} for dimensions j = 0..n-1 and index bits
    k = 0..31 (bit k of the point index selects V_{j,k})."""
    return np.array(_directions(int(n), int(seed), int(candidates), int(m_max)),
                    dtype=np.uint64).astype(np.uint32).reshape(n, BITS)


def digital_shifts(seed: int, n_shifts: int, n: int) -> np.ndarray:
    """(n_shifts, n) uint32 uniform words from one SplitMix64 stream."""
    from . import SplitMix64
    rng = SplitMix64(seed)
    out = np.zeros((n_shifts, n), dtype=np.uint32)
    for s in range(n_shifts):
        for j in range(n):
            out[s, j] = int(rng.next_u64() >> 32)
    return out
