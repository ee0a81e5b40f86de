"""Algorithmic FP64 operation counts of the shared-prefix elimination tree.

Counting rules (real double-precision operations): add, subtract, multiply
and divide count 1, a fused multiply-add counts 2, negation and selection
count 0.  Complex helpers: add/sub 2, multiply 6, multiply-add 8, reciprocal
6 (|p|^2, one division, two products).

``tree_flops(n)`` is the work of the elimination tree over the 2^n Keldysh
index vectors of ONE point with every tree node visited exactly once (the
work the method needs); ``lane_flops(n)`` is what the kernel actually issues,
including the per-lane recomputation of the top levels (for efficiency
accounting only).
"""


def _node(m):
    """Tree node holding an m x m trailing block, m > 2: pivot, reciprocal,
    pivot product, and for both indices the pivot row/column and the rank-1
    update of the (m-1)^2 child block."""
    return 2 + 6 + 6 + 2 * (2 * (m - 1) + 8 * (m - 1) + 8 * (m - 1) ** 2)


LEAF_PAIR = 2 + 8 + 6 + 8 + 18 + 2   # last vertex + measurement, both indices
PAIR_LOOKUP = 16                     # two interpolations (g^<, g^>) per pair
POINT_EPILOGUE = 12                  # prefactor, weight, compensated add


def tree_flops(n):
    """Per point inside the domain."""
    total = 0
    for k in range(n - 1):           # levels with blocks of size n+1-k > 2
        total += (1 << k) * _node(n + 1 - k)
    total += (1 << (n - 1)) * LEAF_PAIR
    return total + PAIR_LOOKUP * n * (n + 1) // 2 + POINT_EPILOGUE


def warp_flops(n):
    """Per lattice point (lattice arithmetic, inverse CDF, weight; each
    transcendental counted as one operation)."""
    return 8 * n + 2


def geometry(n):
    """Block size K, cooperative top levels, per-lane path levels T (each
    lane walks a register tree of depth at most 5)."""
    K = min(n, 8) + 1
    off = n + 1 - K
    T = K - 6 if K - 1 > 5 else 0
    return K, off, T


def lane_flops(n):
    """Operations the kernel issues per point inside the domain."""
    K, off, T = geometry(n)
    path = 0
    for k in range(T):
        path += 2 + 8 * k + 6 + (K - 1 - k) * (10 + 16 * k) + 6
    ct = (K - T) ** 2 * 8 * T
    sub = 0
    for lvl in range(T, K - 2):
        sub += (1 << (lvl - T)) * _node(K - lvl)
    sub += (1 << (K - 2 - T)) * LEAF_PAIR
    per_item = (1 << T) * (path + ct + sub)
    top = 0
    for k in range(off):
        rows = n - k
        top += 2 * (n + 1 - k) + rows * (2 + 6 + 6 + 8 * rows) + 6
    items = 1 << off
    return items * (per_item + top + PAIR_LOOKUP * n * (n + 1) // 2) + POINT_EPILOGUE
