"""Algorithmic FP64 operation counts of the shared-prefix elimination tree.

Counting rules (real double-precision operations): add, subtract, multiply
and divide count 1, a fused multiply-add counts 2, negation and selection
count 0.  Complex helpers: add/sub 2, multiply 6, multiply-add 8, reciprocal
6 (|p|^2, one division, two products).

``tree_flops(n)`` is the work of the tree over the 2^n Keldysh index vectors
of ONE point with every tree node visited exactly once, in the form the
kernel evaluates it: elimination nodes down to 4x4 blocks, the 3x3 nodes by
cofactors, the leaf bracket from per-point constants (the work the method
needs).  ``lane_flops(n)`` is what the kernel actually issues, including the
per-lane recomputation of the levels above each lane's subtree (for
efficiency accounting only).
"""


def _node(m):
    """Elimination node holding an m x m trailing block, m >= 4: pivot,
    reciprocal, for both indices the pivot row/column and the rank-1 update
    of the (m-1)^2 child block except its measurement diagonal (never read),
    and the relative sum p^2 (V_0 - V_1)."""
    return 2 + 6 + 2 * (2 * (m - 1) + 8 * (m - 1) + 8 * ((m - 1) ** 2 - 1)) + 14


# 3x3 node by cofactors: S_ww, p S_ww, p d (d from the leaf constants), and
# for both indices of u four entries, two products, the bracket, the 2x2
# determinant and the product; then the difference.
NODE3 = 2 + 6 + (16 + 6) + 2 * (8 + 12 + 16 + 8 + 6) + 2
ROOT2 = 2 + 16 + 6          # n = 1: the single leaf pair at the root
LEAF_CONSTANTS = 14 + 2     # a and s of the last vertex pair, once per point
PAIR_LOOKUP = 16            # two interpolations (g^<, g^>) per pair
POINT_EPILOGUE = 12         # prefactor, weight, compensated add


def tree_flops(n):
    """Per point inside the domain."""
    if n == 1:
        total = ROOT2
    else:
        total = 0
        for k in range(n - 2):           # blocks of size n+1-k >= 4
            total += (1 << k) * _node(n + 1 - k)
        total += (1 << (n - 2)) * NODE3
    return total + LEAF_CONSTANTS + PAIR_LOOKUP * n * (n + 1) // 2 + POINT_EPILOGUE


def _pair_node(m):
    """Paired-tree node holding an m x m trailing block, m >= 4: the two
    diagonal entries, then for both indices b of the earlier vertex the 2x2
    pivot block (entries, determinant, reciprocal, four scaled entries) and
    the vertex's row and column, and for both indices of the later vertex its
    row and column, the two scaled column vectors and the rank-2 update of
    the (m-2)^2 child block except its measurement diagonal (never read);
    det^2 times the signed child sum."""
    child = 4 * (m - 2) + 28 * (m - 2) + 16 * ((m - 2) ** 2 - 1) + 2
    per_b = 4 + 14 + 6 + 24 + 4 * (m - 2) + 2 * child + 12 + 2
    return 4 + 2 * per_b


def pair_tree_flops(n):
    """Per point inside the domain, paired tree (alpha != 0): pair nodes
    down to a 3x3 node (even n) or a leaf pair (odd n)."""
    total, m, count = 0, n + 1, 1
    while m >= 4:
        total += count * _pair_node(m)
        m -= 2
        count *= 4
    total += count * (NODE3 if m == 3 else ROOT2)
    return total + LEAF_CONSTANTS + PAIR_LOOKUP * n * (n + 1) // 2 + POINT_EPILOGUE


def warp_flops(n):
    """Per lattice point (lattice arithmetic, inverse CDF, weight; each
    transcendental counted as one operation)."""
    return 8 * n + 2


def geometry(n, alt=False):
    """Block size K, cooperative top levels, per-lane path levels T of the
    scalar tree's default lane mapping (a register tree of depth 5, depth 4
    at orders 5 and 6; the full matrix up to order 10, cooperative top
    levels above) or of its alternative (depth 5 at orders 5 and 6, depth 4
    at orders 7, 8 and 11-14, cooperative top levels at 9 and 10)."""
    if n in (5, 6):
        depth = 5 if alt else 4
    else:
        depth = 4 if alt and n not in (9, 10) else 5
    top_from = 8 if alt and n in (9, 10) else 10
    K = n + 1 if n <= top_from else 9
    off = n + 1 - K
    T = K - 1 - depth if K - 1 > depth else 0
    return K, off, T


def lane_flops(n, alt=False):
    """Operations the kernel issues per point inside the domain."""
    K, off, T = geometry(n, alt)
    path = 0
    for k in range(T):
        path += 2 + 8 * k + 6 + (K - 1 - k) * (10 + 16 * k) + 6
    ct = ((K - T) ** 2 - 1) * 8 * T
    sub = 0
    if K == 2:
        sub = ROOT2
    else:
        for lvl in range(T, K - 3):
            sub += (1 << (lvl - T)) * _node(K - lvl)
        sub += (1 << (K - 3 - T)) * NODE3
    per_lane = path + ct + sub + 12 + LEAF_CONSTANTS   # final prod^2 scaling
    per_item = (1 << T) * per_lane
    top = 0
    for k in range(off):
        rows = n - k
        top += 2 * (n + 1 - k) + rows * (2 + 6 + 6 + 8 * rows) + 6
    items = 1 << off
    return items * (per_item + top + PAIR_LOOKUP * n * (n + 1) // 2) + POINT_EPILOGUE
