/*
 * qqmc_tree.h -- per-lane arithmetic of the Keldysh sum (Eq. (integral_gf)).
 *
 * The sum S(u) = sum_a (-1)^{|a|} det_up(a) det_dn(a) runs over the 2^n
 * Keldysh index vectors a.  With the vertices ordered by time, earliest first,
 * and the measurement point last, the 2x2 Keldysh rule of App. E makes every
 * off-diagonal Wick entry depend only on the index of the EARLIER of its two
 * points (for u_k > u_l the first argument is later and
 * [[g^T, g^<],[g^>, g^Tbar]] collapses to g^> for a_l = 0 and g^< for
 * a_l = 1, whatever a_k).  Hence
 *   - eliminating the points in time order without pivoting, the pivot of
 *     step k and every Schur-complement correction carried past step k depend
 *     only on a_0..a_k, so the 2^n determinants share their elimination
 *     prefixes: a depth-first walk over a binary tree whose level-k node
 *     holds the trailing Schur complement after k steps does the work of all
 *     2^n factorisations with one rank-1 update per tree edge (about twelve
 *     complex multiply-adds per index vector instead of ~n^3);
 *   - the n x n spin-down block is the leading block of the (n+1) x (n+1)
 *     spin-up matrix, so det_dn is the product of the first n pivots and
 *     det_up = det_dn * (last pivot);
 *   - the last vertex's two indices differ only in the measurement pivot,
 *     which gives the pair of leaves in closed form (no reciprocal).
 * Off-diagonal entries: for points i earlier than j with tau = t_j - t_i > 0,
 *     entry (i, j) = a_i ? g^>(-tau) : g^<(-tau) = -conj(a_i ? g^> : g^<)(tau)
 *     entry (j, i) = a_i ? g^<(tau)  : g^>(tau);
 * diagonal entries are g^<(0) = i n_sigma.  The measurement point is the
 * latest point, so its own indices (0 as a row, 1 as a column) never enter.
 *
 * Work split across the lanes of one work item (G = 2^T lanes):
 *   block  K x K trailing block the lanes start from (K = n + 1 up to order
 *          10 -- the flat mapping -- and 9 above, with the first n - 8
 *          eliminations done cooperatively before; see Geo for the
 *          alternatives);
 *   path   T levels eliminated per lane, left-looking, for the lane's own
 *          index prefix (lane number within the item);
 *   tree   the remaining K - 1 - T <= 5 levels walked depth first with
 *          the Schur complements held in registers (the subtree of a lane
 *          starts from a block of at most 6 x 6).
 * Everything here is straight-line code for a compile-time order n.
 */
#ifndef QQMC_TREE_H
#define QQMC_TREE_H

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define QQMC_HD __host__ __device__ __forceinline__
#else
#include <cmath>
#define QQMC_HD inline
#endif

namespace qqmc {

struct cplx {
    double x, y;
};

QQMC_HD cplx cmk(double x, double y) { cplx r; r.x = x; r.y = y; return r; }
QQMC_HD cplx cadd(cplx a, cplx b) { return cmk(a.x + b.x, a.y + b.y); }
QQMC_HD cplx csub(cplx a, cplx b) { return cmk(a.x - b.x, a.y - b.y); }
QQMC_HD cplx cmul(cplx a, cplx b)
{
    return cmk(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
/* c + a*b */
QQMC_HD cplx cfma(cplx a, cplx b, cplx c)
{
    return cmk(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
/* c - a*b */
QQMC_HD cplx cfms(cplx a, cplx b, cplx c)
{
    return cmk(fma(-a.x, b.x, fma(a.y, b.y, c.x)), fma(-a.x, b.y, fma(-a.y, b.x, c.y)));
}
/* c + conj(a)*b */
QQMC_HD cplx cfmac(cplx a, cplx b, cplx c)
{
    return cmk(fma(a.x, b.x, fma(a.y, b.y, c.x)), fma(a.x, b.y, fma(-a.y, b.x, c.y)));
}
/* -conj(a) */
QQMC_HD cplx cnc(cplx a) { return cmk(-a.x, a.y); }
QQMC_HD cplx crecip(cplx a)
{
    double d = 1.0 / fma(a.x, a.x, a.y * a.y);
    return cmk(a.x * d, -a.y * d);
}
QQMC_HD cplx csel(int b, cplx one, cplx zero) { return b ? one : zero; }
QQMC_HD double cabs2(cplx a) { return fma(a.x, a.x, a.y * a.y); }
/* max(m, |Re a|, |Im a|): the largest component, within a factor sqrt(2) of
 * |a|, for two maximum instructions with absolute-value operands */
QQMC_HD double cmaxabs(double m, cplx a) { return fmax(m, fmax(fabs(a.x), fabs(a.y))); }

/* 1/a from the hardware reciprocal estimate refined by two Newton steps
 * (e = 1 - a r, r <- r + r e; each step squares the relative error), about
 * half the instructions of the IEEE division sequence.  Pivots here are
 * O(1) complex numbers, far from the denormal and overflow ranges that the
 * division sequence rescales for. */
QQMC_HD double rcp_nr(double a)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(a);
    double e = fma(-a, r, 1.0);
    r = fma(r, e, r);
    e = fma(-a, r, 1.0);
    return fma(r, e, r);
#else
    return 1.0 / a;
#endif
}
QQMC_HD cplx crecip_nr(cplx a)
{
    const double d = rcp_nr(fma(a.x, a.x, a.y * a.y));
    return cmk(a.x * d, -a.y * d);
}

/* g^<(tau), g^>(tau) for a pair of points, tau = later - earlier > 0 */
struct pairv {
    cplx gl, gg;
};

/* index of the pair (i, j), i < j, in the triangular pair table */
QQMC_HD constexpr int pidx(int i, int j) { return j * (j - 1) / 2 + i; }

/* Work split of one item.  PAIR selects the paired tree (vertices
 * eliminated two at a time with 2x2 block pivots, for vertex diagonals that
 * may vanish): its cooperative levels and per-lane path cover whole pairs.
 * MAP selects the lane mapping of the scalar tree: 0 the default (a
 * depth-5 register tree, depth 4 at orders 5 and 6, where it measured
 * faster); 1 a depth-4 register tree (twice the lanes per item, two waves
 * per SIMD); 3 a depth-5 register tree (the second mapping at orders 5 and
 * 6); 2 at orders 9 and 10 the first n - 8 levels eliminated cooperatively
 * by the lanes of each top-level index prefix (the default there is the
 * flat mapping, every lane walking its path from the full matrix). */
constexpr int kMapDefault = 0, kMapDepth4 = 1, kMapTop = 2, kMapDepth5 = 3;
template <int N, bool PAIR = false, int MAP = kMapDefault> struct Geo {
    static_assert(MAP == kMapDefault ||
                      (!PAIR && (MAP == kMapDepth4 || MAP == kMapDepth5 || (N == 9 || N == 10))),
                  "the scalar tree's second mappings: depth 4 or 5, or cooperative top levels at 9, 10");
    /* cooperative levels: the paired tree n - 8 rounded up to even above
     * order 8, the scalar tree n - 8 above order 10 (or above 8 with
     * kMapTop) */
    static constexpr int OFF = PAIR ? (N > 8 ? ((N - 7) & ~1) : 0)
                                    : (N > (MAP == kMapTop ? 8 : 10) ? N - 8 : 0);
    static constexpr int K = N + 1 - OFF;              /* block size          */
    /* register-tree depth */
    static constexpr int B =
        (MAP == kMapDepth4 || (MAP == kMapDefault && !PAIR && (N == 5 || N == 6))) ? 4 : 5;
    /* per-lane path: scalar tree, down to a 6 x 6 block; paired tree, whole
     * pairs down to a block of at most 5 x 5 (a pair node keeps its parent
     * block live under its four children) */
    static constexpr int T = PAIR ? (K > 5 ? 2 * ((K - 4) / 2) : 0)
                                  : ((K - 1 > B) ? K - 1 - B : 0);
    static constexpr int G = 1 << T;                   /* lanes per item      */
    static constexpr int PPW = 64 / G;                 /* items per wave      */
    static constexpr int IPP = 1 << OFF;               /* items per point     */
    static constexpr int NP = N * (N + 1) / 2;         /* pair-table length   */
    /* waves per SIMD the kernels are compiled for: a depth-5 register tree
     * starts from a 6 x 6 block and needs the whole register file of one
     * wave (architectural plus accumulation registers, no scratch); the
     * paired tree's per-lane path keeps four vectors per pair step, so it
     * takes the whole register file too */
    static constexpr int WPS = (PAIR || K - T > 5) ? 1 : 2;
};

template <int M> struct Blk {
    cplx v[M][M];
};

/* The last vertex's pair (n-1, measurement), the same for every leaf of a
 * point: with col_b / row_b the vertex's entries in the measurement column
 * and row, minus the block corrections C01 / C10,
 *   col_1 row_1 - col_0 row_0 = a + s C01 + t C10,
 *   s = row_0 - row_1,  t = col_0 - col_1.
 * The row entries are b ? g^< : g^> of the pair.  For the charge the column
 * entries are -conj(b ? g^> : g^<) of the same pair, so
 *   a = g^< (-conj g^>) - g^> (-conj g^<),  s = g^> - g^<,  t = conj(s);
 * for the current into a lead (CUR) they come from the lead's functions,
 * held as M = (-conj col_0, -conj col_1). */
struct LeafK {
    cplx a, s, t;
};
template <bool CUR = false> QQMC_HD LeafK leaf_constants(const pairv &P, const pairv &M)
{
    LeafK k;
    if constexpr (CUR) {
        k.a = cfms(P.gg, cnc(M.gl), cmul(P.gl, cnc(M.gg)));
        k.s = csub(P.gg, P.gl);
        k.t = csub(cnc(M.gl), cnc(M.gg));
    } else {
        (void)M;
        k.a = cfms(P.gg, cnc(P.gl), cmul(P.gl, cnc(P.gg)));
        k.s = csub(P.gg, P.gl);
        k.t = cmk(0.0, 0.0); /* conj(s), applied through cfmac */
    }
    return k;
}

/* y + t x: t = conj(s) for the charge */
template <bool CUR> QQMC_HD cplx add_col_coef(const LeafK &lk, cplx x, cplx y)
{
    if constexpr (CUR) return cfma(lk.t, x, y);
    else return cfmac(lk.s, x, y);
}

/* Closed form of the last two levels (latest vertex and the measurement)
 * for a trailing block with corrections C: the two leaves differ only in the
 * last pivot g0 - C11 - col_b row_b / p, so
 *   sum_b (-1)^b dn_b up_b / (pivots above)^2 = p (col_1 row_1 - col_0 row_0),
 * the bracket expanded with the point's leaf constants. */
template <bool CUR = false> QQMC_HD cplx leaf_value(const Blk<2> &C, cplx g0, const LeafK &lk)
{
    const cplx p = csub(g0, C.v[0][0]);
    return cmul(p, add_col_coef<CUR>(lk, C.v[1][0], cfma(lk.s, C.v[0][1], lk.a)));
}

/* Closed form of the last three levels: vertices u (global index v0), w (the
 * last one) and the measurement m (global index n), by cofactors instead of
 * elimination (no reciprocal): with S the 3x3 trailing matrix for index b of
 * u,
 *   sum_{b_w} (-1)^{b_w} det S = S_uu d + S_uw S_mu t + S_um S_wu s
 * (the S_mm terms cancel, d as in the leaf with this node's C12, C21),
 * multiplied by the 2x2 vertex determinant S_uu S_ww - S_uw S_wu.  mc holds
 * the measurement-column entries of the current (unused for the charge). */
template <bool CUR = false>
QQMC_HD cplx node3_value(const Blk<3> &C, const pairv *pr, const pairv *mc, int v0, int n,
                         cplx g0, const LeafK &lk)
{
    const cplx p = csub(g0, C.v[0][0]);
    const pairv Pw = pr[pidx(v0, v0 + 1)];
    const pairv Pm = pr[pidx(v0, n)];
    pairv Mu;
    if constexpr (CUR) Mu = mc[v0];
    else { (void)mc; Mu = Pm; }
    const cplx sww = csub(g0, C.v[1][1]);
    const cplx spp = cmul(p, sww);
    const cplx sd = cmul(p, add_col_coef<CUR>(lk, C.v[2][1], cfma(lk.s, C.v[1][2], lk.a)));
    cplx t[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const cplx suw = csub(cnc(b ? Pw.gg : Pw.gl), C.v[0][1]);
        const cplx swu = csub(b ? Pw.gl : Pw.gg, C.v[1][0]);
        const cplx sum_ = csub(cnc(b ? Mu.gg : Mu.gl), C.v[0][2]);
        const cplx smu = csub(b ? Pm.gl : Pm.gg, C.v[2][0]);
        const cplx delta = cfma(cmul(sum_, swu), lk.s, add_col_coef<CUR>(lk, cmul(suw, smu), sd));
        t[b] = cmul(cfms(suw, swu, spp), delta);
    }
    return csub(t[0], t[1]);
}

/* Depth-first walk below block level L (block indices L..K-1 remain).  C is
 * the accumulated Schur correction of the trailing block, so the current
 * trailing matrix is (Wick entries) - C.  Returns the signed sum over the
 * node's leaves relative to the node: a leaf pair's term carries the square
 * of every pivot above it, so with p this node's pivot
 *     V(node) = p^2 (V(child 0) - V(child 1))
 * and the caller multiplies by the square of the pivots above the node.  A
 * node builds the correction blocks of BOTH children (indices 0 and 1 of the
 * level's point) before descending, so while the first child's subtree runs
 * only the second child's (m-1) x (m-1) block is held, not the m x m parent. */
template <int N, int L, bool CUR = false, int MAP = kMapDefault>
QQMC_HD cplx subtree(const Blk<Geo<N, false, MAP>::K - L> &C, const pairv *pr, const pairv *mc,
                     cplx g0, const LeafK &lk)
{
    constexpr int K = Geo<N, false, MAP>::K, OFF = Geo<N, false, MAP>::OFF, M = K - L;
    if constexpr (M == 2) {
        (void)pr;
        (void)mc;
        return leaf_value<CUR>(C, g0, lk);
    } else if constexpr (M == 3) {
        return node3_value<CUR>(C, pr, mc, OFF + L, N, g0, lk);
    } else {
        const cplx p = csub(g0, C.v[0][0]);
        const cplx r = crecip_nr(p);
        Blk<M - 1> D0, D1;
        {
            /* pair (L, L+i) holds (g^<, g^>): index 0 takes column g^> and row
             * -conj(g^<), index 1 column g^< and row -conj(g^>) */
            cplx row0[M - 1], row1[M - 1];
#pragma unroll
            for (int j = 1; j < M; ++j) {
                /* the current's measurement column comes from mc */
                const pairv P = (CUR && j == M - 1) ? mc[OFF + L] : pr[pidx(OFF + L, OFF + L + j)];
                row0[j - 1] = csub(cnc(P.gl), C.v[0][j]);
                row1[j - 1] = csub(cnc(P.gg), C.v[0][j]);
            }
#pragma unroll
            for (int i = 1; i < M; ++i) {
                const pairv P = pr[pidx(OFF + L, OFF + L + i)];
                const cplx c0 = cmul(csub(P.gg, C.v[i][0]), r);
                const cplx c1 = cmul(csub(P.gl, C.v[i][0]), r);
#pragma unroll
                for (int j = 1; j < M; ++j) {
                    D0.v[i - 1][j - 1] = cfma(c0, row0[j - 1], C.v[i][j]);
                    D1.v[i - 1][j - 1] = cfma(c1, row1[j - 1], C.v[i][j]);
                }
            }
        }
        const cplx v0 = subtree<N, L + 1, CUR, MAP>(D0, pr, mc, g0, lk);
        const cplx v1 = subtree<N, L + 1, CUR, MAP>(D1, pr, mc, g0, lk);
        return cmul(cmul(p, p), csub(v0, v1));
    }
}

/* Block correction accessor: zero when the lanes start from the full matrix
 * (n <= 8), otherwise the cooperative block in local memory. */
template <int N, bool PAIR = false, int MAP = kMapDefault> struct BlockSrc {
    const cplx *c; /* K*K row-major, or unused */
    QQMC_HD cplx at(int i, int j) const
    {
        if constexpr (Geo<N, PAIR, MAP>::OFF == 0) {
            (void)i; (void)j;
            return cmk(0.0, 0.0);
        } else {
            return c[i * Geo<N, PAIR, MAP>::K + j];
        }
    }
};

/* One lane's share of an item: index prefix `pre` (T bits, most significant
 * bit = earliest block level), starting block correction C0, product of the
 * pivots eliminated before the block, parity of the indices fixed before.
 * Returns the signed sum over the lane's 2^B index vectors. */
template <int N, bool CUR = false, int MAP = kMapDefault>
QQMC_HD cplx lane_sum(const pairv *pr, const pairv *mc, BlockSrc<N, false, MAP> C0, int pre,
                      cplx prod, int sgn, cplx g0)
{
    using Gm = Geo<N, false, MAP>;
    constexpr int K = Gm::K, OFF = Gm::OFF, T = Gm::T;
    const LeafK lk = leaf_constants<CUR>(pr[pidx(N - 1, N)], mc[N - 1]);
    cplx v;
    if constexpr (T == 0) {
        (void)pre;
        Blk<K> C;
#pragma unroll
        for (int i = 0; i < K; ++i)
#pragma unroll
            for (int j = 0; j < K; ++j) C.v[i][j] = C0.at(i, j);
        v = subtree<N, 0, CUR, MAP>(C, pr, mc, g0, lk);
    } else {
        cplx chat[T][K], rowv[T][K];
#pragma unroll
        for (int k = 0; k < T; ++k) {
            const int b = (pre >> (T - 1 - k)) & 1;
            sgn ^= b;
            cplx pk = csub(g0, C0.at(k, k));
#pragma unroll
            for (int l = 0; l < k; ++l) pk = cfms(chat[l][k], rowv[l][k], pk);
            const cplx r = crecip_nr(pk);
#pragma unroll
            for (int i = k + 1; i < K; ++i) {
                /* the index picks the table half by address: index 1 takes
                 * column g^< and row -conj(g^>), index 0 the other halves */
                const cplx *P = &pr[pidx(OFF + k, OFF + i)].gl;
                const cplx *R = (CUR && i == K - 1) ? &mc[OFF + k].gl : P;
                cplx col = csub(P[b ^ 1], C0.at(i, k));
                cplx row = csub(cnc(R[b]), C0.at(k, i));
#pragma unroll
                for (int l = 0; l < k; ++l) {
                    col = cfms(chat[l][i], rowv[l][k], col);
                    row = cfms(chat[l][k], rowv[l][i], row);
                }
                chat[k][i] = cmul(col, r);
                rowv[k][i] = row;
            }
            prod = cmul(prod, pk);
        }
        Blk<K - T> C;
#pragma unroll
        for (int i = T; i < K; ++i)
#pragma unroll
            for (int j = T; j < K; ++j) {
                cplx c = C0.at(i, j);
#pragma unroll
                for (int l = 0; l < T; ++l) c = cfma(chat[l][i], rowv[l][j], c);
                C.v[i - T][j - T] = c;
            }
        v = subtree<N, T, CUR, MAP>(C, pr, mc, g0, lk);
    }
    v = cmul(cmul(prod, prod), v);
    return sgn ? cmk(-v.x, -v.y) : v;
}

/* Paired tree: a node at block level L eliminates the vertices v = OFF + L
 * and w = v + 1 together.  With the trailing matrix T = (Wick entries) - C,
 * the 2x2 pivot block P_b = [[T_vv, T_vw], [T_wv, T_ww]] depends only on the
 * index b of v (the earlier point of the pair), the rows and columns of v on
 * b and those of w on the index b' of w; with u, x the column and row of v
 * and y, z those of w, the child (b, b') carries
 *     C' = C + U x + V y,  [U V] = [u z] P_b^{-1},
 * and the node's value relative to itself is
 *     V(node) = det(P_0)^2 (V_00 - V_01) - det(P_1)^2 (V_10 - V_11).
 * No scalar pivot of a single vertex is inverted: a zero vertex diagonal
 * (alpha = n_sigma) and the skew-symmetric blocks of the particle-hole
 * symmetric point are handled exactly.  The last one or two vertices end in
 * the closed forms above, which invert nothing either. */
template <int N, int L, bool CUR = false>
QQMC_HD cplx pair_walk(const Blk<Geo<N, true>::K - L> &C, const pairv *pr, const pairv *mc,
                       cplx g0, const LeafK &lk, double &grow)
{
    constexpr int K = Geo<N, true>::K, OFF = Geo<N, true>::OFF, M = K - L;
    if constexpr (M == 2) {
        (void)pr;
        (void)mc;
        return leaf_value<CUR>(C, g0, lk);
    } else if constexpr (M == 3) {
        return node3_value<CUR>(C, pr, mc, OFF + L, N, g0, lk);
    } else {
        constexpr int V0 = OFF + L;
        const cplx a = csub(g0, C.v[0][0]), d = csub(g0, C.v[1][1]);
        const cplx *Pvw = &pr[pidx(V0, V0 + 1)].gl;
        cplx res = cmk(0.0, 0.0);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            /* the table half is picked by address: index 1 takes column g^<
             * and row -conj(g^>), index 0 the other halves */
            const cplx be = csub(cnc(Pvw[b]), C.v[0][1]);
            const cplx ga = csub(Pvw[b ^ 1], C.v[1][0]);
            const cplx det = cfms(be, ga, cmul(a, d));
            const cplx r = crecip_nr(det);
            const cplx dd = cmul(d, r), aa = cmul(a, r), bb = cmul(be, r), gg = cmul(ga, r);
            cplx x[M - 2], u[M - 2];
#pragma unroll
            for (int j = 2; j < M; ++j) {
                const cplx *P = &pr[pidx(V0, V0 + j)].gl;
                const cplx *R = (CUR && j == M - 1) ? &mc[V0].gl : P;
                x[j - 2] = csub(cnc(R[b]), C.v[0][j]);
                u[j - 2] = csub(P[b ^ 1], C.v[j][0]);
            }
            cplx sub = cmk(0.0, 0.0);
#pragma unroll
            for (int bq = 0; bq < 2; ++bq) {
                cplx y[M - 2], z[M - 2];
#pragma unroll
                for (int j = 2; j < M; ++j) {
                    const cplx *Q = &pr[pidx(V0 + 1, V0 + j)].gl;
                    const cplx *R = (CUR && j == M - 1) ? &mc[V0 + 1].gl : Q;
                    y[j - 2] = csub(cnc(R[bq]), C.v[1][j]);
                    z[j - 2] = csub(Q[bq ^ 1], C.v[j][1]);
                }
                Blk<M - 2> D;
#pragma unroll
                for (int i = 2; i < M; ++i) {
                    const cplx Ui = cfms(z[i - 2], gg, cmul(u[i - 2], dd));
                    const cplx Vi = cfms(u[i - 2], bb, cmul(z[i - 2], aa));
                    grow = cmaxabs(cmaxabs(grow, Ui), Vi);
#pragma unroll
                    for (int j = 2; j < M; ++j)
                        D.v[i - 2][j - 2] = cfma(Vi, y[j - 2], cfma(Ui, x[j - 2], C.v[i][j]));
                }
                const cplx w = pair_walk<N, L + 2, CUR>(D, pr, mc, g0, lk, grow);
                sub = bq ? csub(sub, w) : cadd(sub, w);
            }
            const cplx t = cmul(cmul(det, det), sub);
            res = b ? csub(res, t) : cadd(res, t);
        }
        return res;
    }
}

/* One lane's share of an item in the paired tree: the T prefix levels are
 * T/2 pair steps for the lane's index bits (left-looking: each step keeps
 * its U, V columns and x, y rows), then the pair walk. */
template <int N, bool CUR = false>
QQMC_HD cplx lane_sum_pair(const pairv *pr, const pairv *mc, BlockSrc<N, true> C0, int pre,
                           cplx prod, int sgn, cplx g0, double &grow)
{
    constexpr int K = Geo<N, true>::K, OFF = Geo<N, true>::OFF, T = Geo<N, true>::T;
    const LeafK lk = leaf_constants<CUR>(pr[pidx(N - 1, N)], mc[N - 1]);
    cplx v;
    if constexpr (T == 0) {
        (void)pre;
        Blk<K> C;
#pragma unroll
        for (int i = 0; i < K; ++i)
#pragma unroll
            for (int j = 0; j < K; ++j) C.v[i][j] = C0.at(i, j);
        v = pair_walk<N, 0, CUR>(C, pr, mc, g0, lk, grow);
    } else {
        constexpr int TP = T / 2;
        cplx Uc[TP][K], Vc[TP][K], xr[TP][K], yr[TP][K];
#pragma unroll
        for (int s = 0; s < TP; ++s) {
            const int k = 2 * s;
            const int b = (pre >> (T - 1 - k)) & 1, bq = (pre >> (T - 2 - k)) & 1;
            sgn ^= b ^ bq;
            const cplx *Pvw = &pr[pidx(OFF + k, OFF + k + 1)].gl;
            cplx a = csub(g0, C0.at(k, k)), d = csub(g0, C0.at(k + 1, k + 1));
            cplx be = csub(cnc(Pvw[b]), C0.at(k, k + 1));
            cplx ga = csub(Pvw[b ^ 1], C0.at(k + 1, k));
#pragma unroll
            for (int l = 0; l < s; ++l) {
                a = cfms(Vc[l][k], yr[l][k], cfms(Uc[l][k], xr[l][k], a));
                d = cfms(Vc[l][k + 1], yr[l][k + 1], cfms(Uc[l][k + 1], xr[l][k + 1], d));
                be = cfms(Vc[l][k], yr[l][k + 1], cfms(Uc[l][k], xr[l][k + 1], be));
                ga = cfms(Vc[l][k + 1], yr[l][k], cfms(Uc[l][k + 1], xr[l][k], ga));
            }
            const cplx det = cfms(be, ga, cmul(a, d));
            const cplx r = crecip_nr(det);
            const cplx dd = cmul(d, r), aa = cmul(a, r), bb = cmul(be, r), gg = cmul(ga, r);
#pragma unroll
            for (int i = k + 2; i < K; ++i) {
                const cplx *P = &pr[pidx(OFF + k, OFF + i)].gl;
                const cplx *Q = &pr[pidx(OFF + k + 1, OFF + i)].gl;
                const cplx *RP = (CUR && i == K - 1) ? &mc[OFF + k].gl : P;
                const cplx *RQ = (CUR && i == K - 1) ? &mc[OFF + k + 1].gl : Q;
                cplx x = csub(cnc(RP[b]), C0.at(k, i)), u = csub(P[b ^ 1], C0.at(i, k));
                cplx y = csub(cnc(RQ[bq]), C0.at(k + 1, i)), z = csub(Q[bq ^ 1], C0.at(i, k + 1));
#pragma unroll
                for (int l = 0; l < s; ++l) {
                    x = cfms(Vc[l][k], yr[l][i], cfms(Uc[l][k], xr[l][i], x));
                    u = cfms(Vc[l][i], yr[l][k], cfms(Uc[l][i], xr[l][k], u));
                    y = cfms(Vc[l][k + 1], yr[l][i], cfms(Uc[l][k + 1], xr[l][i], y));
                    z = cfms(Vc[l][i], yr[l][k + 1], cfms(Uc[l][i], xr[l][k + 1], z));
                }
                xr[s][i] = x;
                yr[s][i] = y;
                Uc[s][i] = cfms(z, gg, cmul(u, dd));
                Vc[s][i] = cfms(u, bb, cmul(z, aa));
                grow = cmaxabs(cmaxabs(grow, Uc[s][i]), Vc[s][i]);
            }
            prod = cmul(prod, det);
        }
        Blk<K - T> C;
#pragma unroll
        for (int i = T; i < K; ++i)
#pragma unroll
            for (int j = T; j < K; ++j) {
                cplx c = C0.at(i, j);
#pragma unroll
                for (int l = 0; l < TP; ++l) c = cfma(Vc[l][i], yr[l][j], cfma(Uc[l][i], xr[l][j], c));
                C.v[i - T][j - T] = c;
            }
        v = pair_walk<N, T, CUR>(C, pr, mc, g0, lk, grow);
    }
    v = cmul(cmul(prod, prod), v);
    return sgn ? cmk(-v.x, -v.y) : v;
}

/* The shifted grouping of the paired tree.  The lane's 3-bit index prefix
 * covers two left-looking steps of sizes S0 and S1 (a pair and a single
 * vertex: 2 then 1 from the whole matrix, 1 then 2 from a cooperative top's
 * block), then the paired walk continues from block vertex 3.  Against the
 * even grouping (0,1), (2,3), ... every later pair boundary moves by one
 * vertex, so a long time gap that falls inside an even pair (the case that
 * makes its pivot block nearly singular) falls between two pairs here.  With
 * C the correction after a step, the trailing entries are (Wick) - C; a
 * single step adds c row with c = col / p, a pair step U x + V y.  Returns
 * the lane's signed sum and accumulates the largest elimination multiplier
 * as the paired tree does. */
template <int N, bool CUR, int S0, int S1>
QQMC_HD cplx lane_sum_shift(const pairv *pr, const pairv *mc, BlockSrc<N, true> C0, int pre,
                            cplx prod, int sgn, cplx g0, double &grow)
{
    static_assert(S0 + S1 == 3 && (S0 == 1 || S0 == 2), "a pair and a single vertex");
    constexpr int K = Geo<N, true>::K, OFF = Geo<N, true>::OFF;
    static_assert(K >= 5, "the walk needs the measurement and one vertex");
    constexpr int SP = S0 == 2 ? 0 : 1;   /* block index of the pair's first vertex */
    constexpr int SS = S0 == 2 ? 2 : 0;   /* block index of the single vertex        */
    const LeafK lk = leaf_constants<CUR>(pr[pidx(N - 1, N)], mc[N - 1]);
    const int bits[3] = {(pre >> 2) & 1, (pre >> 1) & 1, pre & 1};
    sgn ^= bits[0] ^ bits[1] ^ bits[2];
    const int bp = bits[SP], bq = bits[SP + 1], bs = bits[SS];
    /* table halves by address: row entries -conj(b ? g^> : g^<) (the lead's
     * for the current's measurement column), column entries b ? g^< : g^> */
    auto rowp = [&](int k, int j) -> const cplx * {
        return (CUR && j == K - 1) ? &mc[OFF + k].gl : &pr[pidx(OFF + k, OFF + j)].gl;
    };
    auto colp = [&](int k, int i) -> const cplx * { return &pr[pidx(OFF + k, OFF + i)].gl; };
    cplx U[K], V[K], X[K], Y[K], Cc[K], Rr[K];
    /* correction of block entry (i, j) after the steps taken so far */
    bool pair_done = false, single_done = false;
    auto corr = [&](int i, int j) -> cplx {
        cplx c = C0.at(i, j);
        if (pair_done) c = cfma(V[i], Y[j], cfma(U[i], X[j], c));
        if (single_done) c = cfma(Cc[i], Rr[j], c);
        return c;
    };
#pragma unroll
    for (int step = 0; step < 2; ++step) {
        const bool is_pair = (step == 0) == (S0 == 2);
        if (is_pair) {
            constexpr int k = SP;
            const cplx a = csub(g0, corr(k, k)), d = csub(g0, corr(k + 1, k + 1));
            const cplx be = csub(cnc(colp(k, k + 1)[bp]), corr(k, k + 1));
            const cplx ga = csub(colp(k, k + 1)[bp ^ 1], corr(k + 1, k));
            const cplx det = cfms(be, ga, cmul(a, d));
            const cplx r = crecip_nr(det);
            const cplx dd = cmul(d, r), aa = cmul(a, r), bb = cmul(be, r), gg = cmul(ga, r);
#pragma unroll
            for (int i = k + 2; i < K; ++i) {
                const cplx x = csub(cnc(rowp(k, i)[bp]), corr(k, i));
                const cplx u = csub(colp(k, i)[bp ^ 1], corr(i, k));
                const cplx y = csub(cnc(rowp(k + 1, i)[bq]), corr(k + 1, i));
                const cplx z = csub(colp(k + 1, i)[bq ^ 1], corr(i, k + 1));
                X[i] = x;
                Y[i] = y;
                U[i] = cfms(z, gg, cmul(u, dd));
                V[i] = cfms(u, bb, cmul(z, aa));
                grow = cmaxabs(cmaxabs(grow, U[i]), V[i]);
            }
            prod = cmul(prod, det);
            pair_done = true;
        } else {
            constexpr int k = SS;
            const cplx p = csub(g0, corr(k, k));
            const cplx rp = crecip_nr(p);
#pragma unroll
            for (int i = k + 1; i < K; ++i) {
                const cplx col = csub(colp(k, i)[bs ^ 1], corr(i, k));
                const cplx row = csub(cnc(rowp(k, i)[bs]), corr(k, i));
                Cc[i] = cmul(col, rp);
                Rr[i] = row;
                grow = cmaxabs(grow, Cc[i]);
            }
            prod = cmul(prod, p);
            single_done = true;
        }
    }
    Blk<K - 3> C;
#pragma unroll
    for (int i = 3; i < K; ++i)
#pragma unroll
        for (int j = 3; j < K; ++j) C.v[i - 3][j - 3] = corr(i, j);
    cplx v = pair_walk<N, 3, CUR>(C, pr, mc, g0, lk, grow);
    v = cmul(cmul(prod, prod), v);
    return sgn ? cmk(-v.x, -v.y) : v;
}

/* Wick entry (i, j), i != j, of global elimination indices for index b of
 * the earlier point min(i, j); the index picks the table half by address
 * (upper entries -conj(b ? g^> : g^<), lower entries b ? g^< : g^>). */
QQMC_HD cplx wick_entry(const pairv *pr, int i, int j, int b)
{
    if (i < j) return cnc((&pr[pidx(i, j)].gl)[b]);
    return (&pr[pidx(j, i)].gl)[b ^ 1];
}

/* The same with the current's measurement column (column n) from mc. */
template <bool CUR>
QQMC_HD cplx wick_entry_m(const pairv *pr, const pairv *mc, int i, int j, int n, int b)
{
    if (CUR && i < j && j == n) return cnc((&mc[i].gl)[b]);
    (void)mc;
    (void)n;
    return wick_entry(pr, i, j, b);
}

/* Linear interpolation on the uniform grid tau_j = -t_half + j h, given
 * inv_h = 1/h (index and fraction clamped, so values outside the grid hold
 * the end values).  The table stores (g^<, g^>) per node as four doubles. */
QQMC_HD pairv interp_pair(const double *tab, int n_grid, double t_half, double inv_h,
                          double tau)
{
    const double s = (tau + t_half) * inv_h;
    long j = (long)floor(s);
    if (j < 0) j = 0;
    if (j > n_grid - 2) j = n_grid - 2;
    double phi = s - (double)j;
    if (phi < 0.0) phi = 0.0;
    if (phi > 1.0) phi = 1.0;
    const double q = 1.0 - phi;
    const double *a = tab + 4 * j;
    pairv r;
    r.gl = cmk(q * a[0] + phi * a[4], q * a[1] + phi * a[5]);
    r.gg = cmk(q * a[2] + phi * a[6], q * a[3] + phi * a[7]);
    return r;
}

} // namespace qqmc
#endif
