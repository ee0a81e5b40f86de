/*
 * qqmc_adapt.h -- adaptive block elimination of one point by a whole wave:
 * the accurate path behind the paired elimination tree.
 *
 * Why it exists.  With the vertex diagonal i (n_sigma - alpha) at or near
 * zero (the paper's alpha = n_sigma, App. E), the paired tree eliminates the
 * time-ordered vertices two at a time, (0,1), (2,3), ...  When a pair
 * straddles a long time gap, its 2x2 pivot block couples a vertex that
 * still sees the earlier vertices to one that is nearly decoupled from them:
 * the block is tiny against the entries it divides, the Schur complement
 * grows by orders of magnitude, and the cancellation that follows loses up
 * to eight digits of the term mass.  Which grouping is safe depends on the
 * point (where its gaps are) and on the Green's functions (how fast they
 * decay), so no fixed grouping works for every point.
 *
 * The register tree therefore tracks the largest elimination multiplier of
 * its pair steps (C' = C + U x + V y, qqmc_tree.h); a point with a large one
 * is evaluated again, first by the shifted grouping of the register tree
 * (lane_sum_shift), and where that grows too, here.  This path keeps the time order (so that the Schur corrections of a node depend
 * only on the indices fixed above it, the property the tree rests on) but
 * chooses the size of every elimination block from the data:
 *   - a single vertex (pivot p = g0 - C_kk, children b = 0, 1) when its
 *     growth bound max|col/p| max|row| stays below kGrowthSingle at every
 *     node of the level,
 *   - otherwise a 2x2 block (k, k+1) if its bound is smaller (children
 *     (b, b'), as in the paired tree).
 * Any grouping is an exact block factorisation of the same matrices; each
 * path from the root to a leaf is one elimination, so nodes processed
 * together only need to agree on the grouping among themselves.
 *
 * Work split.  The whole wave works on one point.  Blocks larger than MB x MB
 * (the top levels) are walked depth first: every top path is replayed from
 * the start block (two block buffers instead of a stack), the decision at
 * each top node recomputed from its data.  From a block of at most MB x MB
 * the levels are expanded breadth first in local memory, every entry of a
 * level spread over the lanes, and the last one or two vertices with the
 * measurement end in the division-free closed forms of qqmc_tree.h.
 * Decisions come from maxima that every lane reads from local memory, so they
 * are the same in every lane; sums are taken in a fixed order, so results
 * are reproducible.
 *
 * The same code runs on the host (lanes in a loop) for testing.
 */
#ifndef QQMC_ADAPT_H
#define QQMC_ADAPT_H

#include "qqmc_tree.h"

namespace qqmc {

/* A point of the paired register tree one of whose elimination multipliers
 * (U, V of a pair step; largest component) exceeds kGrowthFlag is evaluated
 * again with the shifted grouping, and if one of that tree's multipliers
 * exceeds kShiftFlag, by the adaptive path.  Set from CPU scans against a
 * quad-precision Keldysh sum (alpha = n_sigma; orders 6-8 on five dots,
 * among them the paper's finite-bandwidth dot at t = 100, 1500 points each):
 * with 128, 2-8% of points are evaluated again and every point the register
 * tree keeps is within 3.5e-14 of its term mass (64: 5-14% evaluated again,
 * 2.4e-14; 256: up to 1.5e-13); 0-0.13% reach the adaptive path.  (Tracking
 * the multipliers alone costs two maximum instructions per value; a bound on
 * the correction's growth, |U| |x| + |V| |y|, flagged slightly fewer points
 * but made the register tree 12-25% slower.) */
constexpr double kGrowthFlag = 128.0;
constexpr double kShiftFlag = 256.0;
/* The adaptive path takes a single-vertex step when its growth bound stays
 * below this at every node of the level. */
constexpr double kGrowthSingle = 4.0;

/* Entry of a correction block, a null block being zero. */
QQMC_HD cplx cld(const cplx *C, int idx) { return C ? C[idx] : cmk(0.0, 0.0); }

/* Local-memory workspace (complex entries) of the adaptive path for order N
 * with breadth-first start blocks of at most MB x MB (4 <= MB <= 8): a level
 * of m x m blocks holds 2^(MB-m) of them. */
template <int N, int MB> struct AdaptWs {
    static_assert(MB >= 4 && MB <= 8, "breadth-first start blocks of 4x4 .. 8x8");
    static constexpr int M0 = N + 1;
    /* replay buffers (two), when the whole point exceeds MB x MB */
    static constexpr int RB = M0 > MB ? M0 * M0 : 0;
    /* a stored level of m x m blocks (m >= 4) holds 2^(MB-m) of them: at
     * most 16 * 2^(MB-4) entries, at m = 4 */
    static constexpr int NODES = 1 << (MB - 4);
    static constexpr int LVL = 16 * NODES;
    /* single-step vectors of a stored step, 4 (m-1) per node, largest at
     * m = 5; a top step needs 2 (m-1) <= 2 N */
    static constexpr int VS0 = MB >= 5 ? (16 << (MB - 5)) : 0;
    static constexpr int VS = VS0 > 2 * N ? VS0 : 2 * N;
    /* pair-step vectors of a stored step, 12 (m-2) per node, largest at
     * m = 6; a top step needs 4 (m-2) <= 4 N */
    static constexpr int VP0 = MB >= 6 ? (48 << (MB - 6)) : 0;
    static constexpr int VP = VP0 > 4 * N ? VP0 : 4 * N;
    static constexpr int rep = 0;
    static constexpr int lvl = rep + 2 * RB;
    static constexpr int vs = lvl + 2 * LVL;
    static constexpr int vp = vs + VS;
    static constexpr int wsn = vp + VP;          /* 64 child weights (single) */
    static constexpr int wpn = wsn + 64;         /* 64 child weights (pair)   */
    static constexpr int nw = wpn + 64;          /* node weights of a level   */
    static constexpr int part = nw + NODES;      /* per-lane partial sums     */
    static constexpr int red = part + 64;        /* 64 doubles                */
    static constexpr int cplx_count = red + 32;
    static constexpr int bytes = cplx_count * 16;
};

/* Lanes of the wave.  On the device every lane runs the body once, then the
 * wave passes an ordering point (one 64-lane wave per workgroup: local
 * memory operations of a wave execute in program order); on the host the
 * body runs for every lane in turn. */
struct WaveLanes {
#if defined(__HIP_DEVICE_COMPILE__)
    template <class F> __device__ __forceinline__ void par(F f)
    {
        f((int)threadIdx.x);
        asm volatile("" ::: "memory");
    }
#else
    template <class F> void par(F f)
    {
        for (int l = 0; l < 64; ++l) f(l);
    }
#endif
};

/* Single-step quantities of a node (block C, m x m, null = zero; first row
 * the global vertex k) for index b: the pivot p, the scaled column col/p
 * and the row (m-1 each, when colp is not null).  Returns the squared growth
 * bound max|col|^2 max|row|^2 / |p|^2. */
template <bool CUR>
QQMC_HD double single_vectors(const cplx *C, int m, int k, int n, int b, const pairv *pr,
                              const pairv *mc, cplx g0, cplx &p, cplx *colp, cplx *row)
{
    p = csub(g0, cld(C, 0));
    const double p2 = cabs2(p);
    const cplx rp = p2 > 0.0 ? crecip(p) : cmk(0.0, 0.0);
    double mc2 = 0.0, mr2 = 0.0;
    for (int i = 1; i < m; ++i) {
        const cplx c = csub(wick_entry(pr, k + i, k, b), cld(C, i * m));
        const cplx r = csub(wick_entry_m<CUR>(pr, mc, k, k + i, n, b), cld(C, i));
        mc2 = fmax(mc2, cabs2(c));
        mr2 = fmax(mr2, cabs2(r));
        if (colp) {
            colp[i - 1] = cmul(c, rp);
            row[i - 1] = r;
        }
    }
    if (!(p2 > 0.0)) return INFINITY;
    const double g = mc2 * mr2 / p2;
    return g == g ? g : INFINITY;
}

/* Pair-step quantities of a node for indices (b, bq): the pivot-block
 * determinant, U, V (columns, m-2 each) and the rows x (vertex k, index b)
 * and y (vertex k+1, index bq), when U is not null.  Returns the squared
 * growth bound 4 max(|U|^2 |x|^2, |V|^2 |y|^2). */
template <bool CUR>
QQMC_HD double pair_vectors(const cplx *C, int m, int k, int n, int b, int bq, const pairv *pr,
                            const pairv *mc, cplx g0, cplx &det, cplx *U, cplx *V, cplx *x,
                            cplx *y)
{
    const cplx a = csub(g0, cld(C, 0)), d = csub(g0, cld(C, m + 1));
    const cplx be = csub(wick_entry(pr, k, k + 1, b), cld(C, 1));
    const cplx ga = csub(wick_entry(pr, k + 1, k, b), cld(C, m));
    det = cfms(be, ga, cmul(a, d));
    const bool ok = cabs2(det) > 0.0;
    const cplx r = ok ? crecip(det) : cmk(0.0, 0.0);
    const cplx dd = cmul(d, r), aa = cmul(a, r), bb = cmul(be, r), gg = cmul(ga, r);
    double mU = 0.0, mV = 0.0, mX = 0.0, mY = 0.0;
    for (int i = 2; i < m; ++i) {
        const cplx u = csub(wick_entry(pr, k + i, k, b), cld(C, i * m));
        const cplx z = csub(wick_entry(pr, k + i, k + 1, bq), cld(C, i * m + 1));
        const cplx Ui = cfms(z, gg, cmul(u, dd));
        const cplx Vi = cfms(u, bb, cmul(z, aa));
        const cplx xi = csub(wick_entry_m<CUR>(pr, mc, k, k + i, n, b), cld(C, i));
        const cplx yi = csub(wick_entry_m<CUR>(pr, mc, k + 1, k + i, n, bq), cld(C, m + i));
        mU = fmax(mU, cabs2(Ui));
        mV = fmax(mV, cabs2(Vi));
        mX = fmax(mX, cabs2(xi));
        mY = fmax(mY, cabs2(yi));
        if (U) {
            U[i - 2] = Ui;
            V[i - 2] = Vi;
            x[i - 2] = xi;
            y[i - 2] = yi;
        }
    }
    if (!ok) return INFINITY;
    const double g = 4.0 * fmax(mU * mX, mV * mY);
    return g == g ? g : INFINITY;
}

/* Weight of a child: the parent's times p^2 (det^2), negated for an odd
 * index sum. */
QQMC_HD cplx child_weight(cplx w, cplx piv, int odd)
{
    const cplx v = cmul(w, cmul(piv, piv));
    return odd ? cmk(-v.x, -v.y) : v;
}

/* Value of a tail node relative to the node: m = 2, the last vertex and the
 * measurement; m = 3, the last two vertices and the measurement. */
template <bool CUR>
QQMC_HD cplx tail_value(const cplx *C, int m, int n, const pairv *pr, const pairv *mc, cplx g0,
                        const LeafK &lk)
{
    if (m == 2) {
        Blk<2> B;
        B.v[0][0] = cld(C, 0); B.v[0][1] = cld(C, 1);
        B.v[1][0] = cld(C, 2); B.v[1][1] = cld(C, 3);
        return leaf_value<CUR>(B, g0, lk);
    }
    Blk<3> B;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B.v[i][j] = cld(C, i * 3 + j);
    return node3_value<CUR>(B, pr, mc, n - 2, n, g0, lk);
}

/* Everything the adaptive path reads and writes. */
template <bool CUR> struct AdaptCtx {
    const pairv *pr, *mc;
    cplx g0;
    LeafK lk;
    int n;
    cplx *lvl, *vs, *vp, *wsn, *wpn, *nw, *part, *rep;
    double *red;
    int lvl_size;   /* complex entries per level buffer */
    int rep_size;   /* complex entries per replay buffer */
};

/* Value, relative to itself, of the child (index b, or (b, bq) for a pair
 * step) of an M x M node (block Pn, first row global vertex k) that ends in
 * a closed form: the child block is built in registers with compile-time
 * indices. */
template <bool CUR, int M, bool PAIRSTEP>
QQMC_HD cplx final_value(const AdaptCtx<CUR> &a, const cplx *Pn, int k, int b, int bq)
{
    constexpr int MM = PAIRSTEP ? M - 2 : M - 1;
    static_assert(MM == 2 || MM == 3, "closed forms cover two or three rows");
    const int n = a.n;
    Blk<MM> B;
    if constexpr (!PAIRSTEP) {
        const cplx p = csub(a.g0, cld(Pn, 0));
        const cplx rp = crecip(p);
        cplx cp[MM], rw[MM];
#pragma unroll
        for (int i = 1; i < M; ++i) {
            cp[i - 1] = cmul(csub(wick_entry(a.pr, k + i, k, b), cld(Pn, i * M)), rp);
            rw[i - 1] = csub(wick_entry_m<CUR>(a.pr, a.mc, k, k + i, n, b), cld(Pn, i));
        }
#pragma unroll
        for (int i = 0; i < MM; ++i)
#pragma unroll
            for (int j = 0; j < MM; ++j) B.v[i][j] = cfma(cp[i], rw[j], cld(Pn, (i + 1) * M + j + 1));
    } else {
        const cplx av = csub(a.g0, cld(Pn, 0)), dv = csub(a.g0, cld(Pn, M + 1));
        const cplx be = csub(wick_entry(a.pr, k, k + 1, b), cld(Pn, 1));
        const cplx ga = csub(wick_entry(a.pr, k + 1, k, b), cld(Pn, M));
        const cplx r = crecip(cfms(be, ga, cmul(av, dv)));
        const cplx dd = cmul(dv, r), aa = cmul(av, r), bb = cmul(be, r), gg = cmul(ga, r);
        cplx U[MM], V[MM], xx[MM], yy[MM];
#pragma unroll
        for (int i = 2; i < M; ++i) {
            const cplx u = csub(wick_entry(a.pr, k + i, k, b), cld(Pn, i * M));
            const cplx z = csub(wick_entry(a.pr, k + i, k + 1, bq), cld(Pn, i * M + 1));
            U[i - 2] = cfms(z, gg, cmul(u, dd));
            V[i - 2] = cfms(u, bb, cmul(z, aa));
            xx[i - 2] = csub(wick_entry_m<CUR>(a.pr, a.mc, k, k + i, n, b), cld(Pn, i));
            yy[i - 2] = csub(wick_entry_m<CUR>(a.pr, a.mc, k + 1, k + i, n, bq), cld(Pn, M + i));
        }
#pragma unroll
        for (int i = 0; i < MM; ++i)
#pragma unroll
            for (int j = 0; j < MM; ++j)
                B.v[i][j] = cfma(V[i], yy[j], cfma(U[i], xx[j], cld(Pn, (i + 2) * M + j + 2)));
    }
    if constexpr (MM == 2) return leaf_value<CUR>(B, a.g0, a.lk);
    else return node3_value<CUR>(B, a.pr, a.mc, n - 2, n, a.g0, a.lk);
}

template <class X> QQMC_HD double lanes_max(X &x, double *red)
{
    (void)x;
    double g = 0.0;
    for (int l = 0; l < 64; ++l) g = fmax(g, red[l]);
    return g;
}

/* Breadth-first evaluation below a start block S (m x m with m <= MB,
 * first row global vertex k; null = zero): adds w0 times the signed sum of
 * its leaves, relative to S, into the lanes' partial sums. */
template <bool CUR, class X>
QQMC_HD void adapt_bfs(X &x, const AdaptCtx<CUR> &a, const cplx *S, int m, int k, cplx w0)
{
    const int n = a.n;
    if (m <= 3) {
        x.par([&](int l) {
            if (l == 0)
                a.part[0] = cadd(a.part[0],
                                 cmul(w0, tail_value<CUR>(S, m, n, a.pr, a.mc, a.g0, a.lk)));
        });
        return;
    }
    const cplx *P = S;
    int c = 1, cur = 0;
    x.par([&](int l) { if (l == 0) a.nw[0] = w0; });
    for (;;) {
        const int m1 = m - 1, m2 = m - 2;
        const bool keep1 = m1 > 3, keep2 = m2 > 3;
        /* single-step growth of every (node, b); vectors for stored children */
        x.par([&](int l) {
            double g = 0.0;
            if (l < 2 * c) {
                const int nd = l >> 1, b = l & 1;
                const cplx *Pn = P ? P + nd * m * m : nullptr;
                cplx p;
                cplx *cp = keep1 ? a.vs + l * 2 * m1 : nullptr;
                g = single_vectors<CUR>(Pn, m, k, n, b, a.pr, a.mc, a.g0, p, cp,
                                        cp ? cp + m1 : nullptr);
                a.wsn[l] = child_weight(a.nw[nd], p, b);
            }
            a.red[l] = g;
        });
        const double g1 = lanes_max(x, a.red);
        bool pair = false;
        if (!(g1 <= kGrowthSingle * kGrowthSingle)) {
            x.par([&](int l) {
                double g = 0.0;
                if (l < 4 * c) {
                    const int nd = l >> 2, b = (l >> 1) & 1, bq = l & 1;
                    const cplx *Pn = P ? P + nd * m * m : nullptr;
                    cplx det;
                    cplx *q = keep2 ? a.vp + nd * 12 * m2 : nullptr;
                    g = pair_vectors<CUR>(Pn, m, k, n, b, bq, a.pr, a.mc, a.g0, det,
                                          q ? q + (b * 2 + bq) * 2 * m2 : nullptr,
                                          q ? q + (b * 2 + bq) * 2 * m2 + m2 : nullptr,
                                          q ? q + 8 * m2 + b * m2 : nullptr,
                                          q ? q + 10 * m2 + bq * m2 : nullptr);
                    a.wpn[l] = child_weight(a.nw[nd], det, b ^ bq);
                }
                a.red[l] = g;
            });
            const double g2 = lanes_max(x, a.red);
            pair = g2 < g1;
        }
        const int mm = pair ? m2 : m1;       /* child size  */
        const int cc = pair ? 4 * c : 2 * c; /* child count */
        const cplx *W = pair ? a.wpn : a.wsn;
        if (mm <= 3) {
            /* last step: each lane builds one child block in registers and
             * evaluates the closed form (a last single step starts from a
             * 4 x 4 block, a last pair step from 4 x 4 or 5 x 5) */
            x.par([&](int l) {
                if (l < cc) {
                    cplx v;
                    if (!pair) {
                        const int nd = l >> 1;
                        v = final_value<CUR, 4, false>(a, P ? P + nd * 16 : nullptr, k, l & 1, 0);
                    } else if (m == 4) {
                        const int nd = l >> 2;
                        v = final_value<CUR, 4, true>(a, P ? P + nd * 16 : nullptr, k, (l >> 1) & 1,
                                                      l & 1);
                    } else {
                        const int nd = l >> 2;
                        v = final_value<CUR, 5, true>(a, P ? P + nd * 25 : nullptr, k, (l >> 1) & 1,
                                                      l & 1);
                    }
                    a.part[l] = cadd(a.part[l], cmul(W[l], v));
                }
            });
            return;
        }
        /* stored step: the children's blocks into the other level buffer,
         * their weights become the next level's node weights */
        cplx *Q = a.lvl + cur * a.lvl_size;
        const int per = mm * mm;
        x.par([&](int l) {
            for (int e = l; e < cc * per; e += 64) {
                const int ch = e / per, ij = e - ch * per, i = ij / mm, j = ij - i * mm;
                cplx v;
                if (!pair) {
                    const int nd = ch >> 1;
                    const cplx *cp = a.vs + ch * 2 * m1;
                    v = cfma(cp[i], cp[m1 + j], cld(P ? P + nd * m * m : nullptr, (i + 1) * m + j + 1));
                } else {
                    const int nd = ch >> 2, b = (ch >> 1) & 1, bq = ch & 1;
                    const cplx *q = a.vp + nd * 12 * m2;
                    const cplx *Uc = q + (b * 2 + bq) * 2 * m2;
                    v = cfma(Uc[m2 + i], q[10 * m2 + bq * m2 + j],
                             cfma(Uc[i], q[8 * m2 + b * m2 + j],
                                  cld(P ? P + nd * m * m : nullptr, (i + 2) * m + j + 2)));
                }
                Q[e] = v;
            }
            if (l < cc) a.nw[l] = W[l];
        });
        P = Q;
        c = cc;
        m = mm;
        k += pair ? 2 : 1;
        cur ^= 1;
    }
}

/* One top step of the replay: from node C (m x m, m > MB) the decision and
 * the child d (0..1 for a single step, 0..3 for a pair, (b, bq) = (d >> 1,
 * d & 1)) into Q.  Returns the child's size (m - 1 or m - 2) and sets
 * `pair` and the child's weight. */
template <bool CUR, class X>
QQMC_HD int adapt_top_step(X &x, const AdaptCtx<CUR> &a, const cplx *C, int m, int k, int d,
                           cplx w, cplx *Q, bool &pair, cplx &wc)
{
    const int n = a.n;
    {
        x.par([&](int l) {
            double g = 0.0;
            if (l < 2) {
                cplx p;
                g = single_vectors<CUR>(C, m, k, n, l, a.pr, a.mc, a.g0, p, nullptr, nullptr);
            }
            a.red[l] = g;
        });
        const double g1 = lanes_max(x, a.red);
        pair = false;
        if (!(g1 <= kGrowthSingle * kGrowthSingle)) {
            x.par([&](int l) {
                double g = 0.0;
                if (l < 4) {
                    cplx det;
                    g = pair_vectors<CUR>(C, m, k, n, l >> 1, l & 1, a.pr, a.mc, a.g0, det,
                                          nullptr, nullptr, nullptr, nullptr);
                }
                a.red[l] = g;
            });
            const double g2 = lanes_max(x, a.red);
            pair = g2 < g1;
        }
    }
    const int mm = pair ? m - 2 : m - 1;
    /* the chosen child's vectors (lane 0), then its entries */
    x.par([&](int l) {
        if (l == 0) {
            if (!pair) {
                cplx p;
                single_vectors<CUR>(C, m, k, n, d & 1, a.pr, a.mc, a.g0, p, a.vs, a.vs + mm);
                a.wsn[0] = child_weight(w, p, d & 1);
            } else {
                cplx det;
                const int b = (d >> 1) & 1, bq = d & 1;
                pair_vectors<CUR>(C, m, k, n, b, bq, a.pr, a.mc, a.g0, det, a.vp, a.vp + mm,
                                  a.vp + 2 * mm, a.vp + 3 * mm);
                a.wsn[0] = child_weight(w, det, b ^ bq);
            }
        }
    });
    x.par([&](int l) {
        for (int e = l; e < mm * mm; e += 64) {
            const int i = e / mm, j = e - i * mm;
            Q[e] = pair ? cfma(a.vp[mm + i], a.vp[3 * mm + j],
                               cfma(a.vp[i], a.vp[2 * mm + j], cld(C, (i + 2) * m + j + 2)))
                        : cfma(a.vs[i], a.vs[mm + j], cld(C, (i + 1) * m + j + 1));
        }
    });
    wc = a.wsn[0];
    x.par([&](int) {});
    return mm;
}

/* Signed leaf sum below a start block S (m x m, first row global vertex k;
 * null = zero, the whole point) times w0, evaluated by the whole wave: top
 * levels depth first with replay while the block exceeds MB x MB, then
 * breadth first.  The result is the same in every lane. */
template <bool CUR, int MB, class X>
QQMC_HD cplx adapt_eval(X &x, const AdaptCtx<CUR> &a, const cplx *S, int m, int k, cplx w0)
{
    x.par([&](int l) { a.part[l] = cmk(0.0, 0.0); });
    if (m <= MB) {
        adapt_bfs<CUR>(x, a, S, m, k, w0);
    } else {
        /* top path: digit per level (2 bits), pair decisions per level */
        uint32_t digits = 0, pairs = 0;
        for (;;) {
            const cplx *C = S;
            int mc_ = m, kc = k, lv = 0, buf = 0;
            cplx w = w0;
            while (mc_ > MB) {
                bool pr_ = false;
                cplx wc;
                cplx *Q = a.rep + buf * a.rep_size;
                const int d = (int)((digits >> (2 * lv)) & 3u);
                const int mm = adapt_top_step<CUR>(x, a, C, mc_, kc, d, w, Q, pr_, wc);
                if (pr_) pairs |= 1u << lv;
                else pairs &= ~(1u << lv);
                kc += mc_ - mm;
                mc_ = mm;
                w = wc;
                C = Q;
                buf ^= 1;
                ++lv;
            }
            adapt_bfs<CUR>(x, a, C, mc_, kc, w);
            /* next top path */
            int l = lv - 1;
            for (; l >= 0; --l) {
                const uint32_t radix = ((pairs >> l) & 1u) ? 4u : 2u;
                const uint32_t dl = ((digits >> (2 * l)) & 3u) + 1u;
                digits &= ~(3u << (2 * l));
                if (dl < radix) {
                    digits |= dl << (2 * l);
                    break;
                }
            }
            if (l < 0) break;
        }
    }
    cplx s = cmk(0.0, 0.0);
    for (int l = 0; l < 64; ++l) s = cadd(s, a.part[l]);
    x.par([&](int) {});
    return s;
}

} // namespace qqmc
#endif
