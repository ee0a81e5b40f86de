/*
 * qqmc_kernels.h -- device code shared by the kernel translation units
 * (qqmc_kernels*.hip): local-memory layout, wave helpers, the cooperative top
 * blocks, the per-point Keldysh sums, the tile function and the kernel
 * templates, and generic launchers for one (order, variant).  Each variant
 * (scalar or paired elimination tree, charge or current, lattice or Sobol'
 * points) is instantiated in its own translation unit, so they compile in
 * parallel; the units call one another only through the named functions
 * declared at the end.
 *
 * Work decomposition.  One workgroup is one 64-lane wavefront.  A work tile
 * is (shift s, 64*c consecutive lattice indices).  For every 64 indices the
 * wave
 *   1. generates the shifted Korobov lattice point and warps it through the
 *      inverse CDF of the product model h(v) = exp(-v/tau) (one lane per
 *      index: Eqs. (warper1d), (x_of_v_simple), (hi_expo)),
 *   2. compacts the points inside the domain 0 < u_n (App. I: points outside
 *      contribute exactly zero) with a ballot,
 *   3. for every compacted point builds the pair table of interpolated
 *      g^<(tau), g^>(tau) in LDS (lanes of the point's group share the work),
 *   4. evaluates the Keldysh sum with the elimination tree of qqmc_tree.h,
 *      G = 2^T lanes per point (or per top-level prefix above order 10),
 *   5. folds -2 i^{n+1} S(u) W into a per-lane compensated accumulator.
 * The tree kernels whose lanes start from a 6 x 6 block (scalar orders 5
 * and up, every paired order from 4) are compiled for one wave per SIMD:
 * the register tree needs the whole register file (architectural and
 * accumulation registers) and spills nothing; the smaller orders run two
 * waves per SIMD (Geo::WPS).
 * The tile's sum goes to one slot of a partials array; a second kernel sums
 * the slots of each shift in a fixed order.  No floating-point atomics are
 * used anywhere, so results are bitwise reproducible.
 */
#ifndef QQMC_KERNELS_H
#define QQMC_KERNELS_H

#include "qqmc_gf.h"
#include "qqmc_internal.h"
#include "qqmc_tree.h"
#include "qqmc_adapt.h"

namespace qqmc {

namespace {

constexpr int WAVE = 64;
constexpr int ilog2(int v) { return v > 1 ? 1 + ilog2(v / 2) : 0; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
/* offset of chain level k's output among the kept chain blocks of order n:
 * the sum of (n - j)^2 over the levels j < k */
constexpr int chain_off(int n, int k) { return k <= 0 ? 0 : chain_off(n, k - 1) + (n - k + 1) * (n - k + 1); }
/* Workgroup size of every kernel that exchanges data through local memory
 * with wave_sync (the tree kernels and the adaptive path): one wavefront,
 * so that its local-memory operations execute in program order.  Their
 * __launch_bounds__ and their launches both take it from here. */
constexpr int WG_TREE = WAVE;
static_assert(WG_TREE == WAVE, "the tree kernels run one wavefront per workgroup");

template <int N, bool PAIR = false, bool CUR = false, bool SOB = false, int MAP = kMapDefault> struct Lds {
    using Gm = Geo<N, PAIR, MAP>;
    /* pair-table stride: the NP pairs, then for the current the n lead
     * values of the measurement column */
    static constexpr int NPS = Gm::NP + (CUR ? N : 0);
    /* queued in-domain points of a tile: up to 63 carried over plus the 64
     * of one step.  The queue runs where it measured faster: one-wave
     * kernels with several lanes per point (scalar tree orders 6-10, paired
     * tree orders 6 and 8).  Elsewhere it was as fast or slower: the
     * two-wave orders 1-4 are limited by local memory, with one lane per
     * point (order 5) the rounds are nearly full anyway, above order 10
     * (three or more cooperative top levels) it measured 1% slower at order
     * 11 and even at 12-14, and the paired order-7 kernel sits at 256
     * registers, which the queue's extra live values overflow into
     * accumulation registers (10% slower).  The paired tree above order 8
     * keeps the per-step loop: its local memory goes to the adaptive path's
     * workspace. */
    static constexpr bool QUEUE =
        Gm::WPS == 1 && Gm::G > 1 && Gm::OFF <= 2 && (!PAIR || (Gm::OFF == 0 && N != 7));
    static constexpr int QCAP = QUEUE ? 128 : 64;
    static constexpr int times = 0;                                    /* QCAP*N doubles */
    static constexpr int w = times + QCAP * N * 8;                     /* QCAP doubles   */
    static constexpr int S = w + QCAP * 8;                             /* QCAP cplx      */
    static constexpr int ids = S + QCAP * 16;                          /* QCAP int32     */
    /* pair tables: one per item group, or one per distinct point of a
     * round when several items share a point */
    static constexpr int tables =
        Gm::IPP == 1 ? Gm::PPW : (Gm::PPW >= Gm::IPP ? Gm::PPW / Gm::IPP : 1);
    static constexpr int pairs = ids + QCAP * 4;                       /* tables*NP pairv */
    /* broadcast rows per group of the paired tree's pair steps and of the
     * per-item top's two-level steps */
    static constexpr int rows = 2;
    static constexpr int row = pairs + tables * NPS * 32;      /* rows*PPW*(N+1) cplx */
    /* the round-shared top of the scalar tree (the default mapping above
     * order 10 and the cooperative-top mapping at orders 9 and 10; the
     * depth-4 mapping, two waves per SIMD, keeps per-item tops, whose fewer
     * live values it measured 1.5-2.2x faster with): instead of the rows, a
     * block buffer (the levels whose children do not go to the c0 blocks),
     * the rank-1 vectors of one level and the pivots */
    static constexpr bool RTOP = !PAIR && Gm::OFF > 0 && MAP != kMapDepth4;
    /* tree levels per point (the round holds `tables` points) */
    static constexpr int TL = RTOP ? ilog2(Gm::PPW / tables) : 0;
    static constexpr int ybuf = RTOP ? cmax(N * N, (Gm::PPW / 2) * (Gm::K + 1) * (Gm::K + 1)) : 0;
    static constexpr int vecn = RTOP ? cmax(2 * N, 2 * Gm::PPW * Gm::K) : 0;
    static constexpr int pivn = 16;
    /* the shared chain levels' outputs but the last, kept from one round of
     * a point to the next (levels 0 .. CH-2, blocks of (n-k)^2) */
    static constexpr int CH = RTOP ? Gm::OFF - TL : 0;
    static constexpr int cbufn = CH >= 2 ? chain_off(N, CH - 1) : 0;
    static constexpr int row_bytes =
        RTOP ? (ybuf + vecn + pivn + cbufn) * 16 : rows * Gm::PPW * (N + 1) * 16;
    static constexpr int c0 = row + (Gm::OFF > 0 ? row_bytes : 0);
    static constexpr int c0_end = c0 + (Gm::OFF > 0 ? Gm::PPW * Gm::K * Gm::K * 16 : 0);
    /* the paired tree's adaptive re-evaluation (qqmc_adapt.h), placed
     * before the Sobol' numbers so that its offset and size are the same with
     * and without them; its breadth-first start size MB is the largest that
     * keeps a workgroup (Sobol' numbers included) within 40 KiB, the share
     * of each of the four one-wave workgroups a compute unit holds in its
     * 160 KiB of local memory */
    /* the paired tree's flagged points carried from one batch of a tile to
     * the next (orders <= 8): up to eight points' times and weights, their
     * count, the results of a pass and the sum of their contributions */
    static constexpr bool CARRY = PAIR && Gm::OFF == 0;
    static constexpr int dq = (c0_end + 15) & ~15;                     /* 8*N doubles */
    static constexpr int dq_w = dq + (CARRY ? 8 * N * 8 : 0);          /* 8 doubles   */
    static constexpr int dq_res = dq_w + (CARRY ? 8 * 8 : 0);          /* 8 cplx      */
    static constexpr int dq_sum = dq_res + (CARRY ? 8 * 16 : 0);       /* cplx        */
    static constexpr int dq_n = dq_sum + (CARRY ? 16 : 0);             /* int         */
    static constexpr int dq_end = dq_n + (CARRY ? 16 : 0);
    static constexpr int adapt = (dq_end + 15) & ~15;
    static constexpr int sob_bytes = N * 32 * 4;
    static constexpr int kShare = 40960;
    static constexpr int MB = !PAIR ? 8
                              : adapt + AdaptWs<N, 8>::bytes + sob_bytes <= kShare ? 8
                              : adapt + AdaptWs<N, 7>::bytes + sob_bytes <= kShare ? 7 : 6;
    /* Sobol' direction numbers, N x 32 words */
    static constexpr int sobv = adapt + (PAIR ? AdaptWs<N, MB>::bytes : 0);
    static constexpr int bytes = sobv + (SOB ? sob_bytes : 0);
    /* one-wave-per-SIMD kernels: four workgroups share a compute unit's
     * 160 KiB of local memory */
    static_assert(Gm::WPS != 1 || bytes <= kShare, "a one-wave workgroup within a quarter of LDS");
};

__device__ __forceinline__ double shfl_xor_d(double v, int m)
{
    return __shfl_xor(v, m, WAVE);
}

/* Ordering point for the single-wave workgroups of the tree kernels: the
 * local-memory operations of one wave execute in program order, so lanes
 * exchanging data through local memory need only keep the compiler from
 * moving memory operations across this point -- no hardware barrier and no
 * wait for outstanding local-memory operations.  Every kernel that uses it
 * is launched with exactly one 64-lane wave per workgroup. */
__device__ __forceinline__ void wave_sync()
{
    asm volatile("" ::: "memory");
}

__device__ __forceinline__ int lane_rank(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

/* Later point j of the pair with triangular index q = j(j-1)/2 + i, i < j:
 * the largest j with j(j-1)/2 <= q (float square root is exact enough for
 * q < 2^20; the two integer corrections make it exact regardless). */
__device__ __forceinline__ int pair_hi(int q)
{
    int j = (int)((1.0f + sqrtf(8.0f * (float)q + 1.0f)) * 0.5f);
    if (j * (j - 1) / 2 > q) --j;
    if ((j + 1) * j / 2 <= q) ++j;
    return j;
}

/* -2 i^{n+1} S: the charge prefactor (spin sum 2, i^n of the expansion, the
 * extra -i of <n> = -i g^<). */
template <int N> __device__ __forceinline__ cplx charge_prefactor(cplx s)
{
    constexpr int q = (N + 1) & 3;
    if constexpr (q == 0) return cmk(-2.0 * s.x, -2.0 * s.y);
    else if constexpr (q == 1) return cmk(2.0 * s.y, -2.0 * s.x);
    else if constexpr (q == 2) return cmk(2.0 * s.x, 2.0 * s.y);
    else return cmk(-2.0 * s.y, 2.0 * s.x);
}

/* -4 i^n S: its real part is the order-n integrand of the particle current
 * into the lead (both spins); the charge's is -2 i^{n+1} S. */
template <int N, bool CUR> __device__ __forceinline__ cplx observable_prefactor(cplx s)
{
    if constexpr (!CUR) {
        return charge_prefactor<N>(s);
    } else {
        constexpr int q = N & 3;
        if constexpr (q == 0) return cmk(-4.0 * s.x, -4.0 * s.y);
        else if constexpr (q == 1) return cmk(4.0 * s.y, -4.0 * s.x);
        else if constexpr (q == 2) return cmk(4.0 * s.x, 4.0 * s.y);
        else return cmk(-4.0 * s.y, 4.0 * s.x);
    }
}

struct Kahan {
    double sx = 0.0, sy = 0.0, cx = 0.0, cy = 0.0;
    __device__ __forceinline__ void add(cplx v)
    {
        double y = v.x - cx, t = sx + y;
        cx = (t - sx) - y; sx = t;
        y = v.y - cy; t = sy + y;
        cy = (t - sy) - y; sy = t;
    }
    __device__ __forceinline__ cplx value() const { return cmk(sx - cx, sy - cy); }
};

/* Fixed-order butterfly over the whole wave; every lane ends with the same
 * bits (IEEE addition is commutative). */
__device__ __forceinline__ cplx wave_sum(cplx v)
{
#pragma unroll
    for (int m = 1; m < WAVE; m <<= 1) {
        v.x += shfl_xor_d(v.x, m);
        v.y += shfl_xor_d(v.y, m);
    }
    return v;
}

/* Environment of the points being evaluated (one parameter point). */
struct Env {
    const double *tab;
    double t_half, inv_h, t_meas;
    cplx g0;      /* vertex diagonal i (n_sigma - alpha)                      */
    cplx gm;      /* measurement diagonal i n_sigma (the direct method only)  */
    const double *col; /* current: the lead's gamma g^<_{0i}, gamma g^>_{0i}
                          on the same grid, or null (the charge)            */
    int n_grid;
};

/* The first OFF = n - 8 eliminations of a work item in the depth-4 mapping
 * (n > 10), done by the G lanes of the item's group with whole matrix rows
 * per lane (row r on lane r mod G; right-looking, no pivoting, index prefix
 * `top`).  Leaves the 9 x 9 trailing correction block in s_c0 and returns
 * the product of the OFF pivots.
 *
 * Levels go two at a time: with T = (Wick entries) - C the trailing matrix,
 * vertices k and k+1 are eliminated together through their 2x2 block
 * P = [[T_kk, T_k,k+1], [T_k+1,k, T_k+1,k+1]] (entries of vertex k on b_k,
 * the later row of k+1 on b_k+1),
 *     C_rj += [T_rk T_r,k+1] P^{-1} [T_kj; T_k+1,j],   j, r > k + 1,
 * which is the two single steps' Schur complement, and det P is the product
 * of their two pivots.  Both owners broadcast their rows through s_row at
 * once, so a pair of levels waits on local memory once instead of twice;
 * an odd last level is a single step. */
template <int N, bool CUR = false, int MAP = kMapDefault>
__device__ cplx top_block(const pairv *pr, const pairv *mc, int top, int sub, cplx g0,
                          cplx *s_row, cplx *s_c0)
{
    using Gm = Geo<N, false, MAP>;
    constexpr int OFF = Gm::OFF, K = Gm::K, G = Gm::G;
    constexpr int RPL = (N + G) / G; /* rows per lane: ceil((N + 1) / G) */
    cplx *s_r0 = s_row, *s_r1 = s_row + (N + 1);
    cplx crow[RPL][N + 1];
#pragma unroll
    for (int m = 0; m < RPL; ++m)
#pragma unroll
        for (int j = 0; j <= N; ++j) crow[m][j] = cmk(0.0, 0.0);
    cplx prod = cmk(1.0, 0.0);
#pragma unroll
    for (int k = 0; k < OFF; k += 2) {
        const int b = (top >> (OFF - 1 - k)) & 1;
        if (k + 1 < OFF) {
            const int bq = (top >> (OFF - 2 - k)) & 1;
#pragma unroll
            for (int m = 0; m < RPL; ++m) {
                const int r = sub + m * G;
                /* every table read before the first store, so the reads
                 * are issued together rather than each behind a store it
                 * might alias */
                if (r == k) {
                    cplx v[N + 1];
#pragma unroll
                    for (int j = k + 1; j <= N; ++j)
                        v[j] = csub(wick_entry_m<CUR>(pr, mc, k, j, N, b), crow[m][j]);
                    s_r0[k] = csub(g0, crow[m][k]);
#pragma unroll
                    for (int j = k + 1; j <= N; ++j) s_r0[j] = v[j];
                } else if (r == k + 1) {
                    cplx v[N + 1];
                    /* (k+1, k): the earlier point is k, so index b */
                    v[k] = csub(wick_entry(pr, k + 1, k, b), crow[m][k]);
#pragma unroll
                    for (int j = k + 2; j <= N; ++j)
                        v[j] = csub(wick_entry_m<CUR>(pr, mc, k + 1, j, N, bq), crow[m][j]);
                    s_r1[k] = v[k];
                    s_r1[k + 1] = csub(g0, crow[m][k + 1]);
#pragma unroll
                    for (int j = k + 2; j <= N; ++j) s_r1[j] = v[j];
                }
            }
            wave_sync();
            const cplx a = s_r0[k], bb = s_r0[k + 1], c = s_r1[k], d = s_r1[k + 1];
            const cplx det = cfms(bb, c, cmul(a, d)); /* a d - bb c */
            const cplx rd = crecip_nr(det);
            const cplx ia = cmul(a, rd), ib = cmul(bb, rd), ic = cmul(c, rd), id = cmul(d, rd);
#pragma unroll
            for (int m = 0; m < RPL; ++m) {
                const int r = sub + m * G;
                if (r > k + 1 && r <= N) {
                    const cplx u = csub(wick_entry(pr, r, k, b), crow[m][k]);
                    const cplx v = csub(wick_entry(pr, r, k + 1, bq), crow[m][k + 1]);
                    /* [x y] = [u v] P^{-1} */
                    const cplx x = cfms(v, ic, cmul(u, id));
                    const cplx y = cfms(u, ib, cmul(v, ia));
#pragma unroll
                    for (int j = k + 2; j <= N; ++j)
                        crow[m][j] = cfma(y, s_r1[j], cfma(x, s_r0[j], crow[m][j]));
                }
            }
            prod = cmul(prod, det);
            wave_sync();
        } else {
#pragma unroll
            for (int m = 0; m < RPL; ++m) {
                if (sub + m * G == k) {
                    cplx v[N + 1];
#pragma unroll
                    for (int j = k + 1; j <= N; ++j)
                        v[j] = csub(wick_entry_m<CUR>(pr, mc, k, j, N, b), crow[m][j]);
                    s_r0[k] = csub(g0, crow[m][k]);
#pragma unroll
                    for (int j = k + 1; j <= N; ++j) s_r0[j] = v[j];
                }
            }
            wave_sync();
            const cplx p = s_r0[k];
            const cplx rp = crecip_nr(p);
#pragma unroll
            for (int m = 0; m < RPL; ++m) {
                const int r = sub + m * G;
                if (r > k && r <= N) {
                    const cplx ch = cmul(csub(wick_entry(pr, r, k, b), crow[m][k]), rp);
#pragma unroll
                    for (int j = k + 1; j <= N; ++j) crow[m][j] = cfma(ch, s_r0[j], crow[m][j]);
                }
            }
            prod = cmul(prod, p);
            wave_sync();
        }
    }
#pragma unroll
    for (int m = 0; m < RPL; ++m) {
        const int r = sub + m * G;
        if (r >= OFF && r <= N) {
#pragma unroll
            for (int j = OFF; j <= N; ++j) s_c0[(r - OFF) * K + (j - OFF)] = crow[m][j];
        }
    }
    wave_sync();
    return prod;
}

/* One level of the round-shared top: NPAR parent correction blocks of
 * size M x M at src (zero when ZERO), each eliminated at its first index
 * (global index gk) for NB index values (both, or the fixed bfix), giving
 * NPAR * NB child blocks of size (M-1) x (M-1) at dst, child (P, b) at
 * position P * NB + b, and the parents' pivots at s_piv[0..NPAR).  Phase
 * one computes every parent's pivot and its rank-1 vectors
 *     c_b[i] = (W_b(i, 0) - C[i][0]) / p,   row_b[j] = W_b(0, j) - C[0][j],
 * phase two every child entry C[i][j] + c_b[i] row_b[j], both spread over
 * the 64 lanes; each phase issues all its local-memory reads before it
 * computes, so a level waits on local memory twice (the first level, whose
 * parent is zero, once). */
template <int N, bool CUR, int NPAR, int NB, int M, bool ZERO, int PPP, int NPS>
__device__ __forceinline__ void rtop_level(const pairv *pr0, int gk, int bfix, cplx g0,
                                           const cplx *src, cplx *dst, cplx *s_vec, cplx *s_piv)
{
    constexpr int S = M - 1;
    /* parent P belongs to point P / PPP of the round, whose pair table is
     * pr0 + (P / PPP) NPS; the measurement column of the current follows
     * the NP pairs, the charge's is the pairs (k, n) */
    constexpr int MC = CUR ? N * (N + 1) / 2 : pidx(0, N);
    const int lane = threadIdx.x;
    if constexpr (!ZERO) {
        /* column and row tasks in separate loops (one vector entry of each
         * per task q = (P NB + b) S + idx - 1), so that no iteration branches
         * on the kind */
        constexpr int NC = NPAR * NB * S;
        constexpr int IC = (NC + WAVE - 1) / WAVE;
        static_assert(NPAR <= WAVE, "one pivot per lane");
        cplx vc[IC], vr[IC];
#pragma unroll
        for (int t = 0; t < IC; ++t) {
            const int q = lane + t * WAVE < NC ? lane + t * WAVE : NC - 1;
            const int idx = q % S + 1;
            const int b = NB == 2 ? (q / S) & 1 : bfix;
            const int P = q / (NB * S);
            const pairv *pr = pr0 + (P / PPP) * NPS;
            const cplx *C = src + P * M * M;
            const cplx p = csub(g0, C[0]);
            vc[t] = cmul(csub(wick_entry(pr, gk + idx, gk, b), C[idx * M]), crecip_nr(p));
            vr[t] = csub(wick_entry_m<CUR>(pr, pr + MC, gk, gk + idx, N, b), C[idx]);
        }
        /* lanes past the end repeat the last task (or parent 0) and store
         * the same value to the same address, so no store needs a branch */
        const int pl = lane < NPAR ? lane : 0;
        const cplx vp = csub(g0, src[pl * M * M]);
#pragma unroll
        for (int t = 0; t < IC; ++t) {
            const int q = lane + t * WAVE < NC ? lane + t * WAVE : NC - 1;
            const int o = (q / S) * 2 * S + q % S;
            s_vec[o] = vc[t];
            s_vec[o + S] = vr[t];
        }
        s_piv[pl] = vp;
        wave_sync();
    } else {
        /* the first level: zero parents, so the vectors are Wick entries
         * (the columns over the vertex diagonal g0), read where they are
         * used below; no vector phase */
        static_assert(NPAR <= WAVE && PPP == 1, "one parent per point at the first level");
        s_piv[lane < NPAR ? lane : 0] = g0;
    }
    constexpr int NE = NPAR * S * S;
    constexpr int IE = (NE + WAVE - 1) / WAVE;
    const cplx r0 = ZERO ? crecip_nr(g0) : cmk(0.0, 0.0);
    cplx cc[IE], cv[IE][NB], rv[IE][NB];
#pragma unroll
    for (int t = 0; t < IE; ++t) {
        const int q = lane + t * WAVE < NE ? lane + t * WAVE : NE - 1;
        const int P = q / (S * S), rem = q % (S * S), i = rem / S, j = rem % S;
        cc[t] = ZERO ? cmk(0.0, 0.0) : src[P * M * M + (i + 1) * M + (j + 1)];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if constexpr (ZERO) {
                const int bb = NB == 2 ? b : bfix;
                const pairv *pr = pr0 + P * NPS;
                cv[t][b] = cmul(wick_entry(pr, gk + i + 1, gk, bb), r0);
                rv[t][b] = wick_entry_m<CUR>(pr, pr + MC, gk, gk + j + 1, N, bb);
            } else {
                cv[t][b] = s_vec[((P * NB + b) * 2 + 0) * S + i];
                rv[t][b] = s_vec[((P * NB + b) * 2 + 1) * S + j];
            }
        }
    }
#pragma unroll
    for (int t = 0; t < IE; ++t) {
        const int q = lane + t * WAVE < NE ? lane + t * WAVE : NE - 1;
        const int P = q / (S * S), rem = q % (S * S);
#pragma unroll
        for (int b = 0; b < NB; ++b)
            dst[(P * NB + b) * S * S + rem] = cfma(cv[t][b], rv[t][b], cc[t]);
    }
    wave_sync();
}

/* Levels LAM.. of the round-shared top: the first CH = OFF - TL are the
 * chain of index bits that the round's items share (one parent, one child),
 * the last TL the tree over the bits in which they differ, for each of the
 * round's PTS points (PTS 2^l parents at tree level l; a chain only with one
 * point per round).  Chain levels before k0 are skipped: their outputs,
 * kept in s_c (all chain levels but the last), are those of the previous
 * round of the same point.  The last chain level writes the buffer that the
 * first tree level does not, and the tree levels alternate between s_x and
 * s_y so that no level reads the buffer it writes; the children of the last
 * level land in the c0 blocks (s_x). */
template <int N, bool CUR, int MAP, int LAM, int OFF, int TL, int PTS>
__device__ __forceinline__ void rtop_levels(const pairv *pr0, int rpre, int k0, cplx g0,
                                            cplx *s_x, cplx *s_y, cplx *s_c, cplx *s_vec,
                                            cplx *s_piv)
{
    if constexpr (LAM < OFF) {
        using L = Lds<N, false, CUR, false, MAP>;
        using Gm = Geo<N, false, MAP>;
        constexpr int CH = OFF - TL;
        constexpr bool TREE = LAM >= CH;
        constexpr int PPP = TREE ? (1 << (LAM - CH)) : 1;
        constexpr int NPAR = TREE ? PTS * PPP : 1, NB = TREE ? 2 : 1;
        constexpr int M = N + 1 - LAM, SH = TREE ? 0 : CH - 1 - LAM;
        /* tree level l writes s_x when TL - 1 - l is even */
        constexpr bool T0_X = ((TL - 1) & 1) == 0;
        constexpr bool TO_X = TREE ? ((OFF - 1 - LAM) & 1) == 0 : (LAM == CH - 1 ? !T0_X : false);
        constexpr bool TO_C = !TREE && LAM < CH - 1;
        static_assert(TO_C || NPAR * NB * (M - 1) * (M - 1) <=
                                  (TO_X ? Gm::PPW * Gm::K * Gm::K : L::ybuf),
                      "the level's children fit their buffer");
        static_assert(!TO_C || chain_off(N, LAM + 1) <= L::cbufn, "the chain level fits its slot");
        static_assert(NPAR * NB * 2 * (M - 1) <= L::vecn, "the level's vectors fit");
        cplx *dst = TO_C ? s_c + chain_off(N, LAM) : (TO_X ? s_x : s_y);
        const cplx *src = LAM == 0          ? nullptr
                          : LAM <= CH - 1   ? s_c + chain_off(N, LAM - 1)
                          : LAM == CH       ? (T0_X ? s_y : s_x)
                                            : (TO_X ? s_y : s_x);
        const int bfix = TREE ? 0 : (rpre >> SH) & 1;
        if (TREE || LAM >= k0)
            rtop_level<N, CUR, NPAR, NB, M, LAM == 0, PPP, L::NPS>(
                pr0, LAM, bfix, g0, src, dst, s_vec, s_piv + (TREE ? CH + PTS * (PPP - 1) : LAM));
        rtop_levels<N, CUR, MAP, LAM + 1, OFF, TL, PTS>(pr0, rpre, k0, g0, s_x, s_y, s_c, s_vec,
                                                        s_piv);
    }
}

/* The first OFF = n - 8 eliminations of the scalar tree (above order 10,
 * and at orders 9 and 10 in the cooperative-top mapping; 8 lanes per
 * item), shared by the PPW items of a round.  The round holds PTS points
 * (their pair tables from pr0 on, NPS pairs apart) of PPW / PTS items each;
 * items of a point differ in the last TL = log2(PPW / PTS) bits of their
 * index prefix and, with one point per round, share the CH = OFF - TL bits
 * before (the round's prefix rpre).  The whole wave eliminates the CH shared levels once and the TL
 * levels as a tree per point (1, 2, 4, ... parents), one level at a time,
 * instead of every item repeating the OFF levels of its own prefix.  Leaves
 * item g's 9 x 9 trailing correction block at c0 + g K K and returns, for
 * the calling lane's item grp, the product of its OFF pivots. */
template <int N, bool CUR, int MAP>
__device__ cplx round_top(const pairv *pr0, int rpre, int grp, cplx g0, char *lds)
{
    using L = Lds<N, false, CUR, false, MAP>;
    using Gm = Geo<N, false, MAP>;
    constexpr int OFF = Gm::OFF, TL = L::TL, CH = OFF - TL, PTS = L::tables;
    static_assert(L::RTOP && PTS * (1 << TL) == Gm::PPW && (PTS == 1 || CH == 0),
                  "whole points per round, a chain only with one point");
    static_assert(PTS == 1 || Gm::IPP == (1 << TL), "every item of a point in the round");
    static_assert(N + 1 - OFF == Gm::K, "the last level leaves K x K blocks");
    static_assert(CH + PTS * ((1 << TL) - 1) <= L::pivn, "pivots of every level");
    static_assert(Gm::PPW * Gm::K * Gm::K >= N * N && L::ybuf >= N * N, "chain children fit");
    static_assert(L::vecn >= 2 * N && L::vecn >= 2 * Gm::PPW * Gm::K, "vectors of every level");
    static_assert(CH == L::CH, "one chain length");
    cplx *s_x = reinterpret_cast<cplx *>(lds + L::c0);
    cplx *s_y = reinterpret_cast<cplx *>(lds + L::row);
    cplx *s_vec = s_y + L::ybuf;
    cplx *s_piv = s_vec + L::vecn;
    cplx *s_c = s_piv + L::pivn;
    /* rounds of a point come in order of rpre, from 0: chain level k (bit
     * CH-1-k of rpre) changed from the previous round iff that bit flipped,
     * i.e. from level CH-1-ctz(rpre) on; a new point (rpre 0) redoes all */
    const int k0 = rpre == 0 ? 0 : CH - 1 - __builtin_ctz((unsigned)rpre);
    /* the previous round's lanes have read their blocks */
    wave_sync();
    rtop_levels<N, CUR, MAP, 0, OFF, TL, PTS>(pr0, rpre, k0, g0, s_x, s_y, s_c, s_vec, s_piv);
    cplx prod = cmk(1.0, 0.0);
#pragma unroll
    for (int k = 0; k < CH; ++k) prod = cmul(prod, s_piv[k]);
#pragma unroll
    for (int l = 0; l < TL; ++l)
        prod = cmul(prod, s_piv[CH + PTS * ((1 << l) - 1) + (grp >> (TL - l))]);
    return prod;
}

/* The paired tree's first OFF eliminations (OFF even, n > 8): pair steps of
 * vertices (k, k+1) with 2x2 block pivots, rows spread over the G lanes as
 * in top_block.  The lanes holding rows k and k+1 broadcast them through
 * s_row (2 (n+1) entries); every lane applies the rank-2 update to its rows
 * below.  Leaves the K x K trailing correction block in s_c0 and returns the
 * product of the pivot-block determinants. */
template <int N, bool CUR = false>
__device__ cplx top_block_pair(const pairv *pr, const pairv *mc, int top, int sub, cplx g0,
                               cplx *s_row, cplx *s_c0, double &grow)
{
    using Gm = Geo<N, true>;
    constexpr int OFF = Gm::OFF, K = Gm::K, G = Gm::G;
    constexpr int RPL = (N + G) / G; /* rows per lane: ceil((N + 1) / G) */
    cplx *s_r0 = s_row, *s_r1 = s_row + (N + 1);
    cplx crow[RPL][N + 1];
#pragma unroll
    for (int m = 0; m < RPL; ++m)
#pragma unroll
        for (int j = 0; j <= N; ++j) crow[m][j] = cmk(0.0, 0.0);
    cplx prod = cmk(1.0, 0.0);
#pragma unroll
    for (int k = 0; k < OFF; k += 2) {
        const int b = (top >> (OFF - 1 - k)) & 1, bq = (top >> (OFF - 2 - k)) & 1;
#pragma unroll
        for (int m = 0; m < RPL; ++m) {
            const int r = sub + m * G;
            if (r == k) {
                cplx v[N + 1];
#pragma unroll
                for (int j = k + 1; j <= N; ++j)
                    v[j] = csub(wick_entry_m<CUR>(pr, mc, k, j, N, b), crow[m][j]);
                s_r0[k] = csub(g0, crow[m][k]);
#pragma unroll
                for (int j = k + 1; j <= N; ++j) s_r0[j] = v[j];
            } else if (r == k + 1) {
                /* (k+1, k): the earlier point is k, so index b */
                cplx v[N + 1];
                v[k] = csub(wick_entry(pr, k + 1, k, b), crow[m][k]);
#pragma unroll
                for (int j = k + 2; j <= N; ++j)
                    v[j] = csub(wick_entry_m<CUR>(pr, mc, k + 1, j, N, bq), crow[m][j]);
                s_r1[k + 1] = csub(g0, crow[m][k + 1]);
                s_r1[k] = v[k];
#pragma unroll
                for (int j = k + 2; j <= N; ++j) s_r1[j] = v[j];
            }
        }
        wave_sync();
        const cplx a = s_r0[k], be = s_r0[k + 1], ga = s_r1[k], d = s_r1[k + 1];
        const cplx det = cfms(be, ga, cmul(a, d));
        const cplx rdet = crecip_nr(det);
        const cplx dd = cmul(d, rdet), aa = cmul(a, rdet), bb = cmul(be, rdet), gg = cmul(ga, rdet);
        /* the step's elimination multipliers U, V, spread over the lanes'
         * rows, enter the lane's largest multiplier */
#pragma unroll
        for (int m = 0; m < RPL; ++m) {
            const int r = sub + m * G;
            if (r > k + 1 && r <= N) {
                const cplx u = csub(wick_entry(pr, r, k, b), crow[m][k]);
                const cplx z = csub(wick_entry(pr, r, k + 1, bq), crow[m][k + 1]);
                const cplx Ui = cfms(z, gg, cmul(u, dd));
                const cplx Vi = cfms(u, bb, cmul(z, aa));
                grow = cmaxabs(cmaxabs(grow, Ui), Vi);
#pragma unroll
                for (int j = k + 2; j <= N; ++j)
                    crow[m][j] = cfma(Vi, s_r1[j], cfma(Ui, s_r0[j], crow[m][j]));
            }
        }
        prod = cmul(prod, det);
        wave_sync();
    }
#pragma unroll
    for (int m = 0; m < RPL; ++m) {
        const int r = sub + m * G;
        if (r >= OFF && r <= N) {
#pragma unroll
            for (int j = OFF; j <= N; ++j) s_c0[(r - OFF) * K + (j - OFF)] = crow[m][j];
        }
    }
    wave_sync();
    return prod;
}

/* The adaptive path (qqmc_adapt.h) on one point whose pair table is pr
 * (measurement column mc), from the start block S (m x m, first row vertex
 * k; null: the whole point) with weight w0, in the local-memory workspace ws
 * of the kernel.  Wave-uniform result.  Not inlined: it runs for few points,
 * and as a separate function its code and registers stay out of the
 * register tree's allocation. */
template <int N, bool CUR, int MB>
__device__ __attribute__((noinline)) cplx adapt_point(const pairv *pr, const pairv *mc, cplx g0,
                                                     char *ws, const cplx *S, int m, int k,
                                                     cplx w0)
{
    using AW = AdaptWs<N, MB>;
    cplx *wsb = reinterpret_cast<cplx *>(ws);
    AdaptCtx<CUR> a;
    a.pr = pr;
    a.mc = mc;
    a.g0 = g0;
    a.n = N;
    a.lk = leaf_constants<CUR>(pr[pidx(N - 1, N)], mc[N - 1]);
    a.rep = wsb + AW::rep;
    a.lvl = wsb + AW::lvl;
    a.vs = wsb + AW::vs;
    a.vp = wsb + AW::vp;
    a.wsn = wsb + AW::wsn;
    a.wpn = wsb + AW::wpn;
    a.nw = wsb + AW::nw;
    a.part = wsb + AW::part;
    a.red = reinterpret_cast<double *>(wsb + AW::red);
    a.lvl_size = AW::LVL;
    a.rep_size = AW::RB;
    WaveLanes x;
    return adapt_eval<CUR, MB>(x, a, S, m, k, w0);
}

__device__ __forceinline__ cplx shfl_cplx(cplx v, int src)
{
    return cmk(__shfl(v.x, src, WAVE), __shfl(v.y, src, WAVE));
}

struct ShiftOut {
    cplx v;
    double grow;
};

/* One lane's share (8 lanes per point or item) of the shifted grouping
 * (lane_sum_shift): from the whole matrix for orders up to 8 (pair, then
 * single vertex), from an item's cooperative block c0 above (single vertex,
 * then pair), with the item's top product and index parity.  Not inlined:
 * it runs for the few flagged points, and as a function its registers stay
 * out of the main tree's allocation. */
template <int N, bool CUR>
__device__ __attribute__((noinline)) ShiftOut shift_lane(const pairv *pr, const pairv *mc,
                                                         const cplx *c0, int pre, int top,
                                                         cplx g0, cplx prod)
{
    BlockSrc<N, true> src;
    src.c = c0;
    ShiftOut o;
    o.grow = 0.0;
    if constexpr (Geo<N, true>::OFF == 0)
        o.v = lane_sum_shift<N, CUR, 2, 1>(pr, mc, src, pre, prod, 0, g0, o.grow);
    else
        o.v = lane_sum_shift<N, CUR, 1, 2>(pr, mc, src, pre, prod, __popc((unsigned)top) & 1, g0,
                                           o.grow);
    return o;
}

/* Entry q of a point's pair table (times tm, elimination order): the pair
 * (i, j) with q = j (j - 1) / 2 + i, or for the current beyond the NP pairs
 * the lead values of vertex q - NP, held as -conj. */
template <int N, bool CUR>
__device__ __forceinline__ pairv pair_entry(int q, const double *tm, const Env &env)
{
    constexpr int NP = N * (N + 1) / 2;
    pairv v;
    if (!CUR || q < NP) {
        const int j = pair_hi(q), i = q - j * (j - 1) / 2;
        const double tj = j == N ? env.t_meas : tm[j];
        v = interp_pair(env.tab, env.n_grid, env.t_half, env.inv_h, tj - tm[i]);
    } else {
        const pairv c = interp_pair(env.col, env.n_grid, env.t_half, env.inv_h, tm[q - NP] - env.t_meas);
        v.gl = cnc(c.gl);
        v.gg = cnc(c.gg);
    }
    return v;
}

/* Evaluates S(u) for the `cnt` points whose vertex times (elimination order,
 * earliest first) sit in s_times; writes S to s_S[0..cnt). */
template <int N, bool CUR, bool CARRY>
__device__ void resolve_flagged(uint64_t deferred, bool flush, const Env &env, char *lds);

template <int N, bool PAIR = false, bool CUR = false, int MAP = kMapDefault, bool CARRY = false>
__device__ void keldysh_points(int cnt, const Env &env, char *lds)
{
    using Gm = Geo<N, PAIR, MAP>;
    using L = Lds<N, PAIR, CUR, false, MAP>;
    constexpr int NPS = L::NPS;
    const double *s_times = reinterpret_cast<const double *>(lds + L::times);
    cplx *s_S = reinterpret_cast<cplx *>(lds + L::S);
    pairv *s_pairs = reinterpret_cast<pairv *>(lds + L::pairs);
    const int lane = threadIdx.x;
    const int grp = lane / Gm::G, sub = lane % Gm::G;
    const int n_items = cnt * Gm::IPP;
    bool point_top_flag = false; /* paired top levels of the current point grew */
    (void)point_top_flag;
    uint64_t deferred = 0;       /* flagged points (orders <= 8), bit per point */
    (void)deferred;
    for (int base = 0; base < n_items; base += Gm::PPW) {
        const int item = base + grp;
        const bool active = item < n_items;
        const int pt = active ? item / Gm::IPP : 0;
        const int top = active ? item % Gm::IPP : 0;
        pairv *prg;
        if constexpr (Gm::IPP == 1) {
            /* one point per group: the group's lanes build its pair table;
             * the loop is unrolled so every table load is issued before the
             * first interpolation waits */
            prg = s_pairs + grp * NPS;
            const double *tm = s_times + pt * N;
            constexpr int PER = (NPS + Gm::G - 1) / Gm::G;
            pairv val[PER];
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int q = sub + k * Gm::G;
                if (q < Gm::NP) {
                    const int j = pair_hi(q), i = q - j * (j - 1) / 2;
                    const double tj = j == N ? env.t_meas : tm[j];
                    val[k] = interp_pair(env.tab, env.n_grid, env.t_half, env.inv_h, tj - tm[i]);
                } else if (CUR && q < NPS) {
                    /* the lead values of vertex q - NP, held as -conj */
                    const pairv c = interp_pair(env.col, env.n_grid, env.t_half, env.inv_h,
                                                tm[q - Gm::NP] - env.t_meas);
                    val[k].gl = cnc(c.gl);
                    val[k].gg = cnc(c.gg);
                }
            }
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int q = sub + k * Gm::G;
                if (q < NPS) prg[q] = val[k];
            }
            wave_sync();
        } else {
            /* several items share a point: PTS distinct points per round
             * (base is a multiple of IPP whenever PTS > 1); their pair
             * tables are built by the whole wave when the points change */
            constexpr int PTS = Gm::PPW >= Gm::IPP ? Gm::PPW / Gm::IPP : 1;
            prg = s_pairs + (grp / Gm::IPP) * NPS;
            if (PTS > 1 || base % Gm::IPP == 0) {
                const int first = base / Gm::IPP;
                for (int q = lane; q < PTS * NPS; q += WAVE) {
                    const int slot = q / NPS, qq = q % NPS;
                    const int p = first + slot < cnt ? first + slot : 0;
                    const double *tm = s_times + p * N;
                    if (!CUR || qq < Gm::NP) {
                        const int j = pair_hi(qq), i = qq - j * (j - 1) / 2;
                        const double tj = j == N ? env.t_meas : tm[j];
                        s_pairs[q] = interp_pair(env.tab, env.n_grid, env.t_half, env.inv_h,
                                                 tj - tm[i]);
                    } else {
                        const pairv c = interp_pair(env.col, env.n_grid, env.t_half, env.inv_h,
                                                    tm[qq - Gm::NP] - env.t_meas);
                        s_pairs[q].gl = cnc(c.gl);
                        s_pairs[q].gg = cnc(c.gg);
                    }
                }
                wave_sync();
            }
        }
        /* measurement-column entries: the lead values for the current, the
         * last row of the pair table (pairs (k, n)) for the charge */
        const pairv *mc = prg + (CUR ? Gm::NP : pidx(0, N));
        cplx prod = cmk(1.0, 0.0);
        int sgn = 0;
        BlockSrc<N, PAIR, MAP> src;
        src.c = nullptr;
        double gtop = 0.0, gbot = 0.0; /* largest elimination multipliers (paired tree) */
        if constexpr (Gm::OFF > 0) {
            cplx *s_c0 = reinterpret_cast<cplx *>(lds + L::c0) + grp * Gm::K * Gm::K;
            cplx *s_row = reinterpret_cast<cplx *>(lds + L::row) + grp * L::rows * (N + 1);
            if constexpr (PAIR)
                prod = top_block_pair<N, CUR>(prg, mc, top, sub, env.g0, s_row, s_c0, gtop);
            else if constexpr (L::RTOP)
                prod = round_top<N, CUR, MAP>(s_pairs, (base % Gm::IPP) / Gm::PPW, grp, env.g0, lds);
            else prod = top_block<N, CUR, MAP>(prg, mc, top, sub, env.g0, s_row, s_c0);
            sgn = __popc((unsigned)top) & 1;
            src.c = s_c0;
        }
        cplx s;
        if constexpr (PAIR) s = lane_sum_pair<N, CUR>(prg, mc, src, sub, prod, sgn, env.g0, gbot);
        else s = lane_sum<N, CUR, MAP>(prg, mc, src, sub, prod, sgn, env.g0);
        if constexpr (PAIR) {
            /* Points (n <= 8) or items (n > 8) whose pair steps grew beyond
             * kGrowthFlag are evaluated again with the shifted grouping
             * (lane_sum_shift, 8 lanes each, up to 8 at a time), and those it
             * flags too by the adaptive path; a point whose cooperative top
             * levels grew is redone whole after its last round.  Flags,
             * groups and results are wave-uniform. */
            constexpr double F2 = kGrowthFlag;
            constexpr uint64_t GM = Gm::G >= 64 ? ~0ull : ((1ull << Gm::G) - 1);
            constexpr bool SHIFT = Gm::K >= 5 && (Gm::OFF > 0 || N >= 4);
            const uint64_t ft = __ballot(active && gtop > F2);
            uint64_t fl = __ballot(active && (gbot > F2 || gtop > F2));
            if constexpr (Gm::OFF > 0) {
                static_assert(Gm::IPP >= Gm::PPW, "a round of the paired top holds one point");
                point_top_flag = point_top_flag || ft != 0;
                if (point_top_flag) fl = 0;
            }
            uint64_t groups = 0; /* flagged groups of the round */
            for (int g = 0; g < Gm::PPW; ++g)
                if ((fl >> (g * Gm::G)) & GM) groups |= 1ull << g;
            if constexpr (Gm::OFF == 0) {
                /* whole points: evaluated again after the batch's rounds,
                 * eight at a time (one group per point, item = point) */
                deferred |= groups << base;
                groups = 0;
            }
            while (groups) {
                /* up to 8 flagged groups, one per 8-lane slot */
                int nf = 0, mine = -1;
                uint64_t taken = 0;
                for (int k = 0; k < 8 && groups; ++k) {
                    const int g = __builtin_ctzll(groups);
                    groups &= groups - 1;
                    taken |= 1ull << g;
                    if ((lane >> 3) == k) mine = g;
                    ++nf;
                }
                (void)nf;
                cplx r = cmk(0.0, 0.0);
                double g2 = 0.0;
                if constexpr (SHIFT) {
                    /* every lane takes part in the shuffle (its source may
                     * sit in an idle slot) */
                    const cplx pm = shfl_cplx(prod, (mine >= 0 ? mine : 0) * Gm::G);
                    if (mine >= 0) {
                        const pairv *tg = Gm::OFF == 0 ? s_pairs + mine * NPS : prg;
                        const pairv *mg = Gm::OFF == 0 ? tg + (CUR ? Gm::NP : pidx(0, N)) : mc;
                        const cplx *c0g =
                            Gm::OFF == 0 ? nullptr
                                         : reinterpret_cast<const cplx *>(lds + L::c0) + mine * Gm::K * Gm::K;
                        const ShiftOut o = shift_lane<N, CUR>(
                            tg, mg, c0g, lane & 7, Gm::OFF == 0 ? 0 : (int)((base + mine) % Gm::IPP),
                            env.g0, Gm::OFF == 0 ? cmk(1.0, 0.0) : pm);
                        r = o.v;
                        g2 = o.grow;
                    }
                    /* the slot's sum over its 8 lanes */
#pragma unroll
                    for (int m = 1; m < 8; m <<= 1) {
                        r.x += shfl_xor_d(r.x, m);
                        r.y += shfl_xor_d(r.y, m);
                    }
                } else {
                    g2 = INFINITY;
                }
                const uint64_t again = __ballot(mine >= 0 && g2 > kShiftFlag);
                /* every taken group in turn: its result, from the shifted
                 * tree or, flagged again, from the adaptive path */
                uint64_t t = taken;
                int k = 0;
                while (t) {
                    const int g = __builtin_ctzll(t);
                    t &= t - 1;
                    cplx rk;
                    rk.x = __shfl(r.x, k * 8, WAVE);
                    rk.y = __shfl(r.y, k * 8, WAVE);
                    if ((again >> (k * 8)) & 0xffull) {
                        if constexpr (Gm::OFF == 0) {
                            const pairv *tg = s_pairs + g * NPS;
                            rk = adapt_point<N, CUR, L::MB>(tg, tg + (CUR ? Gm::NP : pidx(0, N)),
                                                             env.g0, lds + L::adapt, nullptr, N + 1,
                                                             0, cmk(1.0, 0.0));
                        } else {
                            const int tg = (base + g) % Gm::IPP;
                            const cplx pg = shfl_cplx(prod, g * Gm::G);
                            cplx w0 = cmul(pg, pg);
                            if (__popc((unsigned)tg) & 1) w0 = cmk(-w0.x, -w0.y);
                            const cplx *c0g =
                                reinterpret_cast<const cplx *>(lds + L::c0) + g * Gm::K * Gm::K;
                            rk = adapt_point<N, CUR, L::MB>(prg, mc, env.g0, lds + L::adapt, c0g,
                                                             Gm::K, Gm::OFF, w0);
                        }
                    }
                    if (grp == g) s = sub == 0 ? rk : cmk(0.0, 0.0);
                    ++k;
                }
            }
        }
        /* sum over the lanes of a group, then over the groups of the round
         * that share a point: they are SPAN aligned consecutive lanes, all
         * active or all idle (points hold IPP consecutive items and rounds
         * start at multiples of PPW) */
        constexpr int SPAN = Gm::G * (Gm::IPP < Gm::PPW ? Gm::IPP : Gm::PPW);
#pragma unroll
        for (int m = 1; m < SPAN; m <<= 1) {
            s.x += shfl_xor_d(s.x, m);
            s.y += shfl_xor_d(s.y, m);
        }
        if (lane % SPAN == 0 && active) {
            if constexpr (Gm::IPP == 1) s_S[pt] = s;
            else s_S[pt] = cadd(s_S[pt], s);
        }
        wave_sync();
        if constexpr (PAIR && Gm::OFF > 0) {
            /* after the point's last round: redo it whole if a top step grew */
            if ((base + Gm::PPW) % Gm::IPP == 0 && point_top_flag) {
                const int p = base / Gm::IPP;
                const cplx r = adapt_point<N, CUR, L::MB>(prg, mc, env.g0, lds + L::adapt, nullptr, N + 1, 0,
                                                           cmk(1.0, 0.0));
                if (lane == 0) s_S[p] = r;
                wave_sync();
            }
            if ((base + Gm::PPW) % Gm::IPP == 0) point_top_flag = false;
        }
    }
    if constexpr (PAIR && Gm::OFF == 0) resolve_flagged<N, CUR, CARRY>(deferred, false, env, lds);
}

/* The paired tree's flagged points (orders <= 8): re-evaluated eight at a
 * time, each on eight lanes with the shifted grouping, their tables rebuilt
 * in the adaptive path's workspace; a point flagged again is evaluated by
 * the adaptive path (its table rebuilt in the first table slot).  `deferred`
 * holds the batch's flagged points (bit per point of s_times).
 *
 * With CARRY (the tile function, not the learning pass) a pass runs only
 * when eight points are at hand: the batch's leftover flagged points move to
 * a queue in local memory (times and weights; their batch sums become zero)
 * and fill the next batch's first pass, and `flush` (the tile's end) runs
 * whatever is queued.  A queued point's result, prefactor times weight, is
 * added to the queue's sum by lane 0 in slot order; the tile adds that sum
 * once, so tile sums stay reproducible.  Without CARRY every flagged point
 * is resolved into s_S before returning.  Wave-uniform throughout. */
template <int N, bool CUR, bool CARRY>
__device__ void resolve_flagged(uint64_t deferred, bool flush, const Env &env, char *lds)
{
    using Gm = Geo<N, true>;
    using L = Lds<N, true, CUR>;
    constexpr int NPS = L::NPS;
    constexpr bool SHIFT = N >= 4;
    const int lane = threadIdx.x;
    const double *s_times = reinterpret_cast<const double *>(lds + L::times);
    const double *s_w = reinterpret_cast<const double *>(lds + L::w);
    cplx *s_S = reinterpret_cast<cplx *>(lds + L::S);
    pairv *s_pairs = reinterpret_cast<pairv *>(lds + L::pairs);
    pairv *tabs = reinterpret_cast<pairv *>(lds + L::adapt);
    double *q_times = reinterpret_cast<double *>(lds + L::dq);
    double *q_w = reinterpret_cast<double *>(lds + L::dq_w);
    cplx *q_res = reinterpret_cast<cplx *>(lds + L::dq_res);
    cplx *q_sum = reinterpret_cast<cplx *>(lds + L::dq_sum);
    int *q_n = reinterpret_cast<int *>(lds + L::dq_n);
    static_assert(8 * NPS * (int)sizeof(pairv) <= AdaptWs<N, L::MB>::bytes,
                  "eight pair tables fit in the adaptive workspace");
    int carried = CARRY ? *q_n : 0;
    for (;;) {
        const int nb = __popcll(deferred);
        if (carried + nb == 0) break;
        if (CARRY && !flush && carried + nb < 8) break;
        /* slots: the queued points first (all of them: fewer than eight),
         * then points of the batch */
        int pts[8];
        int nf = 0;
        for (int k = 0; k < 8; ++k) {
            pts[k] = -1;
            if (k < carried) {
                pts[k] = k;
                ++nf;
            } else if (deferred) {
                pts[k] = __builtin_ctzll(deferred);
                deferred &= deferred - 1;
                ++nf;
            }
        }
        const int slot = lane >> 3;
        int mine = -1;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (slot == k) mine = pts[k];
        auto times_of = [&](int k, int p) -> const double * {
            return k < carried ? q_times + p * N : s_times + p * N;
        };
        uint64_t again = 0;
        cplx r = cmk(0.0, 0.0);
        if constexpr (SHIFT) {
            for (int e = lane; e < nf * NPS; e += WAVE) {
                const int sl = e / NPS, q = e - sl * NPS;
                int p = 0;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (k == sl) p = pts[k];
                tabs[e] = pair_entry<N, CUR>(q, times_of(sl, p), env);
            }
            wave_sync();
            double g2 = 0.0;
            if (mine >= 0) {
                const pairv *tg = tabs + slot * NPS;
                const ShiftOut o = shift_lane<N, CUR>(tg, tg + (CUR ? Gm::NP : pidx(0, N)), nullptr,
                                                      lane & 7, 0, env.g0, cmk(1.0, 0.0));
                r = o.v;
                g2 = o.grow;
            }
#pragma unroll
            for (int m = 1; m < 8; m <<= 1) {
                r.x += shfl_xor_d(r.x, m);
                r.y += shfl_xor_d(r.y, m);
            }
            again = __ballot(mine >= 0 && g2 > kShiftFlag);
            if (mine >= 0 && (lane & 7) == 0 && !((again >> lane) & 0xffull)) {
                if (slot < carried) q_res[slot] = r;
                else s_S[mine] = r;
            }
            wave_sync();
        } else {
            again = __ballot(mine >= 0);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k >= nf || !((again >> (8 * k)) & 0xffull)) continue;
            const int p = pts[k];
            const double *tm = times_of(k, p);
            for (int q = lane; q < NPS; q += WAVE) s_pairs[q] = pair_entry<N, CUR>(q, tm, env);
            wave_sync();
            const cplx ra = adapt_point<N, CUR, L::MB>(
                s_pairs, s_pairs + (CUR ? Gm::NP : pidx(0, N)), env.g0, lds + L::adapt, nullptr, N + 1,
                0, cmk(1.0, 0.0));
            if (lane == 0) {
                if (k < carried) q_res[k] = ra;
                else s_S[p] = ra;
            }
            wave_sync();
        }
        if constexpr (CARRY) {
            if (carried > 0) {
                if (lane == 0) {
                    cplx acc = *q_sum;
                    for (int k = 0; k < carried; ++k) {
                        const cplx f = observable_prefactor<N, CUR>(q_res[k]);
                        acc = cadd(acc, cmk(f.x * q_w[k], f.y * q_w[k]));
                    }
                    *q_sum = acc;
                }
                wave_sync();
            }
        }
        carried = 0;
    }
    if constexpr (CARRY) {
        /* the batch's leftover flagged points join the queue */
        int k = carried;
        while (deferred) {
            const int p = __builtin_ctzll(deferred);
            deferred &= deferred - 1;
            for (int j = lane; j < N; j += WAVE) q_times[k * N + j] = s_times[p * N + j];
            if (lane == 0) {
                q_w[k] = s_w[p];
                s_S[p] = cmk(0.0, 0.0);
            }
            ++k;
        }
        if (lane == 0) *q_n = k;
        wave_sync();
    }
}

/* Inverse CDF of one coordinate's learned density (App. I): piecewise
 * constant on `bins` equal bins of [0, 1), CDF c[0..bins] at the bin edges.
 * Sets w with F(w) = x and returns the density q(w); the bin is the last b
 * with c[b] <= x (binary search, c non-decreasing, c[0] = 0 <= x < 1). */
__device__ __forceinline__ double model_inverse(const double *__restrict__ c, int bins, double x,
                                                double &w)
{
    int lo = 0, hi = bins;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (c[mid] <= x) lo = mid;
        else hi = mid;
    }
    const double c0 = c[lo], width = c[lo + 1] - c0;
    w = ((double)lo + (x - c0) / width) / (double)bins;
    return (double)bins * width;
}

/* Point idx of a tile (rank-1 lattice or Sobol'), warped: u_m = u_{m-1} -
 * v_m with v_m = -tau log(1 - x_m), after the learned second warp when
 * MODEL.  Sets u, the weight W = C / (p_n prod_j q_j) and pw = p_n prod_j q_j
 * W (the model-mode sample); on Sobol' points also steps the lane's
 * coordinate words to index idx + 64 (base: the step's first index).
 * Returns whether the point lies in the domain (u_n > 0). */
template <int N, bool MODEL, bool SOB>
__device__ __forceinline__ bool warped_point(const ItemDesc &it, uint32_t idx, const double *shift,
                                             uint32_t *word, const uint32_t *s_v, uint32_t base,
                                             double *u, double &W, double &pw)
{
    double prev = it.t_meas, p = 1.0, qm = 1.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double y;
        if constexpr (SOB) {
            y = (double)word[j] * (1.0 / 4294967296.0);
        } else {
            const uint32_t m = (idx * it.z[j]) & it.mask;
            y = (double)m * it.inv_n + shift[j];
            if (y >= 1.0) y -= 1.0;
        }
        /* learned second warp: y -> w = F_j^{-1}(y), weight / q_j(w) */
        if constexpr (MODEL)
            qm *= model_inverse(it.model_cdf + j * (it.model_bins + 1), it.model_bins, y, y);
        const double v = -it.tau * log1p(-y);
        u[j] = prev - v;
        /* the model density of the step, exp(-v / tau), is 1 - y exactly */
        p *= 1.0 - y;
        prev = u[j];
    }
    W = it.tau_n / p;
    if constexpr (MODEL) W /= qm;
    pw = p * qm * W;
    if constexpr (SOB) {
        /* next index: adding 64 flips bits 6 .. 6 + c - 1 of the base,
         * c - 1 the trailing ones of base >> 6, the same in every lane */
        const int c = __builtin_ctz(~(base >> 6)) + 1;
        for (int k = 6; k < 6 + c && k < 32; ++k) {
#pragma unroll
            for (int j = 0; j < N; ++j) word[j] ^= s_v[j * 32 + k];
        }
    }
    return u[N - 1] > 0.0;
}

/* One work tile of one order-n integral: sum of fbar over 64*c lattice
 * indices of one shift.  Returns the wave's sum (same bits in every lane).
 * MODEL: the item has a learned second warp (it.model_cdf).  SAMPLE (the
 * learning pass): also writes Re fbar of every lattice index of the tile to
 * it.sample_out. */
template <int N, bool MODEL, bool SAMPLE = false, bool PAIR = false, bool CUR = false,
          bool SOB = false, int MAP = kMapDefault>
__device__ cplx order_tile(const ItemDesc &it, int64_t tile, char *lds)
{
    using L = Lds<N, PAIR, CUR, SOB, MAP>;
    double *s_times = reinterpret_cast<double *>(lds + L::times);
    double *s_w = reinterpret_cast<double *>(lds + L::w);
    cplx *s_S = reinterpret_cast<cplx *>(lds + L::S);
    int32_t *s_ids = reinterpret_cast<int32_t *>(lds + L::ids);
    (void)s_ids;
    const int lane = threadIdx.x;
    const int s = (int)(tile / it.tiles_per_shift);
    const uint32_t i0 = (uint32_t)(tile % it.tiles_per_shift) * (uint32_t)it.tile_len;
    const double *sh = it.shifts + (int64_t)s * N;
    double shift[N];
#pragma unroll
    for (int j = 0; j < N; ++j) shift[j] = sh[j];
    Env env;
    env.tab = it.tab; env.t_half = it.t_half; env.inv_h = 1.0 / it.h; env.t_meas = it.t_meas;
    env.g0 = cmk(it.g0x, it.g0y); env.gm = cmk(it.g0x, it.g0y + it.alpha);
    env.col = it.col;
    env.n_grid = it.n_grid;
    /* Sobol' points (App. B): each lane keeps the coordinate words of its
     * index; the tile starts at a multiple of 64 and lanes step by 64, so
     * the low six index bits are the lane's and the bits that change from
     * one step to the next are the same in every lane */
    uint32_t word[SOB ? N : 1];
    uint32_t *s_v = reinterpret_cast<uint32_t *>(lds + L::sobv);
    if constexpr (SOB) {
        /* the direction numbers in local memory: every read below has one
         * address for the whole wave */
        for (int q = lane; q < N * 32; q += WAVE) s_v[q] = it.sobol[q];
        wave_sync();
        const uint32_t *ds = it.sobol + N * 32 + (int64_t)s * N;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            uint32_t w = ds[j];
#pragma unroll
            for (int k = 0; k < 6; ++k)
                if ((lane >> k) & 1) w ^= s_v[j * 32 + k];
            word[j] = w;
        }
        for (int k = 6; k < 32; ++k)
            if ((i0 >> k) & 1u) {
#pragma unroll
                for (int j = 0; j < N; ++j) word[j] ^= s_v[j * 32 + k];
            }
    }
    /* the paired tree's queue of flagged points, carried across the
     * tile's batches (not in the learning pass) */
    constexpr bool CARRY = L::CARRY && !SAMPLE;
    if constexpr (CARRY) {
        if (lane == 0) {
            *reinterpret_cast<int *>(lds + L::dq_n) = 0;
            *reinterpret_cast<cplx *>(lds + L::dq_sum) = cmk(0.0, 0.0);
        }
        wave_sync();
    }
    Kahan acc;
    if constexpr (L::QUEUE) {
        /* In-domain points queue in local memory across steps and the trees
         * run on full batches of 64 (every round of PPW points full), the
         * rest on the tile's last step: a step's own in-domain count seldom
         * fills its last round.  `queued` is wave-uniform (ballot counts). */
        int queued = 0;
        for (int c0 = 0;; c0 += WAVE) {
            const bool more = c0 < it.tile_len;
            if (!more && queued == 0) break;
            if (more) {
                const uint32_t idx = i0 + (uint32_t)c0 + (uint32_t)lane;
                double u[N], W, pw;
                const bool inside =
                    warped_point<N, MODEL, SOB>(it, idx, shift, word, s_v, i0 + (uint32_t)c0, u, W, pw);
                if (!CUR && it.mode != QQMC_MODE_CHARGE) {
                    /* the model function is the combined one, p_n prod_j q_j */
                    if (it.mode == QQMC_MODE_MODEL) acc.add(cmk(pw, 0.0));
                    else if (inside) acc.add(cmk(W, 0.0));
                    continue;
                }
                const uint64_t mask = __ballot(inside);
                const int cnt = __popcll(mask);
                if (inside) {
                    const int q = queued + lane_rank(mask);
#pragma unroll
                    for (int k = 0; k < N; ++k) s_times[q * N + k] = u[N - 1 - k];
                    s_w[q] = W;
                    s_S[q] = cmk(0.0, 0.0);
                    if constexpr (SAMPLE) s_ids[q] = (int32_t)idx;
                } else if constexpr (SAMPLE) {
                    it.sample_out[idx] = 0.0;
                }
                queued += cnt;
                wave_sync();
                /* wait for a full batch, except on the tile's last step */
                if (queued < WAVE && c0 + WAVE < it.tile_len) continue;
            }
            /* a batch of 64 queued points, or on the tile's last step the
             * rest (up to 64; what is left then goes in the next pass) */
            const int m = queued < WAVE ? queued : WAVE;
            keldysh_points<N, PAIR, CUR, MAP, CARRY>(m, env, lds);
            if (lane < m) {
                const cplx f = observable_prefactor<N, CUR>(s_S[lane]);
                const double w = s_w[lane];
                acc.add(cmk(f.x * w, f.y * w));
                if constexpr (SAMPLE) it.sample_out[s_ids[lane]] = f.x * w;
            }
            wave_sync();
            /* the points beyond the batch (fewer than 64) move to the front */
            const int left = queued - m;
            if (lane < left) {
                const int q = m + lane;
#pragma unroll
                for (int k = 0; k < N; ++k) s_times[lane * N + k] = s_times[q * N + k];
                s_w[lane] = s_w[q];
                s_S[lane] = cmk(0.0, 0.0);
                if constexpr (SAMPLE) s_ids[lane] = s_ids[q];
            }
            queued = left;
            wave_sync();
        }
    } else {
        /* every step's in-domain points at once */
        for (int c0 = 0; c0 < it.tile_len; c0 += WAVE) {
            const uint32_t idx = i0 + (uint32_t)c0 + (uint32_t)lane;
            double u[N], W, pw;
            const bool inside =
                warped_point<N, MODEL, SOB>(it, idx, shift, word, s_v, i0 + (uint32_t)c0, u, W, pw);
            if (!CUR && it.mode != QQMC_MODE_CHARGE) {
                if (it.mode == QQMC_MODE_MODEL) acc.add(cmk(pw, 0.0));
                else if (inside) acc.add(cmk(W, 0.0));
                continue;
            }
            const uint64_t mask = __ballot(inside);
            const int cnt = __popcll(mask);
            if (inside) {
                const int rk = lane_rank(mask);
#pragma unroll
                for (int k = 0; k < N; ++k) s_times[rk * N + k] = u[N - 1 - k];
                s_w[rk] = W;
                s_S[rk] = cmk(0.0, 0.0);
                if constexpr (SAMPLE) s_ids[rk] = (int32_t)idx;
            } else if constexpr (SAMPLE) {
                it.sample_out[idx] = 0.0;
            }
            wave_sync();
            keldysh_points<N, PAIR, CUR, MAP, CARRY>(cnt, env, lds);
            if (lane < cnt) {
                const cplx f = observable_prefactor<N, CUR>(s_S[lane]);
                const double w = s_w[lane];
                acc.add(cmk(f.x * w, f.y * w));
                if constexpr (SAMPLE) it.sample_out[s_ids[lane]] = f.x * w;
            }
            wave_sync();
        }
    }
    if constexpr (CARRY) {
        /* the queued flagged points: their last pass, and their sum */
        resolve_flagged<N, CUR, true>(0, true, env, lds);
        const cplx q = *reinterpret_cast<const cplx *>(lds + L::dq_sum);
        if (lane == 0 && (q.x != 0.0 || q.y != 0.0)) acc.add(q);
    }
    return wave_sum(acc.value());
}

template <int N, bool MODEL, bool PAIR, bool CUR = false, bool SOB = false>
__global__ void __launch_bounds__(WG_TREE, (Geo<N, PAIR>::WPS)) order_kernel(ItemDesc it)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    for (int64_t tile = blockIdx.x; tile < it.n_tiles; tile += gridDim.x) {
        const cplx v = order_tile<N, MODEL, false, PAIR, CUR, SOB>(it, tile, lds);
        if (threadIdx.x == 0) {
            it.tile_sums[2 * tile] = v.x;
            it.tile_sums[2 * tile + 1] = v.y;
        }
    }
}

/* Learning pass of the learned second warp (App. I): Re fbar of every
 * lattice (or Sobol') index of the item's tiles into it.sample_out
 * (exponential warp only, charge mode). */
template <int N, bool PAIR, bool SOB = false>
__global__ void __launch_bounds__(WG_TREE, (Geo<N, PAIR>::WPS)) sample_kernel(ItemDesc it)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    for (int64_t tile = blockIdx.x; tile < it.n_tiles; tile += gridDim.x)
        (void)order_tile<N, false, true, PAIR, false, SOB>(it, tile, lds);
}

/* Production-kernel evaluation at caller-given vertex times (tree method). */
template <int N, bool PAIR, bool CUR>
__global__ void __launch_bounds__(WG_TREE, (Geo<N, PAIR>::WPS)) points_tree_kernel(Env env, const double *u,
                                                              int64_t n_points, double *f)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    using L = Lds<N, PAIR, CUR>;
    double *s_times = reinterpret_cast<double *>(lds + L::times);
    cplx *s_S = reinterpret_cast<cplx *>(lds + L::S);
    const int lane = threadIdx.x;
    for (int64_t c0 = (int64_t)blockIdx.x * WAVE; c0 < n_points; c0 += (int64_t)gridDim.x * WAVE) {
        const int64_t row = c0 + lane;
        double ur[N];
        bool ok = row < n_points;
        if (ok) {
            double prev = env.t_meas;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                ur[j] = u[row * N + j];
                ok = ok && (ur[j] <= prev);
                prev = ur[j];
            }
            ok = ok && ur[N - 1] >= 0.0;
        }
        const uint64_t mask = __ballot(ok);
        const int cnt = __popcll(mask);
        const int rk = lane_rank(mask);
        if (ok) {
#pragma unroll
            for (int k = 0; k < N; ++k) s_times[rk * N + k] = ur[N - 1 - k];
            s_S[rk] = cmk(0.0, 0.0);
        }
        wave_sync();
        keldysh_points<N, PAIR, CUR>(cnt, env, lds);
        if (row < n_points) {
            cplx v = cmk(__builtin_nan(""), __builtin_nan(""));
            if (ok) v = observable_prefactor<N, CUR>(s_S[rk]);
            f[2 * row] = v.x;
            f[2 * row + 1] = v.y;
        }
        wave_sync();
    }
}

/* Persistent batched kernel for one order: resident workgroups walk a tile
 * list (tiles of many items, all of order N) that the host sorted by
 * decreasing cost, workgroup b taking entries b, b + G, b + 2G, ... (G =
 * grid size).  The loop index comes from blockIdx, so the loop is
 * wave-uniform, and every tile runs the same order_tile code as the
 * single-order kernel, so per-tile sums are the same bits.  Work of several
 * orders runs as concurrent launches of this kernel (graph branches).
 * (A work queue fed by a lane-0 atomic was tried first: the compiler
 * threaded the lane-0 branches at the top and bottom of the loop into an
 * inner cycle for lanes 1..63 that never reached the next atomic.) */
template <int N, bool PAIR, bool CUR = false, bool SOB = false, bool MODEL = false, int MAP = kMapDefault>
__global__ void __launch_bounds__(WG_TREE, (Geo<N, PAIR, MAP>::WPS)) batch_kernel(const ItemDesc *__restrict__ items,
                                                            const TileRef *__restrict__ tiles,
                                                            int64_t n_tiles)
{
    static_assert(!(CUR && MODEL), "the learned warp serves the charge");
    extern __shared__ __attribute__((aligned(16))) char lds[];
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const TileRef ref = tiles[t];
        /* by reference: fields are loaded where they are used (scalar
         * loads), which keeps the descriptor out of the registers the tree
         * needs */
        const ItemDesc &it = items[ref.item];
        const cplx v = order_tile<N, MODEL, false, PAIR, CUR, SOB, MAP>(it, ref.tile, lds);
        if (threadIdx.x == 0) {
            it.tile_sums[2 * ref.tile] = v.x;
            it.tile_sums[2 * ref.tile + 1] = v.y;
        }
    }
}

template <template <int> class F, typename... A>
hipError_t dispatch(int order, A... args)
{
    switch (order) {
    case 1: return F<1>::run(args...);
    case 2: return F<2>::run(args...);
    case 3: return F<3>::run(args...);
    case 4: return F<4>::run(args...);
    case 5: return F<5>::run(args...);
    case 6: return F<6>::run(args...);
    case 7: return F<7>::run(args...);
    case 8: return F<8>::run(args...);
    case 9: return F<9>::run(args...);
    case 10: return F<10>::run(args...);
    case 11: return F<11>::run(args...);
    case 12: return F<12>::run(args...);
    case 13: return F<13>::run(args...);
    case 14: return F<14>::run(args...);
    default: return hipErrorInvalidValue;
    }
}


template <int N, bool MODEL, bool PAIR, bool CUR, bool SOB>
hipError_t go_order(const ItemDesc &it, hipStream_t s)
{
    const int64_t blocks = it.n_tiles < 1048576 ? it.n_tiles : 1048576;
    hipLaunchKernelGGL((order_kernel<N, MODEL, PAIR, CUR, SOB>), dim3((unsigned)blocks), dim3(WG_TREE),
                       (Lds<N, PAIR, CUR, SOB>::bytes), s, it);
    return hipGetLastError();
}

template <int N, bool PAIR, bool SOB = false>
hipError_t go_sample(const ItemDesc &it, hipStream_t s)
{
    const int64_t blocks = it.n_tiles < 1048576 ? it.n_tiles : 1048576;
    hipLaunchKernelGGL((sample_kernel<N, PAIR, SOB>), dim3((unsigned)blocks), dim3(WG_TREE),
                       (Lds<N, PAIR, false, SOB>::bytes), s, it);
    return hipGetLastError();
}

template <int N, bool PAIR, bool CUR>
hipError_t go_points_tree(Env env, const double *u, int64_t n_points, double *f, hipStream_t s)
{
    int64_t blocks = (n_points + WAVE - 1) / WAVE;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((points_tree_kernel<N, PAIR, CUR>), dim3((unsigned)blocks), dim3(WG_TREE),
                       (Lds<N, PAIR, CUR>::bytes), s, env, u, n_points, f);
    return hipGetLastError();
}

template <int N, bool PAIR, bool CUR = false, bool SOB = false, bool MODEL = false, int MAP = kMapDefault>
hipError_t go_batch(const ItemDesc *items_dev, const TileRef *tiles_dev, int64_t n_tiles,
                    int32_t grid_blocks, hipStream_t s)
{
    const int64_t g = grid_blocks < n_tiles ? grid_blocks : n_tiles;
    hipLaunchKernelGGL((batch_kernel<N, PAIR, CUR, SOB, MODEL, MAP>), dim3((unsigned)g), dim3(WG_TREE),
                       (Lds<N, PAIR, CUR, SOB, MAP>::bytes), s, items_dev, tiles_dev, n_tiles);
    return hipGetLastError();
}

template <int N, bool PAIR, bool CUR = false, bool SOB = false, bool MODEL = false, int MAP = kMapDefault>
int32_t occ_batch()
{
    int blocks = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &blocks, batch_kernel<N, PAIR, CUR, SOB, MODEL, MAP>, 64,
        (size_t)Lds<N, PAIR, CUR, SOB, MAP>::bytes);
    return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

inline Env make_env(const double *tab, const double *col, int32_t n_grid, double t_half, double h,
             double n_sigma, double alpha, double t_meas)
{
    Env e;
    e.tab = tab; e.n_grid = n_grid; e.t_half = t_half; e.inv_h = 1.0 / h; e.t_meas = t_meas;
    e.col = col;
    e.g0 = cmk(0.0, n_sigma - alpha);
    e.gm = cmk(0.0, n_sigma);
    return e;
}

} // namespace

/* Variant units.  qqmc_kernels_pair.hip: the paired tree (needs_pair) for
 * the charge on the lattice; qqmc_kernels_cur.hip: the current on the
 * lattice (both trees); qqmc_kernels_sob.hip: Sobol' points (both trees,
 * charge or current). */
hipError_t launch_order_pair(const ItemDesc &it, hipStream_t s);
hipError_t launch_sample_pair(const ItemDesc &it, hipStream_t s);
hipError_t launch_points_tree_pair(const double *tab, int32_t n_grid, double t_half, double h,
                                   double n_sigma, double alpha, int32_t order, double t_meas,
                                   const double *u, int64_t n_points, double *f, hipStream_t s);
hipError_t launch_batch_pair(int32_t order, const ItemDesc *items_dev, const TileRef *tiles_dev,
                             int64_t n_tiles, int32_t grid_blocks, hipStream_t s);
int32_t batch_blocks_per_cu_pair(int32_t order);
hipError_t launch_order_current(const ItemDesc &it, hipStream_t s);
hipError_t launch_batch_current(int32_t order, bool pair, const ItemDesc *items_dev,
                                const TileRef *tiles_dev, int64_t n_tiles, int32_t grid_blocks,
                                hipStream_t s);
int32_t batch_blocks_per_cu_current(int32_t order, bool pair);
hipError_t launch_points_tree_current(const double *tab, const double *col, int32_t n_grid,
                                      double t_half, double h, double n_sigma, double alpha,
                                      int32_t order, double t_meas, const double *u,
                                      int64_t n_points, double *f, hipStream_t s);
hipError_t launch_order_sobol(const ItemDesc &it, hipStream_t s);
hipError_t launch_order_sobol_model(const ItemDesc &it, hipStream_t s);
hipError_t launch_sample_sobol(const ItemDesc &it, hipStream_t s);
hipError_t launch_batch_sobol(int32_t order, bool pair, bool current, const ItemDesc *items_dev,
                              const TileRef *tiles_dev, int64_t n_tiles, int32_t grid_blocks,
                              hipStream_t s);
int32_t batch_blocks_per_cu_sobol(int32_t order, bool pair, bool current);
hipError_t launch_batch_sobol_charge(int32_t order, bool pair, const ItemDesc *items_dev,
                                     const TileRef *tiles_dev, int64_t n_tiles,
                                     int32_t grid_blocks, hipStream_t s);
int32_t batch_blocks_per_cu_sobol_charge(int32_t order, bool pair);
hipError_t launch_batch_model(int32_t order, bool pair, bool sobol, const ItemDesc *items_dev,
                              const TileRef *tiles_dev, int64_t n_tiles, int32_t grid_blocks,
                              hipStream_t s);
int32_t batch_blocks_per_cu_model(int32_t order, bool pair, bool sobol);

} // namespace qqmc

#endif
