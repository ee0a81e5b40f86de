/*
 * qqmc_kernels.hip -- gfx950 kernels of the QQMC hot path (arXiv:2002.12372):
 * the scalar elimination tree for the charge on the lattice, the per-shift
 * reduction, the direct method, the table build, and the routing of every
 * launch to its variant unit (device templates in qqmc_kernels.h).
 *
 * Work decomposition: qqmc_kernels.h (the five steps per 64 lattice
 * indices, the lane mapping, the register budget).
 * The tile's sum goes to one slot of a partials array; a second kernel sums
 * the slots of each shift in a fixed order.  No floating-point atomics are
 * used anywhere, so results are bitwise reproducible.
 */
#include "qqmc_kernels.h"

namespace qqmc {

namespace {

/* Per-shift sums of the tile partials, fixed order: thread j adds tiles
 * j, j+256, ... (compensated), then a fixed tree over the 256 threads. */
__global__ void __launch_bounds__(256) shift_reduce_kernel(const ItemDesc *items,
                                                           const int64_t *shift_base,
                                                           double *shift_sums)
{
    __shared__ double sx[256], sy[256];
    const int item = blockIdx.y;
    const ItemDesc &it = items[item];
    const int s = blockIdx.x;
    if (s >= it.n_shifts) return;
    Kahan acc;
    const int64_t t0 = (int64_t)s * it.tiles_per_shift;
    for (int64_t t = threadIdx.x; t < it.tiles_per_shift; t += 256)
        acc.add(cmk(it.tile_sums[2 * (t0 + t)], it.tile_sums[2 * (t0 + t) + 1]));
    const cplx v = acc.value();
    sx[threadIdx.x] = v.x;
    sy[threadIdx.x] = v.y;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sx[threadIdx.x] += sx[threadIdx.x + w];
            sy[threadIdx.x] += sy[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t o = shift_base[item] + s;
        shift_sums[2 * o] = sx[0];
        shift_sums[2 * o + 1] = sy[0];
    }
}

/* Direct enumeration (no shared elimination): for every index vector a,
 * build the (n+1) x (n+1) Wick matrix in the paper's order (measurement
 * first) from the 2x2 Keldysh rule with the actual time differences, and
 * factorise it and its vertex block with partial pivoting.  One workgroup
 * per point, index vectors spread over the 64 lanes. */
template <int M>
__device__ cplx det_pivoted(cplx (&a)[M][M], int m)
{
    cplx det = cmk(1.0, 0.0);
    for (int k = 0; k < m; ++k) {
        int piv = k;
        double best = hypot(a[k][k].x, a[k][k].y);
        for (int r = k + 1; r < m; ++r) {
            const double v = hypot(a[r][k].x, a[r][k].y);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return cmk(0.0, 0.0);
        if (piv != k) {
            for (int c = 0; c < m; ++c) {
                const cplx t = a[k][c];
                a[k][c] = a[piv][c];
                a[piv][c] = t;
            }
            det = cmk(-det.x, -det.y);
        }
        const cplx p = a[k][k];
        det = cmul(det, p);
        const cplx rp = crecip(p);
        for (int r = k + 1; r < m; ++r) {
            const cplx fct = cmul(a[r][k], rp);
            for (int c = k + 1; c < m; ++c) a[r][c] = cfms(fct, a[k][c], a[r][c]);
        }
    }
    return det;
}

template <int N>
__global__ void __launch_bounds__(64) points_direct_kernel(Env env, const double *u,
                                                          int64_t n_points, double *f,
                                                          double *mass)
{
    constexpr int NP1 = N + 1;
    __shared__ pairv s_g[NP1 * NP1];
    __shared__ double s_tm[NP1];
    __shared__ double sx[WAVE], sy[WAVE], sm[WAVE];
    const int lane = threadIdx.x;
    for (int64_t pt = blockIdx.x; pt < n_points; pt += gridDim.x) {
        if (lane == 0) s_tm[0] = env.t_meas;
        if (lane < N) s_tm[lane + 1] = u[pt * N + lane];
        __syncthreads();
        for (int q = lane; q < NP1 * NP1; q += WAVE) {
            const int r = q / NP1, c = q % NP1;
            /* the current's measurement column is the lead site */
            const double *tab = (c == 0 && env.col) ? env.col : env.tab;
            s_g[q] = interp_pair(tab, env.n_grid, env.t_half, env.inv_h, s_tm[r] - s_tm[c]);
        }
        __syncthreads();
        Kahan acc, acc_m;
        for (int a = lane; a < (1 << N); a += WAVE) {
            cplx up[NP1][NP1], dn[NP1][NP1];
            for (int r = 0; r < NP1; ++r) {
                for (int c = 0; c < NP1; ++c) {
                    cplx v;
                    if (r == c) {
                        v = r == 0 ? (env.col ? s_g[0].gl : env.gm) : env.g0;
                    } else {
                        const int al = r == 0 ? 0 : (a >> (r - 1)) & 1;
                        const int be = c == 0 ? 1 : (a >> (c - 1)) & 1;
                        const double d = s_tm[r] - s_tm[c];
                        const pairv g = s_g[r * NP1 + c];
                        if (al == 0 && be == 0) v = d > 0.0 ? g.gg : g.gl;
                        else if (al == 0) v = g.gl;
                        else if (be == 0) v = g.gg;
                        else v = d > 0.0 ? g.gl : g.gg;
                    }
                    up[r][c] = v;
                    if (r > 0 && c > 0) dn[r - 1][c - 1] = v;
                }
            }
            const cplx du = det_pivoted<NP1>(up, NP1);
            const cplx dd = det_pivoted<NP1>(dn, N);
            cplx term = cmul(du, dd);
            /* term mass: |det_up det_dn| of every index vector */
            acc_m.add(cmk(sqrt(term.x * term.x + term.y * term.y), 0.0));
            if (__popc((unsigned)a) & 1) term = cmk(-term.x, -term.y);
            acc.add(term);
        }
        const cplx v = acc.value();
        sx[lane] = v.x;
        sy[lane] = v.y;
        sm[lane] = acc_m.value().x;
        __syncthreads();
        for (int w = WAVE / 2; w > 0; w >>= 1) {
            if (lane < w) {
                sx[lane] += sx[lane + w];
                sy[lane] += sy[lane + w];
                sm[lane] += sm[lane + w];
            }
            __syncthreads();
        }
        if (lane == 0) {
            const cplx out = env.col ? observable_prefactor<N, true>(cmk(sx[0], sy[0]))
                                     : charge_prefactor<N>(cmk(sx[0], sy[0]));
            f[2 * pt] = out.x;
            f[2 * pt + 1] = out.y;
            /* on the scale of f: |prefactor| sum_a |det_up det_dn| */
            if (mass) mass[pt] = (env.col ? 4.0 : 2.0) * sm[0];
        }
        __syncthreads();
    }
}

/* Device build of the Green's-function grid: one workgroup per node; the
 * 256 threads split the Matsubara terms of g^<(|tau|) (thread j takes
 * k = kmax - j, kmax - j - 256, ..., compensated), a fixed tree combines
 * them, and thread 0 assembles the node (qqmc_gf.h). */
__global__ void __launch_bounds__(256) tables_kernel(double *tab, int32_t n_grid, double t_half,
                                                     double h, double eps_d, double gamma,
                                                     double beta, double bias_v, double n_sigma)
{
    __shared__ double red[4][256];
    const int j = blockIdx.x;
    const double tau = -t_half + j * h;
    const double at = fabs(tau);
    const int tid = threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0}, comp[4] = {0.0, 0.0, 0.0, 0.0};
    if (tau != 0.0) {
        const long kmax = matsubara_kmax(beta, at);
        for (long k = kmax - tid; k >= 0; k -= 256) {
            const cplx tp = matsubara_term(eps_d, gamma, beta, 0.5 * bias_v, at, k);
            const cplx tm = matsubara_term(eps_d, gamma, beta, -0.5 * bias_v, at, k);
            const double v[4] = {tp.x, tp.y, tm.x, tm.y};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double y = v[c] - comp[c], t = acc[c] + y;
                comp[c] = (t - acc[c]) - y;
                acc[c] = t;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) red[c][tid] = acc[c] - comp[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
#pragma unroll
            for (int c = 0; c < 4; ++c) red[c][tid] += red[c][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        cplx gl_abs = cmk(0.0, 0.0);
        if (tau != 0.0)
            gl_abs = lesser_from_sums(eps_d, gamma, beta, bias_v, at, cmk(red[0][0], red[1][0]),
                                      cmk(red[2][0], red[3][0]));
        const pairv v = node_values(eps_d, gamma, tau, gl_abs, n_sigma);
        tab[4 * j + 0] = v.gl.x;
        tab[4 * j + 1] = v.gl.y;
        tab[4 * j + 2] = v.gg.x;
        tab[4 * j + 3] = v.gg.y;
    }
}

template <int N> struct OrderScalar {
    static hipError_t run(const ItemDesc &it, hipStream_t s)
    {
        return it.model_cdf ? go_order<N, true, false, false, false>(it, s)
                            : go_order<N, false, false, false, false>(it, s);
    }
};

template <int N> struct SampleScalar {
    static hipError_t run(const ItemDesc &it, hipStream_t s) { return go_sample<N, false>(it, s); }
};

template <int N> struct PointsScalar {
    static hipError_t run(Env env, const double *u, int64_t n_points, double *f, hipStream_t s)
    {
        return go_points_tree<N, false, false>(env, u, n_points, f, s);
    }
};

template <int N> struct DirectPointsLaunch {
    static hipError_t run(Env env, const double *u, int64_t n_points, double *f, double *mass,
                          hipStream_t s)
    {
        int64_t blocks = n_points < 65536 ? n_points : 65536;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(points_direct_kernel<N>, dim3((unsigned)blocks), dim3(64), 0, s,
                           env, u, n_points, f, mass);
        return hipGetLastError();
    }
};

template <int N> struct BatchScalar {
    static hipError_t run(const ItemDesc *items_dev, const TileRef *tiles_dev, int64_t n_tiles,
                          int32_t grid_blocks, hipStream_t s)
    {
        return go_batch<N, false>(items_dev, tiles_dev, n_tiles, grid_blocks, s);
    }
};

template <int N> struct OccScalar {
    static hipError_t run(int32_t *out)
    {
        *out = occ_batch<N, false>();
        return hipSuccess;
    }
};

} // namespace

hipError_t launch_tables(double *tab, int32_t n_grid, double t_half, double eps_d, double gamma,
                         double beta, double bias_v, double n_sigma, hipStream_t s)
{
    const double h = 2.0 * t_half / (n_grid - 1);
    hipLaunchKernelGGL(tables_kernel, dim3((unsigned)n_grid), dim3(256), 0, s, tab, n_grid, t_half,
                       h, eps_d, gamma, beta, bias_v, n_sigma);
    return hipGetLastError();
}

/* Sobol' points (with or without a learned warp), the current, the paired
 * tree (a vertex diagonal near zero, needs_pair), else the scalar tree. */
hipError_t launch_order(const ItemDesc &it, hipStream_t s)
{
    if (it.sobol) return it.model_cdf ? launch_order_sobol_model(it, s) : launch_order_sobol(it, s);
    if (it.mode == QQMC_MODE_CURRENT) return launch_order_current(it, s);
    if (needs_pair(it.g0y)) return launch_order_pair(it, s);
    return dispatch<OrderScalar>(it.order, it, s);
}

hipError_t launch_sample(const ItemDesc &it, hipStream_t s)
{
    if (it.sobol) return launch_sample_sobol(it, s);
    if (needs_pair(it.g0y)) return launch_sample_pair(it, s);
    return dispatch<SampleScalar>(it.order, it, s);
}

hipError_t launch_shift_reduce(const ItemDesc *items_dev, int32_t n_items,
                               const int64_t *shift_base_dev, double *shift_sums,
                               int32_t max_shifts, hipStream_t s)
{
    hipLaunchKernelGGL(shift_reduce_kernel, dim3((unsigned)max_shifts, (unsigned)n_items),
                       dim3(256), 0, s, items_dev, shift_base_dev, shift_sums);
    return hipGetLastError();
}

hipError_t launch_points_tree(const double *tab, const double *col, int32_t n_grid,
                              double t_half, double h, double n_sigma, double alpha,
                              int32_t order, double t_meas, const double *u, int64_t n_points,
                              double *f, hipStream_t s)
{
    if (n_points <= 0) return hipSuccess;
    if (col)
        return launch_points_tree_current(tab, col, n_grid, t_half, h, n_sigma, alpha, order,
                                          t_meas, u, n_points, f, s);
    if (needs_pair(n_sigma - alpha))
        return launch_points_tree_pair(tab, n_grid, t_half, h, n_sigma, alpha, order, t_meas, u,
                                       n_points, f, s);
    return dispatch<PointsScalar>(order,
                                  make_env(tab, nullptr, n_grid, t_half, h, n_sigma, alpha, t_meas),
                                  u, n_points, f, s);
}

hipError_t launch_points_direct(const double *tab, const double *col, int32_t n_grid,
                                double t_half, double h, double n_sigma, double alpha,
                                int32_t order, double t_meas, const double *u, int64_t n_points,
                                double *f, double *mass, hipStream_t s)
{
    if (n_points <= 0) return hipSuccess;
    return dispatch<DirectPointsLaunch>(order,
                                        make_env(tab, col, n_grid, t_half, h, n_sigma, alpha, t_meas),
                                        u, n_points, f, mass, s);
}

hipError_t launch_batch(int32_t key, const ItemDesc *items_dev, const TileRef *tiles_dev,
                        int64_t n_tiles, int32_t grid_blocks, hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    if (key_model(key))
        return launch_batch_model(key_order(key), key_pair(key), key_sobol(key), items_dev,
                                  tiles_dev, n_tiles, grid_blocks, s);
    if (key_sobol(key))
        return launch_batch_sobol(key_order(key), key_pair(key), key_current(key), items_dev,
                                  tiles_dev, n_tiles, grid_blocks, s);
    if (key_current(key))
        return launch_batch_current(key_order(key), key_pair(key), items_dev, tiles_dev, n_tiles,
                                    grid_blocks, s);
    if (key_pair(key))
        return launch_batch_pair(key_order(key), items_dev, tiles_dev, n_tiles, grid_blocks, s);
    return dispatch<BatchScalar>(key_order(key), items_dev, tiles_dev, n_tiles, grid_blocks, s);
}

int32_t batch_blocks_per_cu(int32_t key)
{
    if (key_model(key))
        return batch_blocks_per_cu_model(key_order(key), key_pair(key), key_sobol(key));
    if (key_sobol(key))
        return batch_blocks_per_cu_sobol(key_order(key), key_pair(key), key_current(key));
    if (key_current(key)) return batch_blocks_per_cu_current(key_order(key), key_pair(key));
    if (key_pair(key)) return batch_blocks_per_cu_pair(key_order(key));
    int32_t b = 1;
    if (dispatch<OccScalar>(key_order(key), &b) != hipSuccess) return 1;
    return b;
}

} // namespace qqmc
