/*
 * qqmc_kernels_cur.hip -- the current into a lead (the lead site in the
 * measurement column) on the lattice, both elimination trees: order, points
 * and batched (plans, server) launches.
 */
#include "qqmc_kernels.h"

namespace qqmc {

namespace {

template <int N> struct OrderCur {
    static hipError_t run(const ItemDesc &it, hipStream_t s)
    {
        return needs_pair(it.g0y) ? go_order<N, false, true, true, false>(it, s)
                               : go_order<N, false, false, true, false>(it, s);
    }
};

template <int N> struct PointsCur {
    static hipError_t run(Env env, bool pair, const double *u, int64_t n_points, double *f,
                          hipStream_t s)
    {
        return pair ? go_points_tree<N, true, true>(env, u, n_points, f, s)
                    : go_points_tree<N, false, true>(env, u, n_points, f, s);
    }
};

template <int N> struct BatchCur {
    static hipError_t run(bool pair, const ItemDesc *items_dev, const TileRef *tiles_dev,
                          int64_t n_tiles, int32_t grid_blocks, hipStream_t s)
    {
        return pair ? go_batch<N, true, true>(items_dev, tiles_dev, n_tiles, grid_blocks, s)
                    : go_batch<N, false, true>(items_dev, tiles_dev, n_tiles, grid_blocks, s);
    }
};

template <int N> struct OccCur {
    static hipError_t run(bool pair, int32_t *out)
    {
        *out = pair ? occ_batch<N, true, true>() : occ_batch<N, false, true>();
        return hipSuccess;
    }
};

} // namespace

hipError_t launch_batch_current(int32_t order, bool pair, const ItemDesc *items_dev,
                                const TileRef *tiles_dev, int64_t n_tiles, int32_t grid_blocks,
                                hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    return dispatch<BatchCur>(order, pair, items_dev, tiles_dev, n_tiles, grid_blocks, s);
}

int32_t batch_blocks_per_cu_current(int32_t order, bool pair)
{
    int32_t b = 1;
    if (dispatch<OccCur>(order, pair, &b) != hipSuccess) return 1;
    return b;
}

hipError_t launch_order_current(const ItemDesc &it, hipStream_t s)
{
    return dispatch<OrderCur>(it.order, it, s);
}

hipError_t launch_points_tree_current(const double *tab, const double *col, int32_t n_grid,
                                      double t_half, double h, double n_sigma, double alpha,
                                      int32_t order, double t_meas, const double *u,
                                      int64_t n_points, double *f, hipStream_t s)
{
    return dispatch<PointsCur>(order,
                               make_env(tab, col, n_grid, t_half, h, n_sigma, alpha, t_meas),
                               needs_pair(n_sigma - alpha), u, n_points, f, s);
}

} // namespace qqmc
