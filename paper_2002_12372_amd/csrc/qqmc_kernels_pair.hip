/*
 * qqmc_kernels_pair.hip -- the paired elimination tree (2x2 block pivots,
 * for a vertex diagonal near zero; qqmc_tree.h) for the charge on the
 * lattice: order, learning pass, points and batched launches.
 */
#include "qqmc_kernels.h"

namespace qqmc {

namespace {

template <int N> struct OrderPair {
    static hipError_t run(const ItemDesc &it, hipStream_t s)
    {
        return it.model_cdf ? go_order<N, true, true, false, false>(it, s)
                            : go_order<N, false, true, false, false>(it, s);
    }
};

template <int N> struct SamplePair {
    static hipError_t run(const ItemDesc &it, hipStream_t s) { return go_sample<N, true>(it, s); }
};

template <int N> struct PointsPair {
    static hipError_t run(Env env, const double *u, int64_t n_points, double *f, hipStream_t s)
    {
        return go_points_tree<N, true, false>(env, u, n_points, f, s);
    }
};

template <int N> struct BatchPair {
    static hipError_t run(const ItemDesc *items_dev, const TileRef *tiles_dev, int64_t n_tiles,
                          int32_t grid_blocks, hipStream_t s)
    {
        return go_batch<N, true>(items_dev, tiles_dev, n_tiles, grid_blocks, s);
    }
};

template <int N> struct OccPair {
    static hipError_t run(int32_t *out)
    {
        *out = occ_batch<N, true>();
        return hipSuccess;
    }
};

} // namespace

hipError_t launch_order_pair(const ItemDesc &it, hipStream_t s)
{
    return dispatch<OrderPair>(it.order, it, s);
}

hipError_t launch_sample_pair(const ItemDesc &it, hipStream_t s)
{
    return dispatch<SamplePair>(it.order, it, s);
}

hipError_t launch_points_tree_pair(const double *tab, int32_t n_grid, double t_half, double h,
                                   double n_sigma, double alpha, int32_t order, double t_meas,
                                   const double *u, int64_t n_points, double *f, hipStream_t s)
{
    return dispatch<PointsPair>(order,
                                make_env(tab, nullptr, n_grid, t_half, h, n_sigma, alpha, t_meas),
                                u, n_points, f, s);
}

hipError_t launch_batch_pair(int32_t order, const ItemDesc *items_dev, const TileRef *tiles_dev,
                             int64_t n_tiles, int32_t grid_blocks, hipStream_t s)
{
    return dispatch<BatchPair>(order, items_dev, tiles_dev, n_tiles, grid_blocks, s);
}

int32_t batch_blocks_per_cu_pair(int32_t order)
{
    int32_t b = 1;
    if (dispatch<OccPair>(order, &b) != hipSuccess) return 1;
    return b;
}

} // namespace qqmc
