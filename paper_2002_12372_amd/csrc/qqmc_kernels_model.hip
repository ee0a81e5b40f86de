/*
 * qqmc_kernels_model.hip -- batched kernels for items with a learned second
 * warp (App. I): the charge on the lattice or on Sobol' points, both
 * elimination trees.  They are separate kernels (a kernel key of their own)
 * so that the batched kernels of the exponential warp carry only that warp.
 */
#include "qqmc_kernels.h"

namespace qqmc {

namespace {

template <int N> struct BatchModel {
    static hipError_t run(bool pair, bool sobol, const ItemDesc *items_dev,
                          const TileRef *tiles_dev, int64_t n_tiles, int32_t grid_blocks,
                          hipStream_t s)
    {
        if (sobol)
            return pair ? go_batch<N, true, false, true, true>(items_dev, tiles_dev, n_tiles,
                                                               grid_blocks, s)
                        : go_batch<N, false, false, true, true>(items_dev, tiles_dev, n_tiles,
                                                                grid_blocks, s);
        return pair ? go_batch<N, true, false, false, true>(items_dev, tiles_dev, n_tiles,
                                                            grid_blocks, s)
                    : go_batch<N, false, false, false, true>(items_dev, tiles_dev, n_tiles,
                                                             grid_blocks, s);
    }
};

template <int N> struct OccModel {
    static hipError_t run(bool pair, bool sobol, int32_t *out)
    {
        *out = sobol ? (pair ? occ_batch<N, true, false, true, true>()
                             : occ_batch<N, false, false, true, true>())
                     : (pair ? occ_batch<N, true, false, false, true>()
                             : occ_batch<N, false, false, false, true>());
        return hipSuccess;
    }
};

} // namespace

hipError_t launch_batch_model(int32_t order, bool pair, bool sobol, const ItemDesc *items_dev,
                              const TileRef *tiles_dev, int64_t n_tiles, int32_t grid_blocks,
                              hipStream_t s)
{
    return dispatch<BatchModel>(order, pair, sobol, items_dev, tiles_dev, n_tiles, grid_blocks,
                                s);
}

int32_t batch_blocks_per_cu_model(int32_t order, bool pair, bool sobol)
{
    int32_t b = 1;
    return dispatch<OccModel>(order, pair, sobol, &b) == hipSuccess ? b : 1;
}

} // namespace qqmc
