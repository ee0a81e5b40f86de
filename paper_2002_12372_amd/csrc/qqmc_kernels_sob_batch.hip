/*
 * qqmc_kernels_sob_batch.hip -- the batched charge on Sobol' points (App. B)
 * for plans and the server, both elimination trees; each tile takes the
 * learned second warp (App. I) or not, as its item says.
 */
#include "qqmc_kernels.h"

namespace qqmc {

namespace {

template <int N> struct BatchSobCharge {
    static hipError_t run(bool pair, const ItemDesc *items_dev, const TileRef *tiles_dev,
                          int64_t n_tiles, int32_t grid_blocks, hipStream_t s)
    {
        return pair ? go_batch<N, true, false, true>(items_dev, tiles_dev, n_tiles, grid_blocks, s)
                    : go_batch<N, false, false, true>(items_dev, tiles_dev, n_tiles, grid_blocks, s);
    }
};

template <int N> struct OccSobCharge {
    static hipError_t run(bool pair, int32_t *out)
    {
        *out = pair ? occ_batch<N, true, false, true>() : occ_batch<N, false, false, true>();
        return hipSuccess;
    }
};

} // namespace

hipError_t launch_batch_sobol_charge(int32_t order, bool pair, const ItemDesc *items_dev,
                                     const TileRef *tiles_dev, int64_t n_tiles,
                                     int32_t grid_blocks, hipStream_t s)
{
    return dispatch<BatchSobCharge>(order, pair, items_dev, tiles_dev, n_tiles, grid_blocks, s);
}

int32_t batch_blocks_per_cu_sobol_charge(int32_t order, bool pair)
{
    int32_t b = 1;
    if (dispatch<OccSobCharge>(order, pair, &b) != hipSuccess) return 1;
    return b;
}

} // namespace qqmc
