/*
 * qqmc_kernels_sob.hip -- Sobol' points (App. B; coordinate words stepped by
 * the direction numbers of the changing index bits) for the charge and the
 * current, both elimination trees, and the batched current on Sobol' points
 * (the learned warp over Sobol' points is in qqmc_kernels_sob_model.hip, the
 * batched charge on them in qqmc_kernels_sob_batch.hip).
 */
#include "qqmc_kernels.h"

namespace qqmc {

namespace {

template <int N> struct OrderSob {
    static hipError_t run(const ItemDesc &it, hipStream_t s)
    {
        const bool pair = needs_pair(it.g0y), cur = it.mode == QQMC_MODE_CURRENT;
        if (cur)
            return pair ? go_order<N, false, true, true, true>(it, s)
                        : go_order<N, false, false, true, true>(it, s);
        return pair ? go_order<N, false, true, false, true>(it, s)
                    : go_order<N, false, false, false, true>(it, s);
    }
};

template <int N> struct BatchSobCur {
    static hipError_t run(bool pair, const ItemDesc *items_dev, const TileRef *tiles_dev,
                          int64_t n_tiles, int32_t grid_blocks, hipStream_t s)
    {
        return pair ? go_batch<N, true, true, true>(items_dev, tiles_dev, n_tiles, grid_blocks, s)
                    : go_batch<N, false, true, true>(items_dev, tiles_dev, n_tiles, grid_blocks, s);
    }
};

template <int N> struct OccSobCur {
    static hipError_t run(bool pair, int32_t *out)
    {
        *out = pair ? occ_batch<N, true, true, true>() : occ_batch<N, false, true, true>();
        return hipSuccess;
    }
};

} // namespace

/* Batched Sobol' tiles: the current here, the charge (with or without a
 * learned warp) in its own unit. */
hipError_t launch_batch_sobol(int32_t order, bool pair, bool current, const ItemDesc *items_dev,
                              const TileRef *tiles_dev, int64_t n_tiles, int32_t grid_blocks,
                              hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    if (!current)
        return launch_batch_sobol_charge(order, pair, items_dev, tiles_dev, n_tiles, grid_blocks, s);
    return dispatch<BatchSobCur>(order, pair, items_dev, tiles_dev, n_tiles, grid_blocks, s);
}

int32_t batch_blocks_per_cu_sobol(int32_t order, bool pair, bool current)
{
    if (!current) return batch_blocks_per_cu_sobol_charge(order, pair);
    int32_t b = 1;
    if (dispatch<OccSobCur>(order, pair, &b) != hipSuccess) return 1;
    return b;
}

hipError_t launch_order_sobol(const ItemDesc &it, hipStream_t s)
{
    return dispatch<OrderSob>(it.order, it, s);
}

} // namespace qqmc
