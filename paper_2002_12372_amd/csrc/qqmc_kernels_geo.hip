/*
 * qqmc_kernels_geo.hip -- the second lane mapping of the scalar-tree charge
 * kernels on the lattice, for the batched plan's autotuner.  Orders 7, 8 and
 * 11-14: a depth-4 register tree (each lane starts from a 5 x 5 trailing
 * block, so twice the lanes share an item: 16 per point at order 8 instead
 * of 8), compiled for two waves per SIMD.  Orders 5 and 6, whose default is
 * the depth-4 tree: the depth-5 tree (half the lanes per point, one wave per
 * SIMD).  Orders 9 and 10: the first n - 8 levels eliminated cooperatively
 * by the 8 lanes of each top-level index prefix, each lane then starting
 * from the prefix's 9 x 9 block (the default there is the flat mapping,
 * 2^(n-5) lanes per point each walking its path from the full matrix).
 * Orders 1-4 have a single mapping (one lane walks the whole tree either
 * way).
 */
#include "qqmc_kernels.h"

namespace qqmc {

namespace {

template <int N> constexpr int alt_map()
{
    return (N == 9 || N == 10) ? kMapTop : (N == 5 || N == 6) ? kMapDepth5 : kMapDepth4;
}

template <int N> struct BatchAlt {
    static hipError_t run(const ItemDesc *items_dev, const TileRef *tiles_dev, int64_t n_tiles,
                          int32_t grid_blocks, hipStream_t s)
    {
        if constexpr (N < 5) return hipErrorInvalidValue;
        else
            return go_batch<N, false, false, false, false, alt_map<N>()>(items_dev, tiles_dev,
                                                                         n_tiles, grid_blocks, s);
    }
};

template <int N> struct OccAlt {
    static hipError_t run(int32_t *out)
    {
        if constexpr (N < 5) return hipErrorInvalidValue;
        else {
            *out = occ_batch<N, false, false, false, false, alt_map<N>()>();
            return hipSuccess;
        }
    }
};

template <int N> struct Shape {
    static hipError_t run(bool pair, bool alt, int32_t *lanes, int32_t *top)
    {
        if (pair) {
            *lanes = Geo<N, true>::G;
            *top = Geo<N, true>::OFF;
        } else if (alt && N >= 5) {
            constexpr int M = N >= 5 ? alt_map<N>() : kMapDefault;
            *lanes = Geo<N, false, M>::G;
            *top = Geo<N, false, M>::OFF;
        } else {
            *lanes = Geo<N>::G;
            *top = Geo<N>::OFF;
        }
        return hipSuccess;
    }
};

} // namespace

hipError_t launch_batch_alt(int32_t order, const ItemDesc *items_dev, const TileRef *tiles_dev,
                            int64_t n_tiles, int32_t grid_blocks, hipStream_t s)
{
    return dispatch<BatchAlt>(order, items_dev, tiles_dev, n_tiles, grid_blocks, s);
}

int32_t batch_blocks_per_cu_alt(int32_t order)
{
    int32_t b = 1;
    return dispatch<OccAlt>(order, &b) == hipSuccess ? b : 1;
}

void mapping_shape(int32_t key, bool alt, int32_t *lanes_per_item, int32_t *top_levels)
{
    *lanes_per_item = 0;
    *top_levels = 0;
    (void)dispatch<Shape>(key_order(key), key_pair(key), alt, lanes_per_item, top_levels);
}

} // namespace qqmc
