/*
 * qqmc_kernels_sob.hip -- Sobol' points (App. B; coordinate words stepped by
 * the direction numbers of the changing index bits) for the charge and the
 * current, both elimination trees (the learned warp over Sobol' points is in
 * qqmc_kernels_sob_model.hip).
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

} // namespace

hipError_t launch_order_sobol(const ItemDesc &it, hipStream_t s)
{
    return dispatch<OrderSob>(it.order, it, s);
}

} // namespace qqmc
