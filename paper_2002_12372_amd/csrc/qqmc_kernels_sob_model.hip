/*
 * qqmc_kernels_sob_model.hip -- Sobol' points (App. B) through the learned
 * second warp (App. I): the charge kernels with the model's inverse CDFs in
 * front of the exponential warp, and the learning pass over Sobol' points,
 * both elimination trees.
 */
#include "qqmc_kernels.h"

namespace qqmc {

namespace {

template <int N> struct OrderSobModel {
    static hipError_t run(const ItemDesc &it, hipStream_t s)
    {
        return needs_pair(it.g0y) ? go_order<N, true, true, false, true>(it, s)
                                  : go_order<N, true, false, false, true>(it, s);
    }
};

template <int N> struct SampleSob {
    static hipError_t run(const ItemDesc &it, hipStream_t s)
    {
        return needs_pair(it.g0y) ? go_sample<N, true, true>(it, s)
                                  : go_sample<N, false, true>(it, s);
    }
};

} // namespace

hipError_t launch_order_sobol_model(const ItemDesc &it, hipStream_t s)
{
    return dispatch<OrderSobModel>(it.order, it, s);
}

hipError_t launch_sample_sobol(const ItemDesc &it, hipStream_t s)
{
    return dispatch<SampleSob>(it.order, it, s);
}

} // namespace qqmc
