/*
 * qqmc_kernels_cur.hip -- the current into a lead (the lead site in the
 * measurement column) on the lattice, both elimination trees: order and
 * points launches.
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

} // namespace

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
