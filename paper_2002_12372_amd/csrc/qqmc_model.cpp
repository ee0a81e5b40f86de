/*
 * qqmc_model.cpp -- the learned second warp of App. I ("Learning h^(i) from
 * the integrand"): the learning pass (GPU), the projection and Gaussian
 * kernel smoothing of the sampled integrand (host), and the model handle.
 *
 * A model holds, per coordinate j of the unit cube, a density q_j that is
 * piecewise constant on n_bins equal bins of [0, 1), stored as its CDF at the
 * bin edges.  The integrand kernels map a lattice point x to w_j =
 * F_j^{-1}(x_j) before the exponential warp and divide the weight by
 * prod_j q_j(w_j).
 */
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "qqmc_internal.h"

namespace qqmc {
namespace {

/* One coordinate: projection h[0..nb) -> smoothed with the Gaussian kernel
 * exp(-(w - w')^2 / lambda^2) over the bin centres (normalised by the kernel
 * weights), normalised to a density p, mixed with the uniform density
 * (q = (1 - floor_eps) p + floor_eps; uniform if the projection is empty),
 * integrated to the CDF c[0..nb] at the bin edges, c[0] = 0, c[nb] = 1. */
void cdf_from_projection(const double *h, int nb, double lambda, double floor_eps, double *c)
{
    std::vector<double> sm((size_t)nb);
    double total = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double wb = (b + 0.5) / nb;
        double num = 0.0, den = 0.0;
        for (int k = 0; k < nb; ++k) {
            const double d = (wb - (k + 0.5) / nb) / lambda;
            const double K = std::exp(-d * d);
            num += K * h[k];
            den += K;
        }
        sm[(size_t)b] = num / den;
        total += sm[(size_t)b] / nb;
    }
    c[0] = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double p = total > 0.0 ? sm[(size_t)b] / total : 1.0;
        const double q = (1.0 - floor_eps) * p + floor_eps;
        c[b + 1] = c[b] + q / nb;
    }
    const double end = c[nb];
    for (int b = 1; b < nb; ++b) c[b] /= end;
    c[nb] = 1.0;
}

qqmc_status upload(qqmc_model_s *m)
{
    hipGetDevice(&m->device);
    hipError_t e = hipMalloc((void **)&m->d_cdf, sizeof(double) * m->cdf.size());
    if (e == hipSuccess)
        e = hipMemcpy(m->d_cdf, m->cdf.data(), sizeof(double) * m->cdf.size(),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "model upload");
    return QQMC_OK;
}

} // namespace
} // namespace qqmc

using namespace qqmc;

extern "C" {

qqmc_status qqmc_learn_model(qqmc_tables t, const qqmc_learn_params *p, void *stream,
                             qqmc_model *out)
{
    if (qqmc_status st = check_tables(t)) return st;
    if (!p || !out) return set_error(QQMC_EINVAL, "NULL argument");
    if (p->n_bins < 1 || p->n_bins > 4096) return set_error(QQMC_EINVAL, "n_bins must be in 1..4096");
    if (!(p->lambda > 0.0) || !std::isfinite(p->lambda))
        return set_error(QQMC_EINVAL, "lambda must be positive");
    if (!(p->floor_eps >= 0.0 && p->floor_eps <= 1.0))
        return set_error(QQMC_EINVAL, "floor_eps must be in [0, 1]");
    if ((p->sobol_v == nullptr) != (p->sobol_shift == nullptr))
        return set_error(QQMC_EINVAL, "sobol_v and sobol_shift go together");
    /* the learning sample is one shifted lattice or the first 2^log2_m
     * digitally shifted Sobol' points, charge mode, no model */
    qqmc_order o;
    std::memset(&o, 0, sizeof(o));
    o.order = p->order;
    o.log2_n = p->log2_m;
    o.lattice_a = p->lattice_a;
    o.n_shifts = 1;
    o.shifts = p->shift;
    o.sobol_v = p->sobol_v;
    o.sobol_shifts = p->sobol_shift;
    o.model_tau = p->model_tau;
    o.t_meas = p->t_meas;
    o.mode = QQMC_MODE_CHARGE;
    o.model = nullptr;
    o.alpha = p->alpha;
    Validated v;
    if (qqmc_status st = validate_order(&o, t->n_grid, t->t_half, &v)) return st;
    ItemDesc &d = v.desc;
    fill_item_tables(d, t);
    const int n = p->order, nb = p->n_bins;
    const int64_t M = (int64_t)1 << p->log2_m;
    d.tile_len = default_tile_len(d, M);
    d.tiles_per_shift = (int32_t)(M / d.tile_len);
    d.n_tiles = d.tiles_per_shift;

    hipStream_t s = (hipStream_t)stream;
    std::vector<double> vals((size_t)M);
    double *d_shift = nullptr, *d_out = nullptr;
    uint32_t *d_sobol = nullptr;
    hipError_t e = hipMallocAsync((void **)&d_shift, sizeof(double) * n, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&d_out, sizeof(double) * (size_t)M, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_shift, v.shifts.data(), sizeof(double) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !v.sobol.empty()) {
        e = hipMallocAsync((void **)&d_sobol, sizeof(uint32_t) * v.sobol.size(), s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_sobol, v.sobol.data(), sizeof(uint32_t) * v.sobol.size(),
                               hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) {
        d.shifts = d_shift;
        d.sobol = d_sobol;
        d.sample_out = d_out;
        e = launch_sample(d, s);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(vals.data(), d_out, sizeof(double) * (size_t)M, hipMemcpyDeviceToHost, s);
    if (d_shift) hipFreeAsync(d_shift, s);
    if (d_sobol) hipFreeAsync(d_sobol, s);
    if (d_out) hipFreeAsync(d_out, s);
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return hip_error(e, "learning pass");

    auto *m = new (std::nothrow) qqmc_model_s();
    if (!m) return set_error(QQMC_ENOMEM, "host allocation failed");
    m->order = n;
    m->n_bins = nb;
    m->hist.assign((size_t)n * nb, 0.0);
    m->cdf.assign((size_t)n * (nb + 1), 0.0);
    /* projection of |Re f~| on each coordinate, in index order; the
     * coordinates are recomputed exactly as the kernel forms them */
    const uint32_t *sv = v.sobol.empty() ? nullptr : v.sobol.data();
    for (int64_t i = 0; i < M; ++i) {
        const double a = std::fabs(vals[(size_t)i]);
        if (a == 0.0) continue;
        for (int j = 0; j < n; ++j) {
            double y;
            if (sv) {
                uint32_t w = sv[(size_t)n * 32 + j];
                for (int k = 0; k < 32; ++k)
                    if (((uint64_t)i >> k) & 1u) w ^= sv[(size_t)j * 32 + k];
                y = (double)w * (1.0 / 4294967296.0);
            } else {
                const uint32_t mm = ((uint32_t)i * d.z[j]) & d.mask;
                y = (double)mm * d.inv_n + v.shifts[(size_t)j];
                if (y >= 1.0) y -= 1.0;
            }
            int b = (int)(y * nb);
            if (b > nb - 1) b = nb - 1;
            m->hist[(size_t)j * nb + b] += a;
        }
    }
    for (int j = 0; j < n; ++j)
        cdf_from_projection(m->hist.data() + (size_t)j * nb, nb, p->lambda, p->floor_eps,
                            m->cdf.data() + (size_t)j * (nb + 1));
    if (qqmc_status st = upload(m)) {
        qqmc_free_model(m);
        return st;
    }
    *out = m;
    return QQMC_OK;
}

qqmc_status qqmc_model_from_host(int32_t order, int32_t n_bins, const double *cdf, void *stream,
                                 qqmc_model *out)
{
    (void)stream;
    if (!cdf || !out) return set_error(QQMC_EINVAL, "NULL argument");
    if (order < 1 || order > QQMC_MAX_ORDER) return set_error(QQMC_EINVAL, "bad order");
    if (n_bins < 1 || n_bins > 4096) return set_error(QQMC_EINVAL, "n_bins must be in 1..4096");
    for (int j = 0; j < order; ++j) {
        const double *c = cdf + (size_t)j * (n_bins + 1);
        if (c[0] != 0.0 || c[n_bins] != 1.0)
            return set_error(QQMC_EINVAL, "every CDF row must run from 0 to 1");
        for (int b = 0; b < n_bins; ++b)
            if (!(c[b + 1] > c[b])) return set_error(QQMC_EINVAL, "every bin needs a positive width");
    }
    auto *m = new (std::nothrow) qqmc_model_s();
    if (!m) return set_error(QQMC_ENOMEM, "host allocation failed");
    m->order = order;
    m->n_bins = n_bins;
    m->cdf.assign(cdf, cdf + (size_t)order * (n_bins + 1));
    m->hist.assign((size_t)order * n_bins, 0.0);
    if (qqmc_status st = upload(m)) {
        qqmc_free_model(m);
        return st;
    }
    *out = m;
    return QQMC_OK;
}

qqmc_status qqmc_model_export(qqmc_model m, int32_t *order, int32_t *n_bins, double *cdf,
                              double *hist)
{
    if (!m) return set_error(QQMC_EINVAL, "model is NULL");
    if (order) *order = m->order;
    if (n_bins) *n_bins = m->n_bins;
    if (cdf) std::memcpy(cdf, m->cdf.data(), sizeof(double) * m->cdf.size());
    if (hist) std::memcpy(hist, m->hist.data(), sizeof(double) * m->hist.size());
    return QQMC_OK;
}

void qqmc_free_model(qqmc_model m)
{
    if (!m) return;
    if (m->d_cdf) hipFree(m->d_cdf);
    delete m;
}

} // extern "C"
