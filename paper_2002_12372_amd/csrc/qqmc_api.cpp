/*
 * qqmc_api.cpp -- C ABI of the QQMC library: argument checking, device
 * buffers, launches, and the host epilogue of the randomised-QMC estimate
 * (mean and standard error over the shifts, App. G).
 */
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "qqmc_internal.h"

namespace qqmc {

namespace {
thread_local std::string g_last_error;
}

qqmc_status set_error(qqmc_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

qqmc_status hip_error(hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return set_error(e == hipErrorOutOfMemory ? QQMC_ENOMEM : QQMC_EDEVICE, m);
}

qqmc_status validate_order(const qqmc_order *ord, int32_t n_grid, double t_half,
                           Validated *out)
{
    (void)n_grid;
    if (!ord) return set_error(QQMC_EINVAL, "order descriptor is NULL");
    const int n = ord->order;
    if (n < 1 || n > QQMC_MAX_ORDER)
        return set_error(QQMC_EINVAL, "order must be in 1.." + std::to_string(QQMC_MAX_ORDER));
    if (ord->log2_n < 6 || ord->log2_n > 24)
        return set_error(QQMC_EINVAL, "log2_n must be in 6..24");
    const uint64_t N = (uint64_t)1 << ord->log2_n;
    const bool sobol = ord->sobol_v != nullptr;
    if (!sobol && ((ord->lattice_a & 1u) == 0 || ord->lattice_a <= 1 || ord->lattice_a >= N))
        return set_error(QQMC_EINVAL, "lattice_a must be odd with 1 < a < N");
    if (ord->n_shifts < 1 || ord->n_shifts > 65535)
        return set_error(QQMC_EINVAL, "n_shifts must be in 1..65535");
    if (!sobol && !ord->shifts) return set_error(QQMC_EINVAL, "shifts is NULL");
    if (sobol && !ord->sobol_shifts) return set_error(QQMC_EINVAL, "sobol_shifts is NULL");
    if (!(ord->model_tau > 0.0) || !std::isfinite(ord->model_tau))
        return set_error(QQMC_EINVAL, "model_tau must be positive");
    if (!(ord->t_meas > 0.0) || !(ord->t_meas <= t_half))
        return set_error(QQMC_EINVAL, "t_meas must satisfy 0 < t_meas <= t_half of the tables");
    if (ord->mode < QQMC_MODE_CHARGE || ord->mode > QQMC_MODE_CURRENT)
        return set_error(QQMC_EINVAL, "unknown mode");
    if (ord->mode == QQMC_MODE_CURRENT && ord->model)
        return set_error(QQMC_EINVAL, "the current has no learned warp");
    if (ord->model && (ord->model->order != n || !ord->model->d_cdf))
        return set_error(QQMC_EINVAL, "model of another order");
    if (!std::isfinite(ord->alpha)) return set_error(QQMC_EINVAL, "alpha must be finite");
    const size_t ns = (size_t)ord->n_shifts * (size_t)n;
    if (sobol) {
        out->shifts.assign(ns, 0.0);
        out->sobol.assign(ord->sobol_v, ord->sobol_v + (size_t)n * 32);
        out->sobol.insert(out->sobol.end(), ord->sobol_shifts, ord->sobol_shifts + ns);
    } else {
        out->shifts.assign(ord->shifts, ord->shifts + ns);
        out->sobol.clear();
    }
    for (double v : out->shifts)
        if (!(v >= 0.0 && v < 1.0)) return set_error(QQMC_EINVAL, "every shift must lie in [0, 1)");
    ItemDesc &d = out->desc;
    std::memset(&d, 0, sizeof(d));
    d.order = n;
    d.mode = ord->mode;
    d.n_shifts = ord->n_shifts;
    d.mask = (uint32_t)(N - 1);
    d.inv_n = 1.0 / (double)N;
    d.t_meas = ord->t_meas;
    d.tau = ord->model_tau;
    d.alpha = ord->alpha;
    d.sobol_points = sobol ? 1 : 0;
    double c = 1.0;
    for (int k = 0; k < n; ++k) c *= ord->model_tau;
    d.tau_n = c;
    uint64_t z = 1;
    for (int j = 0; j < n; ++j) {
        d.z[j] = (uint32_t)z;
        z = (z * ord->lattice_a) % N;
    }
    if (ord->model) {
        d.model_cdf = ord->model->d_cdf;
        d.model_bins = ord->model->n_bins;
    }
    return QQMC_OK;
}

int32_t default_tile_len(const ItemDesc &d, int64_t N)
{
    /* about 64 tiles per resident single-wave workgroup (1024 on 256 CUs)
     * keeps the last round of tiles short */
    int64_t t = 2048;
    while (t > 64 && (int64_t)d.n_shifts * (N / t) < 65536) t /= 2;
    if (t > N) t = N;
    return (int32_t)t;
}

qqmc_status check_tables(qqmc_tables t)
{
    if (!t || !t->d_tab) return set_error(QQMC_EINVAL, "tables handle is NULL");
    return QQMC_OK;
}

void fill_item_tables(ItemDesc &d, const qqmc_tables_s *t)
{
    d.tab = t->d_tab;
    d.n_grid = t->n_grid;
    d.t_half = t->t_half;
    d.h = t->h;
    /* every vertex diagonal is g^<(0) - i alpha (App. E); the measurement
     * diagonal cancels from the Keldysh sum and is never formed here */
    d.g0x = 0.0;
    d.g0y = t->n_sigma - d.alpha;
    d.col = t->d_col;
}

qqmc_status upload_tables(const double *tab4, int32_t n_grid, double t_half, double n_sigma,
                          hipStream_t s, qqmc_tables *out)
{
    auto *t = new (std::nothrow) qqmc_tables_s();
    if (!t) return set_error(QQMC_ENOMEM, "host allocation failed");
    hipGetDevice(&t->device);
    t->n_grid = n_grid;
    t->t_half = t_half;
    t->h = 2.0 * t_half / (n_grid - 1);
    t->n_sigma = n_sigma;
    const size_t bytes = sizeof(double) * 4 * (size_t)n_grid;
    hipError_t e = hipMalloc(&t->d_tab, bytes);
    if (e != hipSuccess) {
        delete t;
        return hip_error(e, "hipMalloc(tables)");
    }
    e = hipMemcpyAsync(t->d_tab, tab4, bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        hipFree(t->d_tab);
        delete t;
        return hip_error(e, "upload of tables");
    }
    *out = t;
    return QQMC_OK;
}

/* Device buffers of one asynchronous order evaluation. */
struct OrderBuffers {
    double *shifts = nullptr, *tile_sums = nullptr, *shift_sums = nullptr;
    uint32_t *sobol = nullptr;
    ItemDesc *item = nullptr;
    int64_t *base = nullptr;
};

void free_async(void *p, hipStream_t s)
{
    if (p) hipFreeAsync(p, s);
}

} // namespace qqmc

using namespace qqmc;

extern "C" {

const char *qqmc_last_error(void) { return g_last_error.c_str(); }

static qqmc_status check_dot(const qqmc_dot *dot)
{
    if (!dot) return set_error(QQMC_EINVAL, "NULL argument");
    if (!(dot->gamma > 0.0) || !(dot->beta > 0.0) || !(dot->t_half > 0.0) ||
        !std::isfinite(dot->eps_d) || !std::isfinite(dot->bias_v) || std::isnan(dot->beta) ||
        !std::isfinite(dot->gamma) || !std::isfinite(dot->t_half))
        return set_error(QQMC_EINVAL,
                         "gamma, t_half must be positive and finite, beta positive (+inf: T = 0)");
    if (dot->n_grid < 2 || dot->n_grid > (1 << 24))
        return set_error(QQMC_EINVAL, "n_grid must be in 2..2^24");
    if (std::isnan(dot->half_bandwidth) || dot->half_bandwidth < 0.0)
        return set_error(QQMC_EINVAL, "half_bandwidth must be >= 0 (0 or +inf: wide band)");
    if (finite_band(dot) && !(std::fabs(dot->eps_d) < dot->half_bandwidth - dot->gamma))
        return set_error(QQMC_EINVAL,
                         "finite band needs |eps_d| < D - gamma (no bound state outside the band)");
    if (dot->lead != 0 && !((dot->lead == 1 || dot->lead == 2) && finite_band(dot)))
        return set_error(QQMC_EINVAL, "lead must be 0, or 1 or 2 with a finite half_bandwidth");
    return QQMC_OK;
}

qqmc_status qqmc_tables_compute_host(const qqmc_dot *dot, double *gl, double *gg, double *n_sigma)
{
    if (qqmc_status st = check_dot(dot)) return st;
    if (!gl || !gg) return set_error(QQMC_EINVAL, "NULL output");
    std::vector<double> tab(4 * (size_t)dot->n_grid);
    double ns;
    if (finite_band(dot)) {
        ns = build_tables_band(dot->eps_d, dot->gamma, dot->beta, dot->bias_v,
                               dot->half_bandwidth, dot->n_grid, dot->t_half, tab.data());
    } else {
        ns = occupation_per_spin(dot->eps_d, dot->gamma, dot->beta, dot->bias_v);
        build_tables_host(dot->eps_d, dot->gamma, dot->beta, dot->bias_v, dot->n_grid,
                          dot->t_half, ns, tab.data());
    }
    for (int32_t j = 0; j < dot->n_grid; ++j) {
        gl[2 * j] = tab[4 * j];
        gl[2 * j + 1] = tab[4 * j + 1];
        gg[2 * j] = tab[4 * j + 2];
        gg[2 * j + 1] = tab[4 * j + 3];
    }
    if (n_sigma) *n_sigma = ns;
    return QQMC_OK;
}

qqmc_status qqmc_make_tables(const qqmc_dot *dot, void *stream, qqmc_tables *out)
{
    if (qqmc_status st = check_dot(dot)) return st;
    if (!out) return set_error(QQMC_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (finite_band(dot)) {
        /* semicircular leads: band quadrature on the host, then upload */
        std::vector<double> tab(4 * (size_t)dot->n_grid);
        const double nsb = build_tables_band(dot->eps_d, dot->gamma, dot->beta, dot->bias_v,
                                             dot->half_bandwidth, dot->n_grid, dot->t_half,
                                             tab.data());
        qqmc_tables t = nullptr;
        if (qqmc_status st = upload_tables(tab.data(), dot->n_grid, dot->t_half, nsb, s, &t))
            return st;
        if (dot->lead) {
            build_lead_tables(dot->eps_d, dot->gamma, dot->beta, dot->bias_v,
                              dot->half_bandwidth, dot->lead, dot->n_grid, dot->t_half,
                              tab.data());
            hipError_t e = hipMalloc(&t->d_col, sizeof(double) * tab.size());
            if (e == hipSuccess)
                e = hipMemcpy(t->d_col, tab.data(), sizeof(double) * tab.size(),
                              hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                qqmc_free_tables(t);
                return hip_error(e, "lead table upload");
            }
        }
        *out = t;
        return QQMC_OK;
    }
    const double ns = occupation_per_spin(dot->eps_d, dot->gamma, dot->beta, dot->bias_v);
    if (std::isinf(dot->beta)) {
        /* zero temperature: contour quadrature on the host, then upload */
        std::vector<double> tab(4 * (size_t)dot->n_grid);
        build_tables_host(dot->eps_d, dot->gamma, dot->beta, dot->bias_v, dot->n_grid,
                          dot->t_half, ns, tab.data());
        return upload_tables(tab.data(), dot->n_grid, dot->t_half, ns, s, out);
    }
    auto *t = new (std::nothrow) qqmc_tables_s();
    if (!t) return set_error(QQMC_ENOMEM, "host allocation failed");
    hipGetDevice(&t->device);
    t->n_grid = dot->n_grid;
    t->t_half = dot->t_half;
    t->h = 2.0 * dot->t_half / (dot->n_grid - 1);
    t->n_sigma = ns;
    hipError_t e = hipMalloc(&t->d_tab, sizeof(double) * 4 * (size_t)dot->n_grid);
    if (e == hipSuccess)
        e = launch_tables(t->d_tab, dot->n_grid, dot->t_half, dot->eps_d, dot->gamma, dot->beta,
                          dot->bias_v, ns, s);
    if (e != hipSuccess) {
        if (t->d_tab) hipFree(t->d_tab);
        delete t;
        return hip_error(e, "device table build");
    }
    *out = t;
    return QQMC_OK;
}

qqmc_status qqmc_tables_from_host(const double *gl, const double *gg, int32_t n_grid,
                                  double t_half, double n_sigma, void *stream,
                                  qqmc_tables *out)
{
    if (!gl || !gg || !out) return set_error(QQMC_EINVAL, "NULL argument");
    if (n_grid < 2 || n_grid > (1 << 24) || !(t_half > 0.0) || !std::isfinite(n_sigma))
        return set_error(QQMC_EINVAL, "bad grid or n_sigma");
    std::vector<double> tab(4 * (size_t)n_grid);
    for (int32_t j = 0; j < n_grid; ++j) {
        tab[4 * j + 0] = gl[2 * j];
        tab[4 * j + 1] = gl[2 * j + 1];
        tab[4 * j + 2] = gg[2 * j];
        tab[4 * j + 3] = gg[2 * j + 1];
    }
    return upload_tables(tab.data(), n_grid, t_half, n_sigma, (hipStream_t)stream, out);
}

qqmc_status qqmc_tables_export(qqmc_tables t, double *gl, double *gg, double *n_sigma)
{
    if (qqmc_status st = check_tables(t)) return st;
    if (n_sigma) *n_sigma = t->n_sigma;
    if (!gl && !gg) return QQMC_OK;
    std::vector<double> tab(4 * (size_t)t->n_grid);
    /* the table may still be being built on the stream given at creation */
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(tab.data(), t->d_tab, sizeof(double) * tab.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_error(e, "hipMemcpy(tables)");
    for (int32_t j = 0; j < t->n_grid; ++j) {
        if (gl) { gl[2 * j] = tab[4 * j]; gl[2 * j + 1] = tab[4 * j + 1]; }
        if (gg) { gg[2 * j] = tab[4 * j + 2]; gg[2 * j + 1] = tab[4 * j + 3]; }
    }
    return QQMC_OK;
}

qqmc_status qqmc_tables_info(qqmc_tables t, int32_t *n_grid, double *t_half)
{
    if (qqmc_status st = check_tables(t)) return st;
    if (n_grid) *n_grid = t->n_grid;
    if (t_half) *t_half = t->t_half;
    return QQMC_OK;
}

void qqmc_free_tables(qqmc_tables t)
{
    if (!t) return;
    if (t->d_tab) hipFree(t->d_tab);
    if (t->d_col) hipFree(t->d_col);
    delete t;
}

qqmc_status qqmc_lead_tables_compute_host(const qqmc_dot *dot, double *cl, double *cg)
{
    if (qqmc_status st = check_dot(dot)) return st;
    if (!cl || !cg) return set_error(QQMC_EINVAL, "NULL output");
    if (dot->lead != 1 && dot->lead != 2) return set_error(QQMC_EINVAL, "lead must be 1 or 2");
    std::vector<double> tab(4 * (size_t)dot->n_grid);
    build_lead_tables(dot->eps_d, dot->gamma, dot->beta, dot->bias_v, dot->half_bandwidth,
                      dot->lead, dot->n_grid, dot->t_half, tab.data());
    for (int32_t j = 0; j < dot->n_grid; ++j) {
        cl[2 * j] = tab[4 * j];
        cl[2 * j + 1] = tab[4 * j + 1];
        cg[2 * j] = tab[4 * j + 2];
        cg[2 * j + 1] = tab[4 * j + 3];
    }
    return QQMC_OK;
}

qqmc_status qqmc_tables_lead_from_host(qqmc_tables t, const double *cl, const double *cg)
{
    if (qqmc_status st = check_tables(t)) return st;
    if (!cl || !cg) return set_error(QQMC_EINVAL, "NULL argument");
    std::vector<double> tab(4 * (size_t)t->n_grid);
    for (int32_t j = 0; j < t->n_grid; ++j) {
        tab[4 * j + 0] = cl[2 * j];
        tab[4 * j + 1] = cl[2 * j + 1];
        tab[4 * j + 2] = cg[2 * j];
        tab[4 * j + 3] = cg[2 * j + 1];
    }
    hipError_t e = hipSuccess;
    if (!t->d_col) e = hipMalloc(&t->d_col, sizeof(double) * tab.size());
    if (e == hipSuccess)
        e = hipMemcpy(t->d_col, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "lead table upload");
    return QQMC_OK;
}

qqmc_status qqmc_eval_order_async(qqmc_tables t, const qqmc_order *ord, int32_t tile_len,
                                  void *stream, double *tile_sums, double *shift_sums,
                                  int64_t *n_tiles_out)
{
    if (qqmc_status st = check_tables(t)) return st;
    if (!shift_sums) return set_error(QQMC_EINVAL, "shift_sums is NULL");
    Validated v;
    if (qqmc_status st = validate_order(ord, t->n_grid, t->t_half, &v)) return st;
    const int64_t N = (int64_t)1 << ord->log2_n;
    ItemDesc d = v.desc;
    fill_item_tables(d, t);
    if (d.mode == QQMC_MODE_CURRENT && !d.col)
        return set_error(QQMC_EINVAL, "the current needs tables with lead functions");
    if (tile_len == 0) tile_len = default_tile_len(d, N);
    if (tile_len < 64 || tile_len % 64 != 0 || N % tile_len != 0)
        return set_error(QQMC_EINVAL, "tile_len must be a multiple of 64 dividing N");
    d.tile_len = tile_len;
    d.tiles_per_shift = (int32_t)(N / tile_len);
    d.n_tiles = (int64_t)d.tiles_per_shift * d.n_shifts;
    if (n_tiles_out) *n_tiles_out = d.n_tiles;
    hipStream_t s = (hipStream_t)stream;
    OrderBuffers b;
    hipError_t e = hipMallocAsync((void **)&b.shifts, sizeof(double) * v.shifts.size(), s);
    if (e == hipSuccess && !tile_sums)
        e = hipMallocAsync((void **)&b.tile_sums, sizeof(double) * 2 * d.n_tiles, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&b.item, sizeof(ItemDesc), s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&b.base, sizeof(int64_t), s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.shifts, v.shifts.data(), sizeof(double) * v.shifts.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !v.sobol.empty()) {
        e = hipMallocAsync((void **)&b.sobol, sizeof(uint32_t) * v.sobol.size(), s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b.sobol, v.sobol.data(), sizeof(uint32_t) * v.sobol.size(),
                               hipMemcpyHostToDevice, s);
    }
    d.shifts = b.shifts;
    d.sobol = b.sobol;
    d.tile_sums = tile_sums ? tile_sums : b.tile_sums;
    const int64_t zero = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.item, &d, sizeof(ItemDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.base, &zero, sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_order(d, s);
    if (e == hipSuccess) e = launch_shift_reduce(b.item, 1, b.base, shift_sums, d.n_shifts, s);
    free_async(b.shifts, s);
    free_async(b.sobol, s);
    free_async(b.tile_sums, s);
    free_async(b.item, s);
    free_async(b.base, s);
    if (e != hipSuccess) return hip_error(e, "qqmc_eval_order launch");
    return QQMC_OK;
}

qqmc_status qqmc_eval_order(qqmc_tables t, const qqmc_order *ord, void *stream,
                            double *q_shift, double *q_mean, double *q_stderr)
{
    if (!q_shift) return set_error(QQMC_EINVAL, "q_shift is NULL");
    if (qqmc_status st = check_tables(t)) return st;
    if (!ord) return set_error(QQMC_EINVAL, "order descriptor is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int K = ord->n_shifts > 0 ? ord->n_shifts : 1;
    double *d_sums = nullptr;
    hipError_t e = hipMallocAsync((void **)&d_sums, sizeof(double) * 2 * K, s);
    if (e != hipSuccess) return hip_error(e, "hipMallocAsync");
    qqmc_status st = qqmc_eval_order_async(t, ord, 0, stream, nullptr, d_sums, nullptr);
    std::vector<double> sums(2 * (size_t)K);
    if (st == QQMC_OK) {
        e = hipMemcpyAsync(sums.data(), d_sums, sizeof(double) * 2 * K, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_error(e, "result copy");
    }
    hipFreeAsync(d_sums, s);
    if (st != QQMC_OK) return st;
    const double N = std::ldexp(1.0, ord->log2_n);
    double mr = 0.0, mi = 0.0;
    for (int k = 0; k < K; ++k) {
        q_shift[2 * k] = sums[2 * k] / N;
        q_shift[2 * k + 1] = sums[2 * k + 1] / N;
        mr += q_shift[2 * k];
        mi += q_shift[2 * k + 1];
    }
    mr /= K;
    mi /= K;
    if (q_mean) { q_mean[0] = mr; q_mean[1] = mi; }
    if (q_stderr) {
        if (K < 2) {
            *q_stderr = std::nan("");
        } else {
            double ss = 0.0;
            for (int k = 0; k < K; ++k) ss += (q_shift[2 * k] - mr) * (q_shift[2 * k] - mr);
            *q_stderr = std::sqrt(ss / (K - 1)) / std::sqrt((double)K);
        }
    }
    return QQMC_OK;
}

qqmc_status qqmc_eval_points(qqmc_tables t, int32_t order, double t_meas, double alpha,
                             int32_t observable, const double *u, int64_t n_points,
                             int32_t method, double *f, double *mass, void *stream)
{
    if (qqmc_status st = check_tables(t)) return st;
    if (order < 1 || order > QQMC_MAX_ORDER) return set_error(QQMC_EINVAL, "bad order");
    if (n_points < 0) return set_error(QQMC_EINVAL, "n_points < 0");
    if (n_points > 0 && (!u || !f)) return set_error(QQMC_EINVAL, "NULL buffer");
    if (!(t_meas > 0.0) || !(t_meas <= t->t_half))
        return set_error(QQMC_EINVAL, "t_meas must satisfy 0 < t_meas <= t_half");
    if (!std::isfinite(alpha)) return set_error(QQMC_EINVAL, "alpha must be finite");
    if (observable != QQMC_OBS_CHARGE && observable != QQMC_OBS_CURRENT)
        return set_error(QQMC_EINVAL, "unknown observable");
    if (observable == QQMC_OBS_CURRENT && !t->d_col)
        return set_error(QQMC_EINVAL, "the current needs tables with lead functions");
    const double *col = observable == QQMC_OBS_CURRENT ? t->d_col : nullptr;
    if (method != QQMC_METHOD_TREE && method != QQMC_METHOD_DIRECT)
        return set_error(QQMC_EINVAL, "unknown method");
    if (mass && method != QQMC_METHOD_DIRECT)
        return set_error(QQMC_EINVAL, "the term mass comes from the direct method only");
    if (n_points == 0) return QQMC_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (method == QQMC_METHOD_TREE)
        e = launch_points_tree(t->d_tab, col, t->n_grid, t->t_half, t->h, t->n_sigma, alpha,
                               order, t_meas, u, n_points, f, s);
    else if (method == QQMC_METHOD_DIRECT)
        e = launch_points_direct(t->d_tab, col, t->n_grid, t->t_half, t->h, t->n_sigma, alpha,
                                 order, t_meas, u, n_points, f, mass, s);
    else
        return set_error(QQMC_EINVAL, "unknown method");
    if (e != hipSuccess) return hip_error(e, "qqmc_eval_points launch");
    return QQMC_OK;
}

} // extern "C"
