/*
 * qqmc_tables.cpp -- host side of the Green's-function tables (App. E):
 * n_sigma from the digamma closed form, and a host build of the grid from
 * the residue series of qqmc_gf.h (the device build is tables_kernel).
 */
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "qqmc_gf.h"
#include "qqmc_internal.h"

namespace qqmc {

namespace {

using cd = std::complex<double>;

/* Complex digamma: upward recurrence psi(z) = psi(z+1) - 1/z to Re z >= 14,
 * then the Stirling series with Bernoulli numbers up to B_14. */
cd digamma(cd z)
{
    cd acc = 0.0;
    while (z.real() < 14.0) {
        acc -= 1.0 / z;
        z += 1.0;
    }
    const cd w = 1.0 / (z * z);
    /* B_2k / (2k) for k = 1..7 */
    const double c[7] = {1.0 / 12.0, -1.0 / 120.0, 1.0 / 252.0, -1.0 / 240.0,
                         1.0 / 132.0, -691.0 / 32760.0, 1.0 / 12.0};
    cd series = 0.0;
    for (int k = 6; k >= 0; --k) series = (series + c[k]) * w;
    return acc + std::log(z) - 0.5 / z - series;
}

/* Compensated sum of the Matsubara terms, smallest (largest k) first. */
cplx matsubara_sum_host(double eps_d, double gamma, double beta, double mu, double tau)
{
    const long kmax = matsubara_kmax(beta, tau);
    double sr = 0.0, si = 0.0, cr = 0.0, ci = 0.0;
    for (long k = kmax; k >= 0; --k) {
        const cplx t = matsubara_term(eps_d, gamma, beta, mu, tau, k);
        double y = t.x - cr, s = sr + y;
        cr = (s - sr) - y;
        sr = s;
        y = t.y - ci;
        s = si + y;
        ci = (s - si) - y;
        si = s;
    }
    return cmk(sr, si);
}

} // namespace

double occupation_per_spin(double eps_d, double gamma, double beta, double bias_v)
{
    double n = 0.0;
    const double mus[2] = {0.5 * bias_v, -0.5 * bias_v};
    for (double mu : mus) {
        const cd z = 0.5 + beta * cd(gamma, eps_d - mu) / (2.0 * kPiGF);
        n += 0.5 * (0.5 - digamma(z).imag() / kPiGF);
    }
    return n;
}

void build_tables_host(double eps_d, double gamma, double beta, double bias_v,
                       int32_t n_grid, double t_half, double n_sigma, double *tab)
{
    const double h = 2.0 * t_half / (n_grid - 1);
    unsigned nt = std::thread::hardware_concurrency();
    if (nt < 1) nt = 1;
    if (nt > 64) nt = 64;
    auto work = [&](unsigned tid) {
        for (int32_t j = (int32_t)tid; j < n_grid; j += (int32_t)nt) {
            const double tau = -t_half + j * h;
            cplx gl_abs = cmk(0.0, 0.0);
            if (tau != 0.0) {
                const double at = std::fabs(tau);
                gl_abs = lesser_from_sums(eps_d, gamma, beta, bias_v, at,
                                          matsubara_sum_host(eps_d, gamma, beta, 0.5 * bias_v, at),
                                          matsubara_sum_host(eps_d, gamma, beta, -0.5 * bias_v, at));
            }
            const pairv v = node_values(eps_d, gamma, tau, gl_abs, n_sigma);
            tab[4 * j + 0] = v.gl.x;
            tab[4 * j + 1] = v.gl.y;
            tab[4 * j + 2] = v.gg.x;
            tab[4 * j + 3] = v.gg.y;
        }
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nt; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto &th : pool) th.join();
}

} // namespace qqmc
