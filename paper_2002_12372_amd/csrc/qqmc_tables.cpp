/*
 * qqmc_tables.cpp -- host side of the Green's-function tables (App. E):
 * n_sigma from the digamma closed form (arctan at zero temperature), and a
 * host build of the grid from the residue series of qqmc_gf.h (the device
 * build is tables_kernel) or, at zero temperature, from the deformed-contour
 * Fourier integral.
 */
#include <algorithm>
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

/* Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_m). */
void legendre_rule(int m, double *x, double *w)
{
    for (int i = 0; i < m; ++i) {
        double z = std::cos(kPiGF * (i + 0.75) / (m + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= m; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = m * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Zero temperature (App. E, "Precision calculation of g^<(t) and g^>(t")):
 * for tau > 0, Int_{-inf}^{mu} zeta(omega) e^{-i omega tau} d omega with
 * zeta = A/2pi = (Gamma/pi) / ((omega - eps_d)^2 + Gamma^2).  The integrand
 * decays in the lower half plane, so left of c = min(mu, eps_d) - Gamma - 1
 * (no pole between the real axis and the vertical line Re omega = c) the
 * path turns down the half-line c - i s:
 *   Int_{-inf}^{c} = i e^{-i c tau} Int_0^inf zeta(c - i s) e^{-s tau} ds;
 * [c, mu] stays on the real axis.  Both parts by composite 16-point
 * Gauss-Legendre (width 0.04 on the segment; on the half-line panels
 * growing by 1.3 from min(0.04, 0.4/tau) out to 64/tau). */
cd zeta0(double eps_d, double gamma, cd w)
{
    const cd d = w - eps_d;
    return gamma / kPiGF / (d * d + gamma * gamma);
}

cd below_mu_T0(double eps_d, double gamma, double mu, double tau)
{
    constexpr int M = 16;
    double gx[M], gw[M];
    legendre_rule(M, gx, gw);
    const double c = std::min(mu, eps_d) - gamma - 1.0;
    const cd I(0.0, 1.0);
    cd seg = 0.0;
    const int panels = std::max(1, (int)std::ceil((mu - c) / 0.04));
    const double wseg = (mu - c) / panels;
    for (int p = 0; p < panels; ++p) {
        const double lo = c + p * wseg;
        cd part = 0.0;
        for (int q = 0; q < M; ++q) {
            const double w = lo + 0.5 * wseg * (gx[q] + 1.0);
            part += gw[q] * zeta0(eps_d, gamma, w) * std::exp(-I * (w * tau));
        }
        seg += 0.5 * wseg * part;
    }
    cd half = 0.0;
    double lo = 0.0, width = std::min(0.04, 0.4 / tau);
    const double smax = 64.0 / tau;
    while (lo < smax) {
        cd part = 0.0;
        for (int q = 0; q < M; ++q) {
            const double sq = lo + 0.5 * width * (gx[q] + 1.0);
            part += gw[q] * zeta0(eps_d, gamma, cd(c, -sq)) * std::exp(-sq * tau);
        }
        half += 0.5 * width * part;
        lo += width;
        width *= 1.3;
    }
    return I * std::exp(-I * (c * tau)) * half + seg;
}

/* g^<(tau), tau > 0, at zero temperature */
cplx lesser_T0(double eps_d, double gamma, double bias_v, double tau)
{
    const cd sum = below_mu_T0(eps_d, gamma, 0.5 * bias_v, tau) +
                   below_mu_T0(eps_d, gamma, -0.5 * bias_v, tau);
    const cd g = cd(0.0, 0.5) * sum;
    return cmk(g.real(), g.imag());
}

} // namespace

double occupation_per_spin(double eps_d, double gamma, double beta, double bias_v)
{
    if (std::isinf(beta))
        return 0.5 * (1.0 + (std::atan((0.5 * bias_v - eps_d) / gamma) +
                             std::atan((-0.5 * bias_v - eps_d) / gamma)) / kPiGF);
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
                if (std::isinf(beta))
                    gl_abs = lesser_T0(eps_d, gamma, bias_v, at);
                else
                    gl_abs = lesser_from_sums(
                        eps_d, gamma, beta, bias_v, at,
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
