/*
 * qqmc_tables.cpp -- host builder of the non-interacting dot Green's
 * functions (App. E) for the wide-band limit Delta(omega) = -i Gamma.
 *
 * With A(w) = 2 Gamma / ((w - eps_d)^2 + Gamma^2) and the lead occupation
 * fbar(w) = [n_F(w - V/2) + n_F(w + V/2)] / 2 (standard Keldysh sign:
 * g^<(w) = i A fbar, g^>(w) = -i A (1 - fbar)):
 *
 *  g^<(tau), tau > 0.  Closing Int dw/2pi A n_F(w - mu) e^{-i w tau} in the
 *  lower half plane picks up the Lorentzian pole eps_d - i Gamma and the
 *  fermionic Matsubara poles mu - i nu_k, nu_k = (2k+1) pi / beta:
 *     I_mu(tau) = n_F(eps_d - mu - i Gamma) e^{-(i eps_d + Gamma) tau}
 *               + (i / beta) e^{-i mu tau} sum_k A(mu - i nu_k) e^{-nu_k tau};
 *     g^<(tau) = (i/2) [I_{V/2} + I_{-V/2}].
 *  g^>(tau) = g^<(tau) - i e^{-i eps_d tau - Gamma |tau|}, since
 *     g^> - g^< = -i Int dw/2pi A e^{-i w tau}.
 *  tau < 0: g(-tau) = -conj(g(tau)).
 *  tau = 0: g^<(0) = i n_sigma, with
 *     n_sigma = (1/2) sum_mu [1/2 - Im psi(1/2 + beta (Gamma + i(eps_d - mu))
 *                                          / (2 pi)) / pi].
 *
 * The table stores (Re g^<, Im g^<, Re g^>, Im g^>) per node so that one
 * interpolation reads 64 contiguous bytes.
 */
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "qqmc_internal.h"

namespace qqmc {

namespace {

using cd = std::complex<double>;
constexpr double kPi = 3.14159265358979323846;

cd fermi(double beta, cd z)
{
    const cd bz = beta * z;
    if (bz.real() > 0.0) {
        const cd e = std::exp(-bz);
        return e / (1.0 + e);
    }
    return 1.0 / (std::exp(bz) + 1.0);
}

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

/* sum_k A(mu - i nu_k) e^{-nu_k tau}, summed from the smallest terms up. */
cd matsubara(double eps_d, double gamma, double beta, double mu, double tau)
{
    const double nu_stop = 46.0 / tau;
    const long kmax = (long)std::ceil((nu_stop * beta / kPi - 1.0) * 0.5) + 1;
    double sr = 0.0, si = 0.0, cr = 0.0, ci = 0.0;
    for (long k = kmax; k >= 0; --k) {
        const double nu = (2.0 * (double)k + 1.0) * kPi / beta;
        const cd d = cd(mu - eps_d, -nu);
        const cd a = 2.0 * gamma / (d * d + gamma * gamma);
        const cd term = a * std::exp(-nu * tau);
        double y = term.real() - cr, t = sr + y;
        cr = (t - sr) - y;
        sr = t;
        y = term.imag() - ci;
        t = si + y;
        ci = (t - si) - y;
        si = t;
    }
    return cd(sr, si);
}

cd lesser_positive(double eps_d, double gamma, double beta, double bias_v, double tau)
{
    const cd lor = std::exp(cd(-gamma * tau, -eps_d * tau));
    cd sum = 0.0;
    const double mus[2] = {0.5 * bias_v, -0.5 * bias_v};
    for (double mu : mus) {
        sum += fermi(beta, cd(eps_d - mu, -gamma)) * lor +
               cd(0.0, 1.0 / beta) * std::exp(cd(0.0, -mu * tau)) *
                   matsubara(eps_d, gamma, beta, mu, tau);
    }
    return cd(0.0, 0.5) * sum;
}

} // namespace

double occupation_per_spin(double eps_d, double gamma, double beta, double bias_v)
{
    double n = 0.0;
    const double mus[2] = {0.5 * bias_v, -0.5 * bias_v};
    for (double mu : mus) {
        const cd z = 0.5 + beta * cd(gamma, eps_d - mu) / (2.0 * kPi);
        n += 0.5 * (0.5 - digamma(z).imag() / kPi);
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
    /* every node j with tau_j >= 0 is computed once; its mirror
     * n_grid - 1 - j gets -conj of it */
    auto work = [&](unsigned tid) {
        for (int32_t j = (int32_t)tid; j < n_grid; j += (int32_t)nt) {
            const double tau = -t_half + j * h;
            cd gl, gg;
            if (tau == 0.0) {
                gl = cd(0.0, n_sigma);
            } else {
                const double at = std::fabs(tau);
                gl = lesser_positive(eps_d, gamma, beta, bias_v, at);
                if (tau < 0.0) gl = -std::conj(gl);
            }
            const double at = std::fabs(tau);
            gg = gl - cd(0.0, 1.0) * std::exp(cd(-gamma * at, -eps_d * tau));
            tab[4 * j + 0] = gl.real();
            tab[4 * j + 1] = gl.imag();
            tab[4 * j + 2] = gg.real();
            tab[4 * j + 3] = gg.imag();
        }
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nt; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto &th : pool) th.join();
}

} // namespace qqmc
