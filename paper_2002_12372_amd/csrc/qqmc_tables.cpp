/*
 * qqmc_tables.cpp -- host side of the Green's-function tables (App. E):
 * n_sigma from the digamma closed form (arctan at zero temperature), and a
 * host build of the grid from the residue series of qqmc_gf.h (the device
 * build is tables_kernel) or, at zero temperature, from the deformed-contour
 * Fourier integral; semicircular leads of finite bandwidth by a graded
 * Gauss-Legendre rule over the band.
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

namespace {

/* Finite bandwidth (App. E, "Model"): semicircular leads of half-bandwidth
 * D, Delta(omega) = (Gamma/D)(omega - i sqrt(D^2 - omega^2)) in the band.
 * With |eps_d| < D - Gamma the retarded function has no pole outside the
 * band, and
 *     A(omega) = 2 g s / ((omega - eps_d - g omega)^2 + (g s)^2),
 *     g = Gamma/D, s = sqrt(D^2 - omega^2),
 *     g^<(tau) =  i Int A fbar     e^{-i omega tau} domega/2pi,
 *     g^>(tau) = -i Int A (1-fbar) e^{-i omega tau} domega/2pi
 * over the band.  Quadrature in theta, omega = -D cos theta (the band-edge
 * square roots become sin theta): 16-point Gauss-Legendre panels, split at
 * the Fermi levels and at eps_d, graded geometrically away from them (a
 * panel next to a Fermi level spans about four units of beta (omega - mu),
 * next to eps_d about Gamma), and never longer than about half a period of
 * e^{-i omega t_half}.  Both functions come from the same nodes. */
struct BandRule {
    std::vector<double> omega, weight, fbar; /* weight includes D sin theta A / 2pi */
    std::vector<double> measure;              /* the same without A                 */
};

BandRule band_rule(double eps_d, double gamma, double beta, double bias_v, double D,
                   double t_half)
{
    constexpr int M = 16;
    double gx[M], gw[M];
    legendre_rule(M, gx, gw);
    const double hmax = std::min(0.2, 3.0 / (D * t_half + 1.0));
    struct Mark {
        double theta, scale;
    };
    std::vector<Mark> marks;
    auto theta_of = [&](double w) { return std::acos(-w / D); };
    const double mus[2] = {0.5 * bias_v, -0.5 * bias_v};
    for (double mu : mus)
        if (std::fabs(mu) < D) {
            const double th = theta_of(mu), st = std::max(std::sin(th), 1e-3);
            marks.push_back({th, std::isinf(beta) ? hmax : 4.0 / (beta * D * st)});
        }
    if (std::fabs(eps_d) < D) {
        const double th = theta_of(eps_d), st = std::max(std::sin(th), 1e-3);
        marks.push_back({th, gamma / (D * st)});
    }
    std::vector<double> edges = {0.0, kPiGF};
    for (const Mark &m : marks) {
        edges.push_back(m.theta);
        const double d0 = std::min(m.scale, hmax);
        for (double d = d0; d < kPiGF; d *= 2.0) {
            edges.push_back(m.theta - d);
            edges.push_back(m.theta + d);
        }
    }
    std::vector<double> e;
    for (double x : edges)
        if (x >= 0.0 && x <= kPiGF) e.push_back(x);
    std::sort(e.begin(), e.end());
    BandRule r;
    const double g = gamma / D;
    for (size_t k = 0; k + 1 < e.size(); ++k) {
        const double a = e[k], b = e[k + 1];
        if (!(b - a > 1e-15)) continue;
        const int pieces = (int)std::ceil((b - a) / hmax);
        const double len = (b - a) / pieces;
        for (int p = 0; p < pieces; ++p) {
            const double lo = a + p * len, mid = lo + 0.5 * len;
            for (int i = 0; i < M; ++i) {
                const double th = mid + 0.5 * len * gx[i];
                const double w = -D * std::cos(th), s = D * std::sin(th);
                const double re = w - eps_d - g * w, im = g * s;
                const double A = 2.0 * g * s / (re * re + im * im);
                double fb;
                if (std::isinf(beta)) {
                    fb = 0.5 * ((w < mus[0] ? 1.0 : 0.0) + (w < mus[1] ? 1.0 : 0.0));
                } else {
                    auto fermi = [&](double x) {
                        const double bx = beta * x;
                        return bx > 0.0 ? std::exp(-bx) / (1.0 + std::exp(-bx))
                                        : 1.0 / (std::exp(bx) + 1.0);
                    };
                    fb = 0.5 * (fermi(w - mus[0]) + fermi(w - mus[1]));
                }
                r.omega.push_back(w);
                r.weight.push_back(0.5 * len * gw[i] * D * std::sin(th) * A / (2.0 * kPiGF));
                r.measure.push_back(0.5 * len * gw[i] * D * std::sin(th) / (2.0 * kPiGF));
                r.fbar.push_back(fb);
            }
        }
    }
    return r;
}

} // namespace

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

double build_tables_band(double eps_d, double gamma, double beta, double bias_v, double D,
                         int32_t n_grid, double t_half, double *tab)
{
    const BandRule r = band_rule(eps_d, gamma, beta, bias_v, D, t_half);
    const size_t m = r.omega.size();
    double n_sigma = 0.0;
    for (size_t k = 0; k < m; ++k) n_sigma += r.weight[k] * r.fbar[k];
    const double h = 2.0 * t_half / (n_grid - 1);
    unsigned nt = std::thread::hardware_concurrency();
    if (nt < 1) nt = 1;
    if (nt > 64) nt = 64;
    auto work = [&](unsigned tid) {
        for (int32_t j = (int32_t)tid; j < n_grid; j += (int32_t)nt) {
            const double tau = -t_half + j * h;
            /* sum over the nodes of weight * e^{-i omega tau}, split by fbar */
            double lr = 0.0, li = 0.0, gr = 0.0, gi = 0.0;
            for (size_t k = 0; k < m; ++k) {
                const double c = std::cos(r.omega[k] * tau), sn = -std::sin(r.omega[k] * tau);
                const double wl = r.weight[k] * r.fbar[k], wg = r.weight[k] - wl;
                lr += wl * c;
                li += wl * sn;
                gr += wg * c;
                gi += wg * sn;
            }
            /* g^< = i (lr + i li), g^> = -i (gr + i gi) */
            tab[4 * j + 0] = -li;
            tab[4 * j + 1] = lr;
            tab[4 * j + 2] = gi;
            tab[4 * j + 3] = -gr;
        }
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nt; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto &th : pool) th.join();
    return n_sigma;
}

void build_lead_tables(double eps_d, double gamma, double beta, double bias_v, double D,
                       int32_t lead, int32_t n_grid, double t_half, double *tab)
{
    /* gamma g^<_{0i} = conj(Delta)/2 g^< + Sigma^<_i g^R,
     * gamma g^>_{0i} = conj(Delta)/2 g^> + Sigma^>_i g^R, with
     * Sigma^<_i = -i f_i Im Delta, Sigma^>_i = i (1 - f_i) Im Delta, per node
     * of the band rule (its panels already meet both Fermi levels) */
    const BandRule r = band_rule(eps_d, gamma, beta, bias_v, D, t_half);
    const size_t m = r.omega.size();
    const double mu = lead == 1 ? -0.5 * bias_v : 0.5 * bias_v, g = gamma / D;
    std::vector<cd> vl(m), vg(m);
    for (size_t k = 0; k < m; ++k) {
        const double w = r.omega[k], sq = std::sqrt(std::max(D * D - w * w, 0.0));
        const cd delta(g * w, -g * sq);
        const cd gr = 1.0 / (w - eps_d - delta);
        const double A = -2.0 * gr.imag();
        double fi;
        if (std::isinf(beta)) {
            fi = w < mu ? 1.0 : 0.0;
        } else {
            const double bx = beta * (w - mu);
            fi = bx > 0.0 ? std::exp(-bx) / (1.0 + std::exp(-bx)) : 1.0 / (std::exp(bx) + 1.0);
        }
        const cd I(0.0, 1.0), half_conj = std::conj(delta) / 2.0;
        vl[k] = r.measure[k] * (half_conj * (I * A * r.fbar[k]) + (-I * fi * delta.imag()) * gr);
        vg[k] = r.measure[k] *
                (half_conj * (-I * A * (1.0 - r.fbar[k])) + (I * (1.0 - fi) * delta.imag()) * gr);
    }
    const double h = 2.0 * t_half / (n_grid - 1);
    unsigned nt = std::thread::hardware_concurrency();
    if (nt < 1) nt = 1;
    if (nt > 64) nt = 64;
    auto work = [&](unsigned tid) {
        for (int32_t j = (int32_t)tid; j < n_grid; j += (int32_t)nt) {
            const double tau = -t_half + j * h;
            cd sl(0.0, 0.0), sg(0.0, 0.0);
            for (size_t k = 0; k < m; ++k) {
                const cd e(std::cos(r.omega[k] * tau), -std::sin(r.omega[k] * tau));
                sl += vl[k] * e;
                sg += vg[k] * e;
            }
            tab[4 * j + 0] = sl.real();
            tab[4 * j + 1] = sl.imag();
            tab[4 * j + 2] = sg.real();
            tab[4 * j + 3] = sg.imag();
        }
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nt; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto &th : pool) th.join();
}

} // namespace qqmc
