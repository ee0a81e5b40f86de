/*
 * qqmc_oracle.c -- CPU FP64 oracle for the QQMC charge integrand of
 * arXiv:2002.12372.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product library.  It is
 * written for a reader holding the paper: plain loops, no blocking, no
 * fusion, one LU factorisation per determinant, every one of the 2^n Keldysh
 * index vectors enumerated.
 *
 * Conventions (readings of the paper, all listed in the design notes):
 *  - Keldysh Green's functions use the standard sign, g^< = +i <c^dag c>,
 *    so g^<(0) = i n_sigma.  The frequency-domain formulas printed in App. E
 *    carry an extra factor -2 relative to this; Q_0 = 1 at eps_d = 0 (main
 *    text, "Benchmark") fixes the standard normalisation.
 *  - Every equal-time (diagonal) Wick entry is g^<(0), whatever the Keldysh
 *    index; off-diagonal entries follow the 2x2 Keldysh rule of App. E with a
 *    strict inequality d > 0 for the time ordering.
 *  - With the alpha-shifted interaction U (n_up - alpha)(n_dn - alpha)
 *    (App. E, "Model"), the diagonal entry of every vertex is shifted by
 *    -i alpha, in both determinants; the measurement point's diagonal entry
 *    keeps g^<(0) (App. E, after the definition of the Wick determinant).
 *  - Q_n = -2 i^{n+1} * integral over 0 < u_n < ... < u_1 < t of S(u): the
 *    factor 2 is the spin sum of Q, the 1/n! of Eq. (integral_gf) is absorbed
 *    by restricting to the time-ordered simplex (S is symmetric).
 *  - The estimator is (C/N) sum_{i=0}^{N-1} f/p (Eq. (warped_int2) with the
 *    sum ending at N-1; App. B drops C, which is restored here).
 */
#define _GNU_SOURCE 1
#include "qqmc_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Non-interacting Green's functions (App. E, "Model" and
 * "Expressions for the integrands"): wide band, Delta(omega) = -i Gamma, so
 * the dot spectral function is the Lorentzian
 *     A(omega) = 2 Gamma / ((omega - eps_d)^2 + Gamma^2),
 * the symmetric bias V gives the mean occupation of the two leads
 *     fbar(omega) = [n_F(omega - V/2) + n_F(omega + V/2)] / 2,
 * and
 *     g^<(tau) =  i Int domega/2pi A fbar      e^{-i omega tau},
 *     g^>(tau) = -i Int domega/2pi A (1-fbar)  e^{-i omega tau}.
 * ------------------------------------------------------------------------ */

/* Fermi function of a complex argument, 1/(e^{beta z} + 1), written so that
 * the exponential never overflows. */
static cplx fermi_c(double beta, cplx z)
{
    cplx bz = beta * z;
    if (creal(bz) > 0.0) {
        cplx e = cexp(-bz);
        return e / (1.0 + e);
    }
    return 1.0 / (cexp(bz) + 1.0);
}

static double fermi_r(double beta, double x)
{
    double bx = beta * x;
    if (bx > 0.0) {
        double e = exp(-bx);
        return e / (1.0 + e);
    }
    return 1.0 / (exp(bx) + 1.0);
}

static cplx lorentz_c(double eps_d, double gamma, cplx z)
{
    cplx d = z - eps_d;
    return 2.0 * gamma / (d * d + gamma * gamma);
}

/* Matsubara part shared by both half-plane closures:
 *   sum_{k>=0} A(mu - i nu_k) e^{-nu_k tau},  nu_k = (2k+1) pi / beta,
 * for tau > 0.  Terms are added from the smallest (largest k) upwards. */
static cplx matsubara_sum(double eps_d, double gamma, double beta, double mu,
                          double tau)
{
    /* stop where e^{-nu_k tau} < e^{-45}; the terms also fall as 1/nu_k^2 */
    double nu_max = 45.0 / tau;
    long kmax = (long)ceil((nu_max * beta / M_PI - 1.0) / 2.0) + 1;
    if (kmax < 1) kmax = 1;
    double sr = 0.0, si = 0.0, cr = 0.0, ci = 0.0; /* Kahan, per component */
    for (long k = kmax; k >= 0; --k) {
        double nu = (2.0 * k + 1.0) * M_PI / beta;
        cplx term = lorentz_c(eps_d, gamma, mu - I * nu) * exp(-nu * tau);
        double y = creal(term) - cr, s = sr + y;
        cr = (s - sr) - y; sr = s;
        y = cimag(term) - ci; s = si + y;
        ci = (s - si) - y; si = s;
    }
    return sr + I * si;
}

/* For tau > 0 close the omega contour in the lower half plane.  Poles there:
 * the Lorentzian pole omega = eps_d - i Gamma (residue of A: i) and the Fermi
 * poles omega = mu - i nu_k (residue of n_F(omega - mu): -1/beta; residue of
 * 1 - n_F(omega - mu) = n_F(mu - omega): +1/beta).  This gives
 *   Int domega/2pi A n_F(omega-mu) e^{-i omega tau}
 *     = n_F(eps_d - mu - i Gamma) e^{-i eps_d tau - Gamma tau}
 *       + (i/beta) e^{-i mu tau} sum_k A(mu - i nu_k) e^{-nu_k tau},
 *   Int domega/2pi A (1 - n_F(omega-mu)) e^{-i omega tau}
 *     = n_F(mu - eps_d + i Gamma) e^{-i eps_d tau - Gamma tau}
 *       - (i/beta) e^{-i mu tau} sum_k A(mu - i nu_k) e^{-nu_k tau}. */
static void gf_positive_tau(double eps_d, double gamma, double beta,
                            double bias_v, double tau, cplx *glt, cplx *ggt)
{
    cplx lor = cexp(-I * eps_d * tau - gamma * tau);
    cplx sum_l = 0.0, sum_g = 0.0;
    for (int side = 0; side < 2; ++side) {
        double mu = side == 0 ? 0.5 * bias_v : -0.5 * bias_v;
        cplx ms = matsubara_sum(eps_d, gamma, beta, mu, tau);
        cplx ph = cexp(-I * mu * tau);
        sum_l += fermi_c(beta, eps_d - mu - I * gamma) * lor + (I / beta) * ph * ms;
        sum_g += fermi_c(beta, mu - eps_d + I * gamma) * lor - (I / beta) * ph * ms;
    }
    *glt = I * 0.5 * sum_l;
    *ggt = -I * 0.5 * sum_g;
}

/* Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_m. */
static void gauss_legendre(int m, double *x, double *w)
{
    for (int i = 0; i < m; ++i) {
        double z = cos(M_PI * (i + 0.75) / (m + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= m; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = m * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* ---- Zero temperature (beta = +infinity), App. E "Precision calculation":
 * the Fourier integrals Int zeta(omega) theta(mu - omega) e^{-i omega tau}
 * with zeta = A/2pi are taken along a deformed path.  For tau > 0 the factor
 * e^{-i omega tau} decays in the lower half plane, so the part of the real
 * axis left of a point c (chosen left of mu and of the pole eps_d - i Gamma,
 * none enclosed) is replaced by the vertical half-line c - i s, s >= 0:
 *   Int_{-inf}^{c} zeta e^{-i omega tau} d omega
 *       = i e^{-i c tau} Int_0^inf zeta(c - i s) e^{-s tau} ds,
 * and the remaining segment [c, mu] stays on the real axis.  The same with a
 * point right of mu gives the part above mu (for g^>):
 *   Int_{c}^{inf} zeta e^{-i omega tau} d omega
 *       = -i e^{-i c tau} Int_0^inf zeta(c - i s) e^{-s tau} ds.
 * Both integrals are composite Gauss-Legendre sums (panels of width 0.05 on
 * the real segment; geometrically growing panels on the half-line). */
static cplx zeta_c(double eps_d, double gamma, cplx w)
{
    cplx d = w - eps_d;
    return gamma / M_PI / (d * d + gamma * gamma);
}

static cplx segment_T0(double eps_d, double gamma, double a, double b, double tau)
{
    enum { M = 20 };
    double gx[M], gw[M];
    gauss_legendre(M, gx, gw);
    long panels = (long)ceil((b - a) / 0.05);
    if (panels < 1) panels = 1;
    double width = (b - a) / panels;
    cplx acc = 0.0;
    for (long p = 0; p < panels; ++p) {
        double lo = a + p * width;
        cplx part = 0.0;
        for (int q = 0; q < M; ++q) {
            double w = lo + 0.5 * width * (gx[q] + 1.0);
            part += gw[q] * zeta_c(eps_d, gamma, w) * cexp(-I * w * tau);
        }
        acc += 0.5 * width * part;
    }
    return acc;
}

/* Int_0^inf zeta(c - i s) e^{-s tau} ds */
static cplx halfline_T0(double eps_d, double gamma, double c, double tau)
{
    enum { M = 20 };
    double gx[M], gw[M];
    gauss_legendre(M, gx, gw);
    double smax = 60.0 / tau, lo = 0.0, width = 0.05 < 0.5 / tau ? 0.05 : 0.5 / tau;
    cplx acc = 0.0;
    while (lo < smax) {
        cplx part = 0.0;
        for (int q = 0; q < M; ++q) {
            double s = lo + 0.5 * width * (gx[q] + 1.0);
            part += gw[q] * zeta_c(eps_d, gamma, c - I * s) * exp(-s * tau);
        }
        acc += 0.5 * width * part;
        lo += width;
        width *= 1.25;
    }
    return acc;
}

static void gf_positive_tau_T0(double eps_d, double gamma, double bias_v, double tau,
                               cplx *glt, cplx *ggt)
{
    cplx sum_l = 0.0, sum_g = 0.0;
    for (int side = 0; side < 2; ++side) {
        double mu = side == 0 ? 0.5 * bias_v : -0.5 * bias_v;
        double cl = (mu < eps_d ? mu : eps_d) - gamma - 1.0;
        double cr = (mu > eps_d ? mu : eps_d) + gamma + 1.0;
        cplx below = I * cexp(-I * cl * tau) * halfline_T0(eps_d, gamma, cl, tau) +
                     segment_T0(eps_d, gamma, cl, mu, tau);
        cplx above = segment_T0(eps_d, gamma, mu, cr, tau) -
                     I * cexp(-I * cr * tau) * halfline_T0(eps_d, gamma, cr, tau);
        sum_l += below;
        sum_g += above;
    }
    *glt = I * 0.5 * sum_l;
    *ggt = -I * 0.5 * sum_g;
}

/* n(mu) = Int domega/2pi A(omega) n_F(omega - mu), written as the exact
 * zero-temperature part plus an exponentially convergent remainder:
 *   n(mu) = 1/2 + atan((mu - eps_d)/Gamma)/pi
 *           + (1/2pi) Int_0^inf [A(mu + x) - A(mu - x)] n_F(x) dx. */
static double occupation_one_lead(double eps_d, double gamma, double beta,
                                  double mu)
{
    enum { M = 20 };
    double gx[M], gw[M];
    gauss_legendre(M, gx, gw);
    double xmax = 45.0 / beta;
    double feature = gamma < 1.0 / beta ? gamma : 1.0 / beta;
    long panels = (long)ceil(xmax / (0.25 * feature));
    if (panels < 8) panels = 8;
    double width = xmax / panels, acc = 0.0;
    for (long p = 0; p < panels; ++p) {
        double a = p * width, part = 0.0;
        for (int q = 0; q < M; ++q) {
            double x = a + 0.5 * width * (gx[q] + 1.0);
            double ap = 2.0 * gamma / ((mu + x - eps_d) * (mu + x - eps_d) + gamma * gamma);
            double am = 2.0 * gamma / ((mu - x - eps_d) * (mu - x - eps_d) + gamma * gamma);
            part += gw[q] * (ap - am) * fermi_r(beta, x);
        }
        acc += 0.5 * width * part;
    }
    return 0.5 + atan((mu - eps_d) / gamma) / M_PI + acc / (2.0 * M_PI);
}

double oracle_n_sigma(double eps_d, double gamma, double beta, double bias_v)
{
    if (isinf(beta))
        return 0.5 * (1.0 + (atan((0.5 * bias_v - eps_d) / gamma) +
                             atan((-0.5 * bias_v - eps_d) / gamma)) / M_PI);
    return 0.5 * (occupation_one_lead(eps_d, gamma, beta, 0.5 * bias_v) +
                  occupation_one_lead(eps_d, gamma, beta, -0.5 * bias_v));
}

void oracle_gf_direct(double eps_d, double gamma, double beta, double bias_v,
                      double tau, double *out)
{
    cplx l, g;
    if (tau != 0.0) {
        if (isinf(beta))
            gf_positive_tau_T0(eps_d, gamma, bias_v, fabs(tau), &l, &g);
        else
            gf_positive_tau(eps_d, gamma, beta, bias_v, fabs(tau), &l, &g);
        if (tau < 0.0) {
            /* g(-tau) = -conj(g(tau)): the Fourier integral of i * (real
             * spectral weight) is hermitian in this sense. */
            l = -conj(l);
            g = -conj(g);
        }
    } else {
        double ns = oracle_n_sigma(eps_d, gamma, beta, bias_v);
        l = I * ns;
        g = I * (ns - 1.0);
    }
    out[0] = creal(l); out[1] = cimag(l);
    out[2] = creal(g); out[3] = cimag(g);
}

int oracle_tables(double eps_d, double gamma, double beta, double bias_v,
                  int n_grid, double t_half,
                  double *gl, double *gg, double *n_sigma)
{
    if (n_grid < 2 || !(t_half > 0.0) || !(gamma > 0.0) || !(beta > 0.0))
        return -1;
    double h = 2.0 * t_half / (n_grid - 1);
    double ns = oracle_n_sigma(eps_d, gamma, beta, bias_v);
    #pragma omp parallel for schedule(dynamic, 8)
    for (int j = 0; j < n_grid; ++j) {
        double tau = -t_half + j * h;
        double v[4];
        if (tau == 0.0) {
            v[0] = 0.0; v[1] = ns; v[2] = 0.0; v[3] = ns - 1.0;
        } else {
            oracle_gf_direct(eps_d, gamma, beta, bias_v, tau, v);
        }
        gl[2 * j] = v[0]; gl[2 * j + 1] = v[1];
        gg[2 * j] = v[2]; gg[2 * j + 1] = v[3];
    }
    *n_sigma = ns;
    return 0;
}

/* ---- Finite bandwidth (App. E, "Model"): each lead has a semicircular
 * density of states of half-bandwidth D; with Gamma = 4 gamma^2 / D the
 * hybridisation inside the band is
 *     Delta(omega) = (Gamma/D) (omega - i sqrt(D^2 - omega^2)),
 * real outside.  The retarded function 1/(omega - eps_d - Delta) has no pole
 * outside the band when |eps_d| < D - Gamma (then the band carries the whole
 * spectral weight; the paper's frequency formulas have no bound-state
 * terms, and this oracle accepts only that regime).  The spectral function
 *     A(omega) = 2 (Gamma/D) s |g^R|^2,  s = sqrt(D^2 - omega^2),
 *     |g^R|^2 = 1 / ((omega - eps_d - (Gamma/D) omega)^2 + (Gamma s / D)^2),
 * and, with fbar the mean Fermi function of the two leads,
 *     g^<(tau) =  i Int_{-D}^{D} A fbar      e^{-i omega tau} domega / 2pi,
 *     g^>(tau) = -i Int_{-D}^{D} A (1-fbar)  e^{-i omega tau} domega / 2pi.
 * The integrals run over theta in [0, pi] with omega = -D cos theta (the
 * square roots at the band edges become sin theta), split at the Fermi
 * levels and the level eps_d, each piece by adaptive Gauss-Legendre. */
typedef struct {
    double eps_d, gamma, beta, bias_v, D, tau;
    int lesser;
} band_ctx;

/* Fermi function with the T = 0 step (1/2 at the step itself) */
static double fermi_band(double beta, double x)
{
    if (isinf(beta)) return x < 0.0 ? 1.0 : (x > 0.0 ? 0.0 : 0.5);
    double bx = beta * x;
    if (bx > 0.0) {
        double e = exp(-bx);
        return e / (1.0 + e);
    }
    return 1.0 / (exp(bx) + 1.0);
}

static double band_spectral(double eps_d, double gamma, double D, double omega)
{
    double s2 = D * D - omega * omega;
    if (s2 <= 0.0) return 0.0;
    double s = sqrt(s2), g = gamma / D;
    double re = omega - eps_d - g * omega, im = g * s;
    return 2.0 * g * s / (re * re + im * im);
}

static cplx band_integrand(const band_ctx *c, double theta)
{
    double omega = -c->D * cos(theta);
    double A = band_spectral(c->eps_d, c->gamma, c->D, omega);
    double fb = 0.5 * (fermi_band(c->beta, omega - 0.5 * c->bias_v) +
                       fermi_band(c->beta, omega + 0.5 * c->bias_v));
    double wgt = c->lesser ? fb : 1.0 - fb;
    return A * wgt * cexp(-I * omega * c->tau) * c->D * sin(theta) / (2.0 * M_PI);
}

static cplx band_gl(const band_ctx *c, double a, double b, const double *gx, const double *gw,
                    int m)
{
    double hw = 0.5 * (b - a), mid = 0.5 * (a + b);
    cplx acc = 0.0;
    for (int i = 0; i < m; ++i) acc += gw[i] * band_integrand(c, mid + hw * gx[i]);
    return hw * acc;
}

/* Adaptive bisection: accept the two halves when they agree with the whole
 * piece to 1e-14 per unit of theta (at most about 3e-14 in all), or to the
 * rounding level of the halves themselves. */
static cplx band_adapt(const band_ctx *c, double a, double b, cplx whole, int depth,
                       const double *gx, const double *gw, int m)
{
    double mid = 0.5 * (a + b);
    cplx l = band_gl(c, a, mid, gx, gw, m), r = band_gl(c, mid, b, gx, gw, m);
    double diff = cabs(l + r - whole);
    if (depth >= 30 || diff <= 1e-14 * (b - a) || diff <= 1e-15 * (cabs(l) + cabs(r)))
        return l + r;
    return band_adapt(c, a, mid, l, depth + 1, gx, gw, m) +
           band_adapt(c, mid, b, r, depth + 1, gx, gw, m);
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* g^< (lesser = 1) or g^> at tau, finite bandwidth. */
static cplx band_gf(double eps_d, double gamma, double beta, double bias_v, double D,
                    double tau, int lesser)
{
    enum { M = 10 };
    double gx[M], gw[M];
    gauss_legendre(M, gx, gw);
    band_ctx c = { eps_d, gamma, beta, bias_v, D, tau, lesser };
    double br[5];
    int nb = 0;
    br[nb++] = 0.0;
    double pts[3] = { 0.5 * bias_v, -0.5 * bias_v, eps_d };
    for (int k = 0; k < 3; ++k)
        if (fabs(pts[k]) < D) br[nb++] = acos(-pts[k] / D);
    br[nb++] = M_PI;
    qsort(br, (size_t)nb, sizeof(double), cmp_double);
    cplx total = 0.0;
    for (int k = 0; k + 1 < nb; ++k) {
        double a = br[k], b = br[k + 1];
        if (!(b > a)) continue;
        cplx whole = band_gl(&c, a, b, gx, gw, M);
        total += band_adapt(&c, a, b, whole, 0, gx, gw, M);
    }
    return (lesser ? I : -I) * total;
}

static int band_ok(double eps_d, double gamma, double beta, double D)
{
    return D > 0.0 && isfinite(D) && gamma > 0.0 && beta > 0.0 && fabs(eps_d) < D - gamma;
}

double oracle_n_sigma_band(double eps_d, double gamma, double beta, double bias_v, double D)
{
    if (!band_ok(eps_d, gamma, beta, D)) return NAN;
    return cimag(band_gf(eps_d, gamma, beta, bias_v, D, 0.0, 1));
}

void oracle_gf_band(double eps_d, double gamma, double beta, double bias_v, double D,
                    double tau, double *out)
{
    cplx l = band_gf(eps_d, gamma, beta, bias_v, D, tau, 1);
    cplx g = band_gf(eps_d, gamma, beta, bias_v, D, tau, 0);
    out[0] = creal(l); out[1] = cimag(l);
    out[2] = creal(g); out[3] = cimag(g);
}

int oracle_tables_band(double eps_d, double gamma, double beta, double bias_v, double D,
                       int n_grid, double t_half, double *gl, double *gg, double *n_sigma)
{
    if (n_grid < 2 || !(t_half > 0.0) || !band_ok(eps_d, gamma, beta, D)) return -1;
    double h = 2.0 * t_half / (n_grid - 1);
    #pragma omp parallel for schedule(dynamic, 8)
    for (int j = 0; j < n_grid; ++j) {
        double tau = -t_half + j * h, v[4];
        oracle_gf_band(eps_d, gamma, beta, bias_v, D, tau, v);
        gl[2 * j] = v[0]; gl[2 * j + 1] = v[1];
        gg[2 * j] = v[2]; gg[2 * j + 1] = v[3];
    }
    *n_sigma = oracle_n_sigma_band(eps_d, gamma, beta, bias_v, D);
    return 0;
}

/* Lead Green's functions for the current (finite bandwidth only): with lead
 * i at chemical potential mu_i (lead 1: -V/2, lead 2: +V/2) and self-energy
 * Sigma_i = Delta/2, the dot-lead function g_{0i} = g_{00} gamma G_i gives
 * (Langreth rules)
 *     gamma g^<_{0i} = conj(Delta)/2 g^<_{00} + Sigma^<_i g^R,
 *     gamma g^>_{0i} = conj(Delta)/2 g^>_{00} + Sigma^>_i g^R,
 *     Sigma^<_i = -i f_i Im Delta,  Sigma^>_i = i (1 - f_i) Im Delta,
 * all inside the band (no bound state).  Same theta quadrature as above. */
typedef struct {
    double eps_d, gamma, beta, bias_v, D, tau, mu;
    int lesser;
} lead_ctx;

static cplx lead_integrand(const lead_ctx *c, double theta)
{
    double omega = -c->D * cos(theta);
    double s = c->D * sin(theta), g = c->gamma / c->D;
    cplx delta = g * omega - I * g * s;
    cplx gr = 1.0 / (omega - c->eps_d - delta);
    double A = -2.0 * cimag(gr);
    double fb = 0.5 * (fermi_band(c->beta, omega - 0.5 * c->bias_v) +
                       fermi_band(c->beta, omega + 0.5 * c->bias_v));
    double fi = fermi_band(c->beta, omega - c->mu);
    cplx v;
    if (c->lesser)
        v = conj(delta) / 2.0 * (I * A * fb) + (-I * fi * cimag(delta)) * gr;
    else
        v = conj(delta) / 2.0 * (-I * A * (1.0 - fb)) + (I * (1.0 - fi) * cimag(delta)) * gr;
    return v * cexp(-I * omega * c->tau) * s / (2.0 * M_PI);
}

static cplx lead_gl(const lead_ctx *c, double a, double b, const double *gx, const double *gw,
                    int m)
{
    double hw = 0.5 * (b - a), mid = 0.5 * (a + b);
    cplx acc = 0.0;
    for (int i = 0; i < m; ++i) acc += gw[i] * lead_integrand(c, mid + hw * gx[i]);
    return hw * acc;
}

static cplx lead_adapt(const lead_ctx *c, double a, double b, cplx whole, int depth,
                       const double *gx, const double *gw, int m)
{
    double mid = 0.5 * (a + b);
    cplx l = lead_gl(c, a, mid, gx, gw, m), r = lead_gl(c, mid, b, gx, gw, m);
    double diff = cabs(l + r - whole);
    if (depth >= 30 || diff <= 1e-14 * (b - a) || diff <= 1e-15 * (cabs(l) + cabs(r)))
        return l + r;
    return lead_adapt(c, a, mid, l, depth + 1, gx, gw, m) +
           lead_adapt(c, mid, b, r, depth + 1, gx, gw, m);
}

void oracle_gf_lead(double eps_d, double gamma, double beta, double bias_v, double D, int lead,
                    double tau, double *out)
{
    enum { M = 10 };
    double gx[M], gw[M];
    gauss_legendre(M, gx, gw);
    double br[5];
    int nb = 0;
    br[nb++] = 0.0;
    double pts[3] = { 0.5 * bias_v, -0.5 * bias_v, eps_d };
    for (int k = 0; k < 3; ++k)
        if (fabs(pts[k]) < D) br[nb++] = acos(-pts[k] / D);
    br[nb++] = M_PI;
    qsort(br, (size_t)nb, sizeof(double), cmp_double);
    for (int which = 0; which < 2; ++which) {
        lead_ctx c = { eps_d, gamma, beta, bias_v, D, tau, lead == 1 ? -0.5 * bias_v : 0.5 * bias_v,
                       which == 0 };
        cplx total = 0.0;
        for (int k = 0; k + 1 < nb; ++k) {
            double a = br[k], b = br[k + 1];
            if (!(b > a)) continue;
            total += lead_adapt(&c, a, b, lead_gl(&c, a, b, gx, gw, M), 0, gx, gw, M);
        }
        out[2 * which] = creal(total);
        out[2 * which + 1] = cimag(total);
    }
}

int oracle_lead_tables(double eps_d, double gamma, double beta, double bias_v, double D,
                       int lead, int n_grid, double t_half, double *cl, double *cg)
{
    if (n_grid < 2 || !(t_half > 0.0) || !band_ok(eps_d, gamma, beta, D) ||
        (lead != 1 && lead != 2))
        return -1;
    double h = 2.0 * t_half / (n_grid - 1);
    #pragma omp parallel for schedule(dynamic, 8)
    for (int j = 0; j < n_grid; ++j) {
        double v[4];
        oracle_gf_lead(eps_d, gamma, beta, bias_v, D, lead, -t_half + j * h, v);
        cl[2 * j] = v[0]; cl[2 * j + 1] = v[1];
        cg[2 * j] = v[2]; cg[2 * j + 1] = v[3];
    }
    return 0;
}

/* Linear interpolation on the uniform grid; outside the grid the end value is
 * held (the index and the fraction are both clamped). */
static cplx interp_c(const double *tab, int n_grid, double t_half, double tau)
{
    double h = 2.0 * t_half / (n_grid - 1);
    double s = (tau + t_half) / h;
    double fl = floor(s);
    long j = (long)fl;
    if (j < 0) j = 0;
    if (j > n_grid - 2) j = n_grid - 2;
    double phi = s - (double)j;
    if (phi < 0.0) phi = 0.0;
    if (phi > 1.0) phi = 1.0;
    cplx a = tab[2 * j] + I * tab[2 * j + 1];
    cplx b = tab[2 * j + 2] + I * tab[2 * j + 3];
    return (1.0 - phi) * a + phi * b;
}

void oracle_interp(const double *tab, int n_grid, double t_half, double tau,
                   double *out)
{
    cplx v = interp_c(tab, n_grid, t_half, tau);
    out[0] = creal(v); out[1] = cimag(v);
}

/* ------------------------------------------------------------------------ */
/* Determinants (textbook LU with partial pivoting).                        */
/* ------------------------------------------------------------------------ */
static cplx det_lu(int m, cplx *a /* m*m, destroyed */)
{
    cplx det = 1.0;
    for (int k = 0; k < m; ++k) {
        int piv = k;
        double best = cabs(a[k * m + k]);
        for (int r = k + 1; r < m; ++r) {
            double v = cabs(a[r * m + k]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return 0.0;
        if (piv != k) {
            for (int c = 0; c < m; ++c) {
                cplx t = a[k * m + c];
                a[k * m + c] = a[piv * m + c];
                a[piv * m + c] = t;
            }
            det = -det;
        }
        cplx p = a[k * m + k];
        det *= p;
        for (int r = k + 1; r < m; ++r) {
            cplx f = a[r * m + k] / p;
            for (int c = k + 1; c < m; ++c) a[r * m + c] -= f * a[k * m + c];
        }
    }
    return det;
}

void oracle_det(int m, const double *a, double *out)
{
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)(m > 0 ? m * m : 1));
    for (int i = 0; i < m * m; ++i) w[i] = a[2 * i] + I * a[2 * i + 1];
    cplx d = m > 0 ? det_lu(m, w) : 1.0;
    free(w);
    out[0] = creal(d); out[1] = cimag(d);
}

/* ------------------------------------------------------------------------ */
/* Wick matrices of Eq. (integral_gf) with the Keldysh 2x2 rule of App. E:  */
/*   g[(u,a),(u',a')] = [[g^T, g^<], [g^>, g^Tbar]]_{a a'} at d = u - u',    */
/*   g^T(d) = d > 0 ? g^>(d) : g^<(d),  g^Tbar(d) = d > 0 ? g^<(d) : g^>(d). */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;            /* number of vertices                                 */
    cplx g0;          /* vertex diagonal g^<(0) - i alpha = i (n_sigma - alpha) */
    cplx gm;          /* measurement diagonal g^<(0) = i n_sigma             */
    const cplx *gl_d; /* (n+1)^2: g^<(tau_r - tau_c), point 0 = measurement  */
    const cplx *gg_d; /* (n+1)^2: g^>(tau_r - tau_c)                         */
    const double *tm; /* (n+1): times, tm[0] = t, tm[k] = u_k                */
    /* current: the measurement column (i, t, 1) is a lead site; cl_d[r],
     * cg_d[r] hold gamma g^<_{0i}, gamma g^>_{0i} at tau_r - t (NULL: the
     * charge, column from the dot's own functions) */
    const cplx *cl_d, *cg_d;
} wick_ctx;

static cplx keldysh_entry(const wick_ctx *w, int r, int a_r, int c, int a_c)
{
    int np1 = w->n + 1;
    double d = w->tm[r] - w->tm[c];
    cplx gl = w->gl_d[r * np1 + c], gg = w->gg_d[r * np1 + c];
    if (c == 0 && w->cl_d) {
        gl = w->cl_d[r];
        gg = w->cg_d[r];
    }
    if (a_r == 0 && a_c == 0) return d > 0.0 ? gg : gl;
    if (a_r == 0 && a_c == 1) return gl;
    if (a_r == 1 && a_c == 0) return gg;
    return d > 0.0 ? gl : gg;
}

/* Spin-up matrix: rows (0,t,0), U_1..U_n; columns (0,t,1), U_1..U_n. */
static void build_up(const wick_ctx *w, const int *a, cplx *m)
{
    int np1 = w->n + 1;
    for (int r = 0; r < np1; ++r) {
        for (int c = 0; c < np1; ++c) {
            if (r == c) {
                /* the corner (0,t,0)-(i,t,1) is the lead function at 0 for the
                 * current; it cancels from the Keldysh sum in any case */
                m[r * np1 + c] = r == 0 ? (w->cl_d ? w->cl_d[0] : w->gm) : w->g0;
                continue;
            }
            int ar = r == 0 ? 0 : a[r - 1];
            int ac = c == 0 ? 1 : a[c - 1];
            m[r * np1 + c] = keldysh_entry(w, r, ar, c, ac);
        }
    }
}

static void fill_pair_values(const double *gl, const double *gg, int n_grid,
                             double t_half, int n, const double *tm,
                             cplx *gl_d, cplx *gg_d)
{
    int np1 = n + 1;
    for (int r = 0; r < np1; ++r)
        for (int c = 0; c < np1; ++c) {
            double d = tm[r] - tm[c];
            gl_d[r * np1 + c] = interp_c(gl, n_grid, t_half, d);
            gg_d[r * np1 + c] = interp_c(gg, n_grid, t_half, d);
        }
}

void oracle_wick_matrix(const double *gl, const double *gg, int n_grid,
                        double t_half, double n_sigma, double alpha, double t_meas,
                        int n, const double *u, const int *a, double *out)
{
    int np1 = n + 1;
    double *tm = (double *)malloc(sizeof(double) * np1);
    cplx *gl_d = (cplx *)malloc(sizeof(cplx) * np1 * np1);
    cplx *gg_d = (cplx *)malloc(sizeof(cplx) * np1 * np1);
    cplx *m = (cplx *)malloc(sizeof(cplx) * np1 * np1);
    tm[0] = t_meas;
    for (int k = 0; k < n; ++k) tm[k + 1] = u[k];
    fill_pair_values(gl, gg, n_grid, t_half, n, tm, gl_d, gg_d);
    wick_ctx w = { n, I * (n_sigma - alpha), I * n_sigma, gl_d, gg_d, tm, NULL, NULL };
    build_up(&w, a, m);
    for (int i = 0; i < np1 * np1; ++i) {
        out[2 * i] = creal(m[i]);
        out[2 * i + 1] = cimag(m[i]);
    }
    free(tm); free(gl_d); free(gg_d); free(m);
}

/* S(u) of Eq. (integral_gf): sum over a in {0,1}^n, natural binary order
 * (bit k-1 of the counter is a_k), of (-1)^{sum a} det_up(a) det_dn(a),
 * where det_dn is the vertex block (rows/columns 1..n) of the up matrix. */
/* S(u) with the measurement column from a lead's tables (cl, cg: gamma
 * g^<_{0i}, gamma g^>_{0i} on the same grid), or from the dot's (cl = NULL). */
void oracle_keldysh_sum_lead(const double *gl, const double *gg, const double *cl,
                             const double *cg, int n_grid, double t_half, double n_sigma,
                             double alpha, double t_meas, int n, const double *u,
                             double *S_out, double *M_out)
{
    int np1 = n + 1;
    double tm[32];
    cplx gl_d[32 * 32], gg_d[32 * 32], up[32 * 32], dn[32 * 32], cl_d[32], cg_d[32];
    int a[32];
    tm[0] = t_meas;
    for (int k = 0; k < n; ++k) tm[k + 1] = u[k];
    fill_pair_values(gl, gg, n_grid, t_half, n, tm, gl_d, gg_d);
    if (cl) {
        for (int r = 0; r < np1; ++r) {
            cl_d[r] = interp_c(cl, n_grid, t_half, tm[r] - t_meas);
            cg_d[r] = interp_c(cg, n_grid, t_half, tm[r] - t_meas);
        }
    }
    wick_ctx w = { n, I * (n_sigma - alpha), I * n_sigma, gl_d, gg_d, tm,
                   cl ? cl_d : NULL, cl ? cg_d : NULL };
    double sr = 0.0, si = 0.0, cr = 0.0, ci = 0.0, mass = 0.0;
    for (long mask = 0; mask < (1L << n); ++mask) {
        int parity = 0;
        for (int k = 0; k < n; ++k) {
            a[k] = (int)((mask >> k) & 1L);
            parity ^= a[k];
        }
        build_up(&w, a, up);
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) dn[r * n + c] = up[(r + 1) * np1 + (c + 1)];
        cplx d_up = det_lu(np1, up);
        cplx d_dn = det_lu(n, dn);
        cplx term = d_up * d_dn;
        if (parity) term = -term;
        mass += cabs(term);
        double y = creal(term) - cr, s = sr + y;
        cr = (s - sr) - y; sr = s;
        y = cimag(term) - ci; s = si + y;
        ci = (s - si) - y; si = s;
    }
    S_out[0] = sr; S_out[1] = si;
    *M_out = mass;
}

void oracle_keldysh_sum(const double *gl, const double *gg, int n_grid,
                        double t_half, double n_sigma, double alpha, double t_meas,
                        int n, const double *u, double *S_out, double *M_out)
{
    oracle_keldysh_sum_lead(gl, gg, NULL, NULL, n_grid, t_half, n_sigma, alpha, t_meas, n, u,
                            S_out, M_out);
}

/* ------------------------------------------------------------------------ */
/* Points: randomly shifted rank-1 lattice (randomised QMC, App. G) and the  */
/* product-model warping (Eqs. (warper1d), (x_of_v_simple), (hi_expo)).     */
/* ------------------------------------------------------------------------ */
void oracle_lattice_point(uint64_t i, int n, int log2_n, uint64_t lattice_a,
                          const double *shift, double *x)
{
    uint64_t N = (uint64_t)1 << log2_n, z = 1 % N;
    for (int j = 0; j < n; ++j) {
        uint64_t m = (i * z) % N;
        double y = (double)m / (double)N + shift[j];
        if (y >= 1.0) y -= 1.0;
        x[j] = y;
        z = (z * lattice_a) % N;
    }
}

/* x_m(v_m) = Int_0^{v_m} h / Int_0^inf h = 1 - e^{-v_m/tau} for
 * h(v) = e^{-v/tau}, so v_m = -tau log(1 - x_m); u_0 = t, u_m = u_{m-1} - v_m;
 * p_n(u) = prod_m h(u_{m-1} - u_m); C = Int_{[0,inf)^n} p_n dv = tau^n;
 * the Jacobian |du/dx| = C/p_n(u) (App. D). */
int oracle_warp(int n, const double *x, double model_tau, double t_meas,
                double *u, double *W)
{
    double prev = t_meas, p = 1.0, c = 1.0;
    for (int m = 0; m < n; ++m) {
        double v = -model_tau * log1p(-x[m]);
        u[m] = prev - v;
        p *= exp(-(prev - u[m]) / model_tau);
        prev = u[m];
        c *= model_tau;
    }
    *W = c / p;
    return u[n - 1] > 0.0 ? 1 : 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

double oracle_model_inverse(const double *cdf, int n_bins, double x, double *w)
{
    int b = 0;
    for (int k = 1; k < n_bins; ++k)
        if (cdf[k] <= x) b = k;
    const double width = cdf[b + 1] - cdf[b];
    *w = ((double)b + (x - cdf[b]) / width) / (double)n_bins;
    return (double)n_bins * width;
}

int oracle_model_from_hist(int n, int n_bins, const double *hist, double lambda,
                           double floor_eps, double *cdf)
{
    if (n < 1 || n_bins < 1 || !(lambda > 0.0) || !(floor_eps >= 0.0) || !(floor_eps <= 1.0))
        return -1;
    double *sm = (double *)malloc(sizeof(double) * (size_t)n_bins);
    if (!sm) return -1;
    for (int j = 0; j < n; ++j) {
        const double *h = hist + (size_t)j * n_bins;
        /* Gaussian kernel smoothing K(w, w') = exp(-(w - w')^2 / lambda^2)
         * over the bin centres, normalised by the kernel weights */
        double total = 0.0;
        for (int b = 0; b < n_bins; ++b) {
            const double wb = (b + 0.5) / n_bins;
            double num = 0.0, den = 0.0;
            for (int k = 0; k < n_bins; ++k) {
                const double d = (wb - (k + 0.5) / n_bins) / lambda;
                const double K = exp(-d * d);
                num += K * h[k];
                den += K;
            }
            sm[b] = num / den;
            total += sm[b] / n_bins;
        }
        double *c = cdf + (size_t)j * (n_bins + 1);
        c[0] = 0.0;
        for (int b = 0; b < n_bins; ++b) {
            const double p = total > 0.0 ? sm[b] / total : 1.0;
            const double q = (1.0 - floor_eps) * p + floor_eps;
            c[b + 1] = c[b] + q / n_bins;
        }
        const double end = c[n_bins];
        for (int b = 1; b < n_bins; ++b) c[b] /= end;
        c[n_bins] = 1.0;
    }
    free(sm);
    return 0;
}

/* The first warp followed by the learned one: x -> w -> (u, W). */
static int warp_model(int n, const double *x, const double *cdf, int n_bins,
                      double model_tau, double t_meas, double *u, double *W,
                      double *qprod)
{
    double w[32];
    double q = 1.0;
    for (int j = 0; j < n; ++j) {
        if (cdf)
            q *= oracle_model_inverse(cdf + (size_t)j * (n_bins + 1), n_bins, x[j], &w[j]);
        else
            w[j] = x[j];
    }
    const int inside = oracle_warp(n, w, model_tau, t_meas, u, W);
    *W /= q;
    *qprod = q;
    return inside;
}

/* Sobol' point i with a random digital shift (App. B): coordinate j is
 * (XOR over the set bits k of i of V[j][k]) XOR dshift[j], times 2^-32. */
void oracle_sobol_point(uint64_t i, int n, const uint32_t *V, const uint32_t *dshift, double *x)
{
    for (int j = 0; j < n; ++j) {
        uint32_t v = dshift ? dshift[j] : 0u;
        for (int k = 0; k < 32; ++k)
            if ((i >> k) & 1u) v ^= V[j * 32 + k];
        x[j] = (double)v * (1.0 / 4294967296.0);
    }
}

/* The estimator over the lattice (sobol_v == NULL) or over Sobol' points
 * (sobol_v: n x 32 direction numbers, sobol_shifts: n_shifts x n words). */
static int eval_sums_core(const double *gl, const double *gg, int n_grid,
                          double t_half, double n_sigma, double alpha, double t_meas,
                          int n, int log2_n, uint64_t lattice_a,
                          int n_shifts, const double *shifts, const uint32_t *sobol_v,
                          const uint32_t *sobol_shifts, double model_tau,
                          const double *cdf, int n_bins,
                          int mode, int64_t i_begin, int64_t i_end, int n_threads,
                          double *sums)
{
    if (n < 1 || n > 24 || log2_n < 1 || log2_n > 40 || i_end < i_begin ||
        i_begin < 0 || n_shifts < 1 || mode < 0 || mode > 2 || (cdf && n_bins < 1))
        return -1;
    int64_t cnt = i_end - i_begin;
    double *vals = (double *)malloc(sizeof(double) * 2 * (size_t)(cnt > 0 ? cnt : 1));
    if (!vals) return -1;
    int nt = n_threads > 0 ? n_threads : oracle_max_threads();
    /* i^{n+1} */
    cplx ipow = 1.0;
    for (int k = 0; k < n + 1; ++k) ipow *= I;
    for (int s = 0; s < n_shifts; ++s) {
        const double *sh = sobol_v ? NULL : shifts + (size_t)s * n;
        #pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
        for (int64_t q = 0; q < cnt; ++q) {
            double x[32], u[32], W, S[2], M, qp;
            if (sobol_v)
                oracle_sobol_point((uint64_t)(i_begin + q), n, sobol_v,
                                   sobol_shifts + (size_t)s * n, x);
            else
                oracle_lattice_point((uint64_t)(i_begin + q), n, log2_n, lattice_a, sh, x);
            int inside = warp_model(n, x, cdf, n_bins, model_tau, t_meas, u, &W, &qp);
            cplx f = 0.0;
            if (mode == 1) {
                /* f := p_n q on the whole v-domain: f W = C */
                double p = 1.0, prev = t_meas;
                for (int m = 0; m < n; ++m) {
                    p *= exp(-(prev - u[m]) / model_tau);
                    prev = u[m];
                }
                f = p * qp * W;
            } else if (inside) {
                if (mode == 2) {
                    f = W;
                } else {
                    oracle_keldysh_sum(gl, gg, n_grid, t_half, n_sigma, alpha, t_meas,
                                       n, u, S, &M);
                    f = -2.0 * ipow * (S[0] + I * S[1]) * W;
                }
            }
            vals[2 * q] = creal(f);
            vals[2 * q + 1] = cimag(f);
        }
        double sr = 0.0, si = 0.0, cr = 0.0, ci = 0.0;
        for (int64_t q = 0; q < cnt; ++q) {
            double y = vals[2 * q] - cr, t = sr + y;
            cr = (t - sr) - y; sr = t;
            y = vals[2 * q + 1] - ci; t = si + y;
            ci = (t - si) - y; si = t;
        }
        sums[2 * s] = sr;
        sums[2 * s + 1] = si;
    }
    free(vals);
    return 0;
}

int oracle_eval_sums_model(const double *gl, const double *gg, int n_grid,
                           double t_half, double n_sigma, double alpha, double t_meas,
                           int n, int log2_n, uint64_t lattice_a,
                           int n_shifts, const double *shifts, double model_tau,
                           const double *cdf, int n_bins,
                           int mode, int64_t i_begin, int64_t i_end, int n_threads,
                           double *sums)
{
    return eval_sums_core(gl, gg, n_grid, t_half, n_sigma, alpha, t_meas, n, log2_n, lattice_a,
                          n_shifts, shifts, NULL, NULL, model_tau, cdf, n_bins, mode, i_begin,
                          i_end, n_threads, sums);
}

int oracle_eval_sums_sobol(const double *gl, const double *gg, int n_grid,
                           double t_half, double n_sigma, double alpha, double t_meas,
                           int n, const uint32_t *sobol_v, int n_shifts,
                           const uint32_t *sobol_shifts, double model_tau,
                           const double *cdf, int n_bins, int mode,
                           int64_t i_begin, int64_t i_end, int n_threads, double *sums)
{
    if (!sobol_v || !sobol_shifts) return -1;
    return eval_sums_core(gl, gg, n_grid, t_half, n_sigma, alpha, t_meas, n, 32, 0, n_shifts,
                          NULL, sobol_v, sobol_shifts, model_tau, cdf, n_bins, mode, i_begin,
                          i_end, n_threads, sums);
}

/* Term mass of the charge estimate (exponential warp): per shift, the sum
 * over lattice indices [i_begin, i_end) of 2 W(u) M(u), with M the sum over
 * index vectors of |det_up det_dn|: the scale that rounding in the Keldysh
 * sum is relative to. */
int oracle_eval_mass(const double *gl, const double *gg, int n_grid,
                     double t_half, double n_sigma, double alpha, double t_meas,
                     int n, int log2_n, uint64_t lattice_a,
                     int n_shifts, const double *shifts, double model_tau,
                     int64_t i_begin, int64_t i_end, int n_threads, double *mass)
{
    if (n < 1 || n > 24 || log2_n < 1 || log2_n > 40 || i_end < i_begin ||
        i_begin < 0 || n_shifts < 1)
        return -1;
    int nt = n_threads > 0 ? n_threads : oracle_max_threads();
    for (int s = 0; s < n_shifts; ++s) {
        const double *sh = shifts + (size_t)s * n;
        double acc = 0.0;
        #pragma omp parallel for schedule(dynamic, 4) num_threads(nt) reduction(+:acc)
        for (int64_t q = i_begin; q < i_end; ++q) {
            double x[32], u[32], W, S[2], M;
            oracle_lattice_point((uint64_t)q, n, log2_n, lattice_a, sh, x);
            if (oracle_warp(n, x, model_tau, t_meas, u, &W)) {
                oracle_keldysh_sum(gl, gg, n_grid, t_half, n_sigma, alpha, t_meas, n, u, S, &M);
                acc += 2.0 * W * M;
            }
        }
        mass[s] = acc;
    }
    return 0;
}

/* The current into lead i (measurement column from the lead's tables cl,
 * cg), exponential warp: per shift, the sums over lattice indices
 * [i_begin, i_end) of f W with f = -4 i^n S(u) (Re f is the order-n
 * integrand of the particle current from the dot into the lead, both spins:
 * the lead's particle number changes at the rate -2 Re(gamma G^<_{0i}(t,t))
 * per spin), and, if mass is not NULL, of 4 W M(u). */
int oracle_eval_sums_lead(const double *gl, const double *gg, const double *cl,
                          const double *cg, int n_grid, double t_half, double n_sigma,
                          double alpha, double t_meas, int n, int log2_n, uint64_t lattice_a,
                          int n_shifts, const double *shifts, double model_tau,
                          int64_t i_begin, int64_t i_end, int n_threads, double *sums,
                          double *mass)
{
    if (n < 1 || n > 24 || log2_n < 1 || log2_n > 40 || i_end < i_begin ||
        i_begin < 0 || n_shifts < 1 || !cl || !cg)
        return -1;
    int64_t cnt = i_end - i_begin;
    double *vals = (double *)malloc(sizeof(double) * 3 * (size_t)(cnt > 0 ? cnt : 1));
    if (!vals) return -1;
    int nt = n_threads > 0 ? n_threads : oracle_max_threads();
    cplx ipow = 1.0;
    for (int k = 0; k < n; ++k) ipow *= I;
    for (int s = 0; s < n_shifts; ++s) {
        const double *sh = shifts + (size_t)s * n;
        #pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
        for (int64_t q = 0; q < cnt; ++q) {
            double x[32], u[32], W, S[2], M = 0.0;
            cplx f = 0.0;
            oracle_lattice_point((uint64_t)(i_begin + q), n, log2_n, lattice_a, sh, x);
            if (oracle_warp(n, x, model_tau, t_meas, u, &W)) {
                oracle_keldysh_sum_lead(gl, gg, cl, cg, n_grid, t_half, n_sigma, alpha, t_meas,
                                        n, u, S, &M);
                f = -4.0 * ipow * (S[0] + I * S[1]) * W;
                M *= 4.0 * W;
            }
            vals[3 * q] = creal(f);
            vals[3 * q + 1] = cimag(f);
            vals[3 * q + 2] = M;
        }
        double sr = 0.0, si = 0.0, cr = 0.0, ci = 0.0, ms = 0.0;
        for (int64_t q = 0; q < cnt; ++q) {
            double y = vals[3 * q] - cr, t = sr + y;
            cr = (t - sr) - y; sr = t;
            y = vals[3 * q + 1] - ci; t = si + y;
            ci = (t - si) - y; si = t;
            ms += vals[3 * q + 2];
        }
        sums[2 * s] = sr;
        sums[2 * s + 1] = si;
        if (mass) mass[s] = ms;
    }
    free(vals);
    return 0;
}

int oracle_eval_sums(const double *gl, const double *gg, int n_grid,
                     double t_half, double n_sigma, double alpha, double t_meas,
                     int n, int log2_n, uint64_t lattice_a,
                     int n_shifts, const double *shifts, double model_tau,
                     int mode, int64_t i_begin, int64_t i_end, int n_threads,
                     double *sums)
{
    return oracle_eval_sums_model(gl, gg, n_grid, t_half, n_sigma, alpha, t_meas, n, log2_n,
                                  lattice_a, n_shifts, shifts, model_tau, NULL, 0, mode,
                                  i_begin, i_end, n_threads, sums);
}

/* Point i of the learning sample: the shifted lattice, or (sobol_v set)
 * Sobol' point i with the digital shift dshift. */
static void learn_point(int64_t i, int n, int log2_m, uint64_t lattice_a, const double *shift,
                        const uint32_t *sobol_v, const uint32_t *dshift, double *x)
{
    if (sobol_v)
        oracle_sobol_point((uint64_t)i, n, sobol_v, dshift, x);
    else
        oracle_lattice_point((uint64_t)i, n, log2_m, lattice_a, shift, x);
}

static int learn_core(const double *gl, const double *gg, int n_grid,
                      double t_half, double n_sigma, double alpha, double t_meas,
                      int n, int log2_m, uint64_t lattice_a, const double *shift,
                      const uint32_t *sobol_v, const uint32_t *dshift,
                      double model_tau, int n_bins, double lambda, double floor_eps,
                      int n_threads, double *hist, double *cdf)
{
    if (n < 1 || n > 24 || log2_m < 1 || log2_m > 30 || n_bins < 1) return -1;
    const int64_t M = (int64_t)1 << log2_m;
    double *vals = (double *)malloc(sizeof(double) * (size_t)M);
    double *h = (double *)calloc((size_t)n * n_bins, sizeof(double));
    if (!vals || !h) {
        free(vals);
        free(h);
        return -1;
    }
    int nt = n_threads > 0 ? n_threads : oracle_max_threads();
    cplx ipow = 1.0;
    for (int k = 0; k < n + 1; ++k) ipow *= I;
    /* samples of f~ over the unit cube after the exponential warp */
    #pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (int64_t i = 0; i < M; ++i) {
        double x[32], u[32], W, S[2], Mass;
        learn_point(i, n, log2_m, lattice_a, shift, sobol_v, dshift, x);
        double v = 0.0;
        if (oracle_warp(n, x, model_tau, t_meas, u, &W)) {
            oracle_keldysh_sum(gl, gg, n_grid, t_half, n_sigma, alpha, t_meas, n, u, S, &Mass);
            v = fabs(creal(-2.0 * ipow * (S[0] + I * S[1]) * W));
        }
        vals[i] = v;
    }
    /* projection on each coordinate: bin sums in index order */
    for (int64_t i = 0; i < M; ++i) {
        if (vals[i] == 0.0) continue;
        double x[32];
        learn_point(i, n, log2_m, lattice_a, shift, sobol_v, dshift, x);
        for (int j = 0; j < n; ++j) {
            int b = (int)(x[j] * n_bins);
            if (b > n_bins - 1) b = n_bins - 1;
            h[(size_t)j * n_bins + b] += vals[i];
        }
    }
    if (hist) memcpy(hist, h, sizeof(double) * (size_t)n * n_bins);
    const int rc = oracle_model_from_hist(n, n_bins, h, lambda, floor_eps, cdf);
    free(vals);
    free(h);
    return rc;
}

int oracle_learn_model(const double *gl, const double *gg, int n_grid,
                       double t_half, double n_sigma, double alpha, double t_meas,
                       int n, int log2_m, uint64_t lattice_a,
                       const double *shift, double model_tau, int n_bins,
                       double lambda, double floor_eps, int n_threads,
                       double *hist, double *cdf)
{
    return learn_core(gl, gg, n_grid, t_half, n_sigma, alpha, t_meas, n, log2_m, lattice_a,
                      shift, NULL, NULL, model_tau, n_bins, lambda, floor_eps, n_threads,
                      hist, cdf);
}

int oracle_learn_model_sobol(const double *gl, const double *gg, int n_grid,
                             double t_half, double n_sigma, double alpha, double t_meas,
                             int n, int log2_m, const uint32_t *sobol_v,
                             const uint32_t *dshift, double model_tau, int n_bins,
                             double lambda, double floor_eps, int n_threads,
                             double *hist, double *cdf)
{
    if (!sobol_v || !dshift) return -1;
    return learn_core(gl, gg, n_grid, t_half, n_sigma, alpha, t_meas, n, log2_m, 0, NULL,
                      sobol_v, dshift, model_tau, n_bins, lambda, floor_eps, n_threads,
                      hist, cdf);
}
