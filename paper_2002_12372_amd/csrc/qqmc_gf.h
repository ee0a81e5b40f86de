/*
 * qqmc_gf.h -- non-interacting dot Green's functions of the wide-band
 * Anderson model (App. E, Delta(omega) = -i Gamma), shared by the host
 * table builder and the device table kernel.
 *
 * With A(w) = 2 Gamma / ((w - eps_d)^2 + Gamma^2) and the lead occupation
 * fbar(w) = [n_F(w - V/2) + n_F(w + V/2)] / 2 (standard Keldysh sign:
 * g^<(w) = i A fbar, g^>(w) = -i A (1 - fbar)):
 *
 *  g^<(tau), tau > 0: closing Int dw/2pi A n_F(w - mu) e^{-i w tau} in the
 *  lower half plane picks up the Lorentzian pole eps_d - i Gamma and the
 *  fermionic Matsubara poles mu - i nu_k, nu_k = (2k+1) pi / beta:
 *     I_mu(tau) = n_F(eps_d - mu - i Gamma) e^{-(i eps_d + Gamma) tau}
 *               + (i / beta) e^{-i mu tau} sum_k A(mu - i nu_k) e^{-nu_k tau},
 *     g^<(tau) = (i/2) [I_{V/2} + I_{-V/2}];
 *  g^>(tau) = g^<(tau) - i e^{-i eps_d tau - Gamma |tau|}  (g^> - g^< is the
 *     Fourier transform of -i A);
 *  tau < 0: g(-tau) = -conj(g(tau));  tau = 0: g^<(0) = i n_sigma with
 *     n_sigma = (1/2) sum_mu [1/2 - Im psi(1/2 + beta(Gamma + i(eps_d - mu))
 *                                         / (2 pi)) / pi].
 *
 * The Matsubara sum is truncated where e^{-nu_k tau} < e^{-46}; its terms
 * also fall as 1/nu_k^2, so the remainder is far below double precision.
 */
#ifndef QQMC_GF_H
#define QQMC_GF_H

#include "qqmc_tree.h"

namespace qqmc {

constexpr double kPiGF = 3.14159265358979323846;

/* e^{x + i y} */
QQMC_HD cplx cexp_(double x, double y)
{
    const double m = exp(x);
    return cmk(m * cos(y), m * sin(y));
}

QQMC_HD cplx cdiv_(cplx a, cplx b) { return cmul(a, crecip(b)); }

/* 1 / (e^{beta z} + 1), never overflowing */
QQMC_HD cplx fermi_c(double beta, cplx z)
{
    const double bx = beta * z.x, by = beta * z.y;
    if (bx > 0.0) {
        const cplx e = cexp_(-bx, -by);
        return cdiv_(e, cmk(1.0 + e.x, e.y));
    }
    const cplx e = cexp_(bx, by);
    return crecip(cmk(e.x + 1.0, e.y));
}

/* Index of the last Matsubara term kept at time tau > 0. */
QQMC_HD long matsubara_kmax(double beta, double tau)
{
    const double nu_stop = 46.0 / tau;
    const long k = (long)ceil((nu_stop * beta / kPiGF - 1.0) * 0.5) + 1;
    return k < 1 ? 1 : k;
}

/* A(mu - i nu_k) e^{-nu_k tau} */
QQMC_HD cplx matsubara_term(double eps_d, double gamma, double beta, double mu, double tau,
                            long k)
{
    const double nu = (2.0 * (double)k + 1.0) * kPiGF / beta;
    const cplx d = cmk(mu - eps_d, -nu);
    const cplx den = cmk(d.x * d.x - d.y * d.y + gamma * gamma, 2.0 * d.x * d.y);
    const double e = exp(-nu * tau);
    const cplx a = crecip(den);
    return cmk(2.0 * gamma * e * a.x, 2.0 * gamma * e * a.y);
}

/* g^<(tau) for tau > 0 given the two Matsubara sums s_plus (mu = V/2) and
 * s_minus (mu = -V/2). */
QQMC_HD cplx lesser_from_sums(double eps_d, double gamma, double beta, double bias_v,
                              double tau, cplx s_plus, cplx s_minus)
{
    const cplx lor = cexp_(-gamma * tau, -eps_d * tau);
    cplx sum = cmk(0.0, 0.0);
    for (int side = 0; side < 2; ++side) {
        const double mu = side == 0 ? 0.5 * bias_v : -0.5 * bias_v;
        const cplx ms = side == 0 ? s_plus : s_minus;
        const cplx f = fermi_c(beta, cmk(eps_d - mu, -gamma));
        const cplx ph = cexp_(0.0, -mu * tau);
        const cplx pm = cmul(ph, ms);
        /* (i / beta) * pm */
        sum = cadd(sum, cadd(cmul(f, lor), cmk(-pm.y / beta, pm.x / beta)));
    }
    /* (i/2) * sum */
    return cmk(-0.5 * sum.y, 0.5 * sum.x);
}

/* (g^<, g^>) at grid time tau from g^<(|tau|) (or the exact tau = 0 value). */
QQMC_HD pairv node_values(double eps_d, double gamma, double tau, cplx gl_abs, double n_sigma)
{
    pairv r;
    if (tau == 0.0) {
        r.gl = cmk(0.0, n_sigma);
    } else {
        r.gl = tau < 0.0 ? cnc(gl_abs) : gl_abs;
    }
    const cplx e = cexp_(-gamma * fabs(tau), -eps_d * tau);
    /* g^> = g^< - i e */
    r.gg = cmk(r.gl.x + e.y, r.gl.y - e.x);
    return r;
}

} // namespace qqmc
#endif
