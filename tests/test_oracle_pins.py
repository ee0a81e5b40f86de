"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every expected value is a
closed form, a value printed in the paper (tests/golden/), an independent
library routine (scipy's QAWF Fourier quadrature, mpmath's digamma), or a
brute-force evaluation (Leibniz determinant expansion, plain Monte Carlo).
"""
import itertools
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate

from qqmc_inputs import Dot, order_job

DOTS = [
    Dot(0.0, 1.0, 20.0, 0.0),
    Dot(0.7, 0.5, 20.0, 1.0),
    Dot(-2.5, 2.0, 20.0, 0.5),
    Dot(-0.5, 1.0, 20.0, 0.2),
]


def _tables(oracle_mod, d, n_grid=8192, t_half=10.0):
    return oracle_mod.Tables(d.eps_d, d.gamma, d.beta, d.bias_v, n_grid, t_half)


# --------------------------------------------------------------------------
# Green's function tables (App. E)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("d", DOTS)
def test_greater_minus_lesser_is_fourier_of_lorentzian(oracle_mod, d):
    """g^>(tau) - g^<(tau) = -i Int A e^{-i w tau} dw/2pi
    = -i exp(-i eps_d tau - Gamma |tau|), for any bias and temperature."""
    tb = _tables(oracle_mod, d)
    tau = tb.grid
    exact = -1j * np.exp(-1j * d.eps_d * tau - d.gamma * np.abs(tau))
    assert np.max(np.abs(tb.gg_c() - tb.gl_c() - exact)) < 1e-13


@pytest.mark.parametrize("d", DOTS)
def test_tables_hermitian(oracle_mod, d):
    """g(-tau) = -conj(g(tau)) on the symmetric grid."""
    tb = _tables(oracle_mod, d)
    for g in (tb.gl_c(), tb.gg_c()):
        assert np.max(np.abs(g[::-1] + np.conj(g))) < 1e-14


def test_symmetric_point_real_part(oracle_mod):
    """At eps_d = 0, V = 0: Re[g^<(tau)/i] = Int A (n_F(w)+n_F(-w))/2 cos/2pi
    = exp(-Gamma |tau|)/2 exactly."""
    d = Dot(0.0, 1.3, 20.0, 0.0)
    tb = _tables(oracle_mod, d)
    ref = 0.5 * np.exp(-d.gamma * np.abs(tb.grid))
    assert np.max(np.abs((tb.gl_c() / 1j).real - ref)) < 1e-14


@pytest.mark.parametrize("d", DOTS + [Dot(2.9, 0.6, 35.0, 0.9)])
def test_n_sigma_digamma(oracle_mod, d):
    """n_sigma = (1/2) sum_{mu=+-V/2} [1/2 - Im psi(1/2 + beta(Gamma +
    i(eps_d - mu))/2pi)/pi] (Lorentzian times Fermi, summed over Matsubara
    poles), evaluated with mpmath."""
    mpmath.mp.dps = 30
    ref = 0.0
    for mu in (0.5 * d.bias_v, -0.5 * d.bias_v):
        z = 0.5 + d.beta * (d.gamma + 1j * (d.eps_d - mu)) / (2 * math.pi)
        ref += 0.5 * (0.5 - float(mpmath.im(mpmath.digamma(z))) / math.pi)
    assert abs(oracle_mod.n_sigma(d.eps_d, d.gamma, d.beta, d.bias_v) - ref) < 1e-14


def test_q0_is_one_at_symmetric_point(oracle_mod):
    """Q_0 = -2 i g^<(0) = 2 n_sigma = 1 at eps_d = 0 (main text,
    "Benchmark")."""
    for beta in (5.0, 20.0, 100.0):
        assert abs(2.0 * oracle_mod.n_sigma(0.0, 1.0, beta, 0.0) - 1.0) < 1e-14


def _qawf_gf(d, tau):
    """g^<(tau), g^>(tau) by scipy's QAWF Fourier-integral quadrature of the
    defining integrals, split at omega = 0."""
    def A(w):
        return 2 * d.gamma / ((w - d.eps_d) ** 2 + d.gamma ** 2)

    def nf(x):
        return 0.5 * (1 - math.tanh(0.5 * d.beta * x))

    def fbar(w):
        return 0.5 * (nf(w - 0.5 * d.bias_v) + nf(w + 0.5 * d.bias_v))

    out = []
    for occ in (fbar, lambda w: 1.0 - fbar(w)):
        def fpos(w):
            return A(w) * occ(w)

        def fneg(x):
            return A(-x) * occ(-x)
        kw = dict(weight="cos", wvar=tau, limlst=200, limit=400, epsabs=1e-13)
        c = integrate.quad(fpos, 0, np.inf, **kw)[0] + integrate.quad(fneg, 0, np.inf, **kw)[0]
        kw["weight"] = "sin"
        s = integrate.quad(fpos, 0, np.inf, **kw)[0] - integrate.quad(fneg, 0, np.inf, **kw)[0]
        out.append((c - 1j * s) / (2 * math.pi))
    return 1j * out[0], -1j * out[1]


@pytest.mark.parametrize("d", DOTS)
@pytest.mark.parametrize("tau", [0.37, 1.5, 4.2, 9.9, -2.7])
def test_gf_against_fourier_quadrature(oracle_mod, d, tau):
    gl_ref, gg_ref = _qawf_gf(d, tau)
    gl, gg = oracle_mod.gf_direct(d.eps_d, d.gamma, d.beta, d.bias_v, tau)
    assert abs(gl - gl_ref) < 2e-9
    assert abs(gg - gg_ref) < 2e-9


def test_interpolation_is_linear_between_nodes(oracle_mod, tiny_tables):
    tb = tiny_tables
    g = tb.gl_c()
    tau = tb.grid
    for j in (0, 17, 4095, 4096, 8190):
        for phi in (0.0, 0.25, 0.5, 1.0):
            x = tau[j] + phi * (tau[j + 1] - tau[j])
            exp = (1 - phi) * g[j] + phi * g[j + 1]
            assert abs(tb.interp("<", x) - exp) < 1e-13
    # outside the grid the end values are held
    assert abs(tb.interp("<", 11.0) - g[-1]) == 0.0
    assert abs(tb.interp("<", -11.0) - g[0]) == 0.0


# --------------------------------------------------------------------------
# Determinants
# --------------------------------------------------------------------------
def _leibniz(m):
    n = m.shape[0]
    tot = 0j
    for perm in itertools.permutations(range(n)):
        sgn = 1
        p = list(perm)
        for i in range(n):
            while p[i] != i:
                j = p[i]
                p[i], p[j] = p[j], p[i]
                sgn = -sgn
        prod = 1 + 0j
        for i in range(n):
            prod *= m[i, perm[i]]
        tot += sgn * prod
    return tot


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
def test_det_matches_leibniz(oracle_mod, m):
    rng = np.random.default_rng(100 + m)
    for _ in range(5):
        a = rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))
        ref = _leibniz(a)
        assert abs(oracle_mod.det(a) - ref) <= 1e-13 * max(1.0, abs(ref))


def test_det_singular_and_pivoting(oracle_mod):
    a = np.array([[0, 1j], [2, 0]], dtype=complex)      # needs a row swap
    assert abs(oracle_mod.det(a) - (-2j)) < 1e-15
    b = np.array([[1, 2], [2, 4]], dtype=complex)
    assert oracle_mod.det(b) == 0


def test_wick_matrices_leibniz(oracle_mod, tiny_tables):
    """det_up and det_dn of the actual Wick matrices against Leibniz."""
    u = np.array([9.1, 6.0, 3.3, 0.4])
    for a in itertools.product((0, 1), repeat=4):
        m = oracle_mod.wick_matrix(tiny_tables, 10.0, u, a)
        assert abs(oracle_mod.det(m) - _leibniz(m)) < 1e-14
        assert abs(oracle_mod.det(m[1:, 1:]) - _leibniz(m[1:, 1:])) < 1e-14


def test_keldysh_sum_and_mass_brute_force(oracle_mod, tiny_tables):
    """S(u) = sum_a (-1)^|a| det_up det_dn and the term mass
    M(u) = sum_a |det_up det_dn| against a sum written out here over the 2^n
    index vectors, with Leibniz determinants of the Wick matrices."""
    for u in (np.array([8.2, 4.4, 1.3]), np.array([9.1, 6.0, 3.3, 0.4])):
        n = len(u)
        S_ref, M_ref = 0.0, 0.0
        for a in itertools.product((0, 1), repeat=n):
            m = oracle_mod.wick_matrix(tiny_tables, 10.0, u, a)
            term = _leibniz(m) * _leibniz(m[1:, 1:])
            S_ref += (-1) ** sum(a) * term
            M_ref += abs(term)
        S, M = oracle_mod.keldysh_sum(tiny_tables, 10.0, u)
        assert abs(S - S_ref) <= 1e-13 * M_ref
        assert abs(M - M_ref) <= 1e-13 * M_ref


def test_wick_matrix_keldysh_rule(oracle_mod, tiny_tables):
    """Spot entries of the 2x2 Keldysh rule of App. E: rows (0,t,0), U_k;
    columns (0,t,1), U_k; g^T = g^> for a later first argument."""
    tb = tiny_tables
    t = 10.0
    u = np.array([7.0, 2.0])
    m = oracle_mod.wick_matrix(tb, t, u, (0, 1))
    g0 = 1j * tb.n_sigma
    assert m[0, 0] == g0 and m[1, 1] == g0 and m[2, 2] == g0
    # (t,0) vs (u1,0): time ordered, t later -> g^>(t - u1)
    assert m[0, 1] == tb.interp(">", t - 7.0)
    # (t,0) vs (u2,1): lesser
    assert m[0, 2] == tb.interp("<", t - 2.0)
    # (u1,0) vs (t,1): lesser at u1 - t
    assert m[1, 0] == tb.interp("<", 7.0 - t)
    # (u2,1) vs (t,1): anti-time-ordered, t later -> g^>(u2 - t)
    assert m[2, 0] == tb.interp(">", 2.0 - t)
    # (u1,0) vs (u2,1): lesser at u1 - u2
    assert m[1, 2] == tb.interp("<", 5.0)
    # (u2,1) vs (u1,0): greater at u2 - u1
    assert m[2, 1] == tb.interp(">", -5.0)


# --------------------------------------------------------------------------
# Integrand invariants
# --------------------------------------------------------------------------
def test_order_one_closed_form(oracle_mod, tiny_tables):
    """n = 1: S = g^<(0) [g^<(tau) g^>(-tau) - g^>(tau) g^<(-tau)],
    tau = t - u, written out from the two 2x2 determinants by hand."""
    tb = tiny_tables
    g0 = 1j * tb.n_sigma
    for u in (0.3, 4.4, 9.7):
        tau = 10.0 - u
        ref = g0 * (tb.interp("<", tau) * tb.interp(">", -tau)
                    - tb.interp(">", tau) * tb.interp("<", -tau))
        S, M = oracle_mod.keldysh_sum(tb, 10.0, [u])
        assert abs(S - ref) < 1e-15


def _random_points(rng, n, t, count):
    out = []
    while len(out) < count:
        v = -np.log1p(-rng.random(n))
        u = t - np.cumsum(v)
        if u[-1] > 0:
            out.append(u)
    return out


@pytest.mark.parametrize("d", DOTS[:3])
@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_causality(oracle_mod, d, n):
    """A vertex after the measurement time makes S vanish (the Keldysh sum
    over that latest vertex's index cancels term by term)."""
    tb = _tables(oracle_mod, d)
    rng = np.random.default_rng(7 * n)
    t = 8.0
    for _ in range(4):
        u = rng.uniform(0.0, 9.5, size=n)
        u[rng.integers(n)] = rng.uniform(8.05, 9.9)
        S, M = oracle_mod.keldysh_sum(tb, t, u)
        assert abs(S) <= 1e-14 * M


@pytest.mark.parametrize("d", DOTS)
@pytest.mark.parametrize("n", [1, 2, 3, 4, 6])
def test_reality_and_permutation(oracle_mod, d, n):
    """f_n = -2 i^{n+1} S is real (g(A,B)* = -g(Bbar, Abar) pairs every
    Wick matrix with its conjugate), and S is symmetric in the vertices."""
    tb = _tables(oracle_mod, d)
    rng = np.random.default_rng(11 * n)
    for u in _random_points(rng, n, 10.0, 3):
        f, M2 = oracle_mod.integrand(tb, 10.0, u)
        assert abs(f.imag) <= 1e-14 * M2
        perm = rng.permutation(n)
        f2, _ = oracle_mod.integrand(tb, 10.0, u[perm])
        assert abs(f2 - f) <= 1e-14 * M2


# --------------------------------------------------------------------------
# Points, warping and estimator
# --------------------------------------------------------------------------
def test_lattice_points_brute_force(oracle_mod):
    log2_n, n = 10, 4
    N = 1 << log2_n
    a = 0x1F5
    shift = np.array([0.0, 0.25, 0.5, 0.875])
    z = [pow(a, j, N) for j in range(n)]
    pts = set()
    for i in range(N):
        x = oracle_mod.lattice_point(i, n, log2_n, a, shift)
        exp = [((i * z[j]) % N) / N + shift[j] for j in range(n)]
        exp = [e - 1 if e >= 1 else e for e in exp]
        assert list(x) == exp
        pts.add(tuple(x))
    assert len(pts) == N  # z_0 = 1: the points are distinct


def test_warp_closed_form(oracle_mod):
    x = np.array([0.1, 0.5, 0.3])
    u, W, inside = oracle_mod.warp(x, 0.95, 10.0)
    v = -0.95 * np.log1p(-x)
    assert np.allclose(u, 10.0 - np.cumsum(v), rtol=0, atol=1e-14)
    assert abs(W - 0.95 ** 3 * np.exp(np.sum(v) / 0.95)) < 1e-12
    assert inside
    _, _, inside = oracle_mod.warp(np.array([0.999999, 0.99]), 1.0, 10.0)
    assert not inside


@pytest.mark.parametrize("tau", [1.0, 0.95, 1.5])
@pytest.mark.parametrize("n", [1, 3, 6])
def test_model_function_mode_is_exact(oracle_mod, tiny_tables, tau, n):
    """f := p_n makes every warped sample equal C = tau^n (App. D)."""
    job = order_job(5, n, 10, 4, model_tau=tau, mode=1)
    q, mean, _ = oracle_mod.eval_order(tiny_tables, 10.0, n, job.log2_n,
                                       job.lattice_a, job.shifts, tau, mode=1)
    assert np.max(np.abs(q - tau ** n)) <= 1e-13 * tau ** n


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_constant_integrand_gives_simplex_volume(oracle_mod, tiny_tables, n):
    """f := 1 on 0 < u_n < ... < u_1 < t integrates to t^n/n!."""
    job = order_job(6, n, 14, 16, mode=2)
    q, mean, se = oracle_mod.eval_order(tiny_tables, 10.0, n, job.log2_n,
                                        job.lattice_a, job.shifts, 1.0, mode=2)
    exact = 10.0 ** n / math.factorial(n)
    assert abs(mean.real - exact) < 5 * se + 1e-9 * exact


# --------------------------------------------------------------------------
# Physics pins of the whole charge coefficient
# --------------------------------------------------------------------------
def test_q1_closed_form(oracle_mod, tiny_tables):
    """Q_1 = 2 n_sigma dn/deps_d (Hartree shift of the level); for the
    Lorentzian at eps_d = 0, V = 0 and t -> infinity this is
    -(beta/2 pi^2) psi'(1/2 + beta Gamma/2 pi).  At t = 10 the transient
    and the grid interpolation leave a few 1e-6."""
    beta, gam = 20.0, 1.0
    mpmath.mp.dps = 30
    closed = -beta / (2 * math.pi ** 2) * float(mpmath.psi(1, 0.5 + beta * gam / (2 * math.pi)))

    def f1(u):
        f, _ = oracle_mod.integrand(tiny_tables, 10.0, [u])
        return f.real
    quad = integrate.quad(f1, 0, 10.0, limit=200, epsabs=1e-12, epsrel=1e-12)[0]
    assert abs(quad - closed) < 2e-5
    # the QMC estimate (n = 1, N = 2^14, 16 shifts) agrees with the quadrature
    job = order_job(1, 1, 14, 16)
    q, mean, se = oracle_mod.eval_order(tiny_tables, 10.0, 1, job.log2_n,
                                        job.lattice_a, job.shifts, 1.0)
    assert abs(mean.real - quad) < 5 * se + 1e-9
    assert abs(mean.imag) < 1e-12


@pytest.fixture(scope="module")
def q2_quadrature(oracle_mod, tiny_tables):
    """Q_2 by nested adaptive quadrature over the ordered simplex."""
    def inner(u1):
        return integrate.quad(lambda u2: oracle_mod.integrand(tiny_tables, 10.0, [u1, u2])[0].real,
                              0, u1, epsabs=1e-11, epsrel=1e-10, limit=200)[0]
    return integrate.quad(inner, 0, 10.0, epsabs=1e-10, epsrel=1e-9, limit=200)[0]


def test_q2_two_dimensional_quadrature(oracle_mod, tiny_tables, q2_quadrature):
    """Q_2 by nested adaptive quadrature over the ordered simplex agrees with
    the warped lattice estimate within its randomised-QMC error bar."""
    quad = q2_quadrature
    job = order_job(1, 2, 14, 16)
    q, mean, se = oracle_mod.eval_order(tiny_tables, 10.0, 2, job.log2_n,
                                        job.lattice_a, job.shifts, 1.0)
    assert abs(mean.real - quad) < 5 * se + 1e-8


@pytest.mark.parametrize("n", [2, 3])
def test_plain_monte_carlo(oracle_mod, tiny_tables, n):
    """Plain Monte Carlo with numpy's MT19937, uniform on the simplex
    (sorted uniforms), against the warped lattice estimate."""
    rs = np.random.RandomState(1234 + n)
    M = 6000
    vals = np.empty(M)
    for k in range(M):
        u = np.sort(rs.uniform(0, 10.0, size=n))[::-1]
        vals[k] = oracle_mod.integrand(tiny_tables, 10.0, u)[0].real
    vol = 10.0 ** n / math.factorial(n)
    mc, mc_se = vol * vals.mean(), vol * vals.std(ddof=1) / math.sqrt(M)
    job = order_job(1, n, 14, 16)
    q, mean, se = oracle_mod.eval_order(tiny_tables, 10.0, n, job.log2_n,
                                        job.lattice_a, job.shifts, 1.0)
    assert abs(mean.real - mc) < 4 * math.hypot(mc_se, se)


def test_bethe_orders_close_at_low_temperature(oracle_mod, tiny_tables):
    """The printed Bethe-ansatz Q_1..Q_3 hold at T = 0, t -> infinity; at
    beta = 20, t = 10 the finite-temperature and transient shifts are a few
    percent, far below any sign or factor error."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "bethe_qn.txt")
    bethe = {int(l.split()[0]): float(l.split()[1]) for l in open(path)
             if l.strip() and not l.startswith("#")}
    for n, tol in ((1, 0.02), (2, 0.03), (3, 0.08)):
        job = order_job(1, n, 14, 16)
        q, mean, se = oracle_mod.eval_order(tiny_tables, 10.0, n, job.log2_n,
                                            job.lattice_a, job.shifts, 1.0)
        assert abs(mean.real / bethe[n] - 1.0) < tol, (n, mean, bethe[n])


# --------------------------------------------------------------------------
# Learned second warp (App. I, "Learning h^(i) from the integrand")
# --------------------------------------------------------------------------
def _learn(oracle_mod, tables, n, log2_m=10, n_bins=50, lam=0.05, floor_eps=1e-3, seed=21):
    job = order_job(seed, n, log2_m, 1)
    return oracle_mod.learn_model(tables, 10.0, n, log2_m, job.lattice_a, job.shifts[0],
                                  1.0, n_bins, lam, floor_eps)


def test_model_projection_brute_force(oracle_mod, tiny_tables):
    """The per-coordinate projection of |Re f~| over 64 lattice points, redone
    here point by point from the integrand, the warp and the lattice."""
    n, log2_m, n_bins = 3, 6, 8
    job = order_job(21, n, log2_m, 1)
    hist, _ = oracle_mod.learn_model(tiny_tables, 10.0, n, log2_m, job.lattice_a,
                                     job.shifts[0], 1.0, n_bins, 0.05, 1e-3)
    ref = np.zeros((n, n_bins))
    for i in range(1 << log2_m):
        x = oracle_mod.lattice_point(i, n, log2_m, job.lattice_a, job.shifts[0])
        u, W, inside = oracle_mod.warp(x, 1.0, 10.0)
        if not inside:
            continue
        f, _ = oracle_mod.integrand(tiny_tables, 10.0, u)
        for j in range(n):
            ref[j, min(int(x[j] * n_bins), n_bins - 1)] += abs((f * W).real)
    assert np.allclose(hist, ref, rtol=1e-12, atol=0)


def test_model_cdf_is_a_distribution(oracle_mod, tiny_tables):
    _, cdf = _learn(oracle_mod, tiny_tables, 4)
    nb = cdf.shape[1] - 1
    assert np.all(cdf[:, 0] == 0.0) and np.all(cdf[:, -1] == 1.0)
    q = nb * np.diff(cdf, axis=1)
    assert np.all(q >= 1e-3 * (1 - 1e-12))           # the uniform floor
    assert np.allclose(q.sum(axis=1) / nb, 1.0, rtol=1e-13)


def test_model_smoothing_limits(oracle_mod):
    """lambda -> 0 keeps the binned projection (only the floor is mixed in);
    lambda -> infinity flattens it to the uniform density."""
    rng = np.random.default_rng(3)
    hist = rng.random((2, 12)) + 0.1
    eps = 0.01
    cdf = oracle_mod.model_from_hist(hist, 1e-6, eps)
    p = hist / hist.mean(axis=1, keepdims=True)
    q = (1 - eps) * p + eps
    ref = np.concatenate([np.zeros((2, 1)), np.cumsum(q, axis=1) / 12], axis=1)
    ref /= ref[:, -1:]
    assert np.allclose(cdf, ref, rtol=1e-13, atol=1e-15)
    flat = oracle_mod.model_from_hist(hist, 1e6, eps)
    assert np.allclose(flat, np.linspace(0, 1, 13)[None, :], rtol=0, atol=1e-12)


def test_model_inverse_round_trip(oracle_mod, tiny_tables):
    """F(F^{-1}(x)) = x with F the piecewise-linear CDF (numpy interpolation),
    and q(w) the slope of F on w's bin."""
    _, cdf = _learn(oracle_mod, tiny_tables, 3)
    nb = cdf.shape[1] - 1
    edges = np.linspace(0.0, 1.0, nb + 1)
    rng = np.random.default_rng(5)
    for j in range(3):
        for x in np.concatenate([rng.random(50), cdf[j, :-1]]):
            w, q = oracle_mod.model_inverse(cdf[j], x)
            assert 0.0 <= w < 1.0
            assert abs(np.interp(w, edges, cdf[j]) - x) < 1e-14
            b = min(int(np.searchsorted(cdf[j], x, side="right")) - 1, nb - 1)
            assert abs(w * nb - b) <= 1.0 + 1e-12 and abs(q - nb * (cdf[j, b + 1] - cdf[j, b])) <= 1e-12 * q


@pytest.mark.parametrize("n", [1, 3, 6])
def test_learned_model_mode_is_exact(oracle_mod, tiny_tables, n):
    """With f := p_n prod_j q_j (the combined model), every sample is C = tau^n:
    the Jacobian of the second warp is exactly 1/prod_j q_j."""
    _, cdf = _learn(oracle_mod, tiny_tables, n)
    job = order_job(5, n, 10, 4, mode=1)
    q, _, _ = oracle_mod.eval_order(tiny_tables, 10.0, n, job.log2_n, job.lattice_a,
                                    job.shifts, 1.0, mode=1, cdf=cdf)
    assert np.max(np.abs(q - 1.0)) <= 1e-12


def test_flat_model_reduces_to_the_exponential_warp(oracle_mod, tiny_tables):
    """A uniform second warp (lambda -> infinity, no floor needed) is the
    identity: the estimates equal the exponential-warp ones."""
    n = 3
    hist = np.ones((n, 20))
    cdf = oracle_mod.model_from_hist(hist, 1e6, 0.0)
    job = order_job(7, n, 10, 4)
    a, _, _ = oracle_mod.eval_order(tiny_tables, 10.0, n, job.log2_n, job.lattice_a,
                                    job.shifts, 1.0)
    b, _, _ = oracle_mod.eval_order(tiny_tables, 10.0, n, job.log2_n, job.lattice_a,
                                    job.shifts, 1.0, cdf=cdf)
    assert np.allclose(a, b, rtol=1e-11, atol=0)


@pytest.mark.parametrize("n", [2, 3])
def test_learned_warp_constant_integrand_gives_simplex_volume(oracle_mod, tiny_tables, n):
    _, cdf = _learn(oracle_mod, tiny_tables, n)
    job = order_job(6, n, 14, 16, mode=2)
    q, mean, se = oracle_mod.eval_order(tiny_tables, 10.0, n, job.log2_n, job.lattice_a,
                                        job.shifts, 1.0, mode=2, cdf=cdf)
    exact = 10.0 ** n / math.factorial(n)
    assert abs(mean.real - exact) < 5 * se + 1e-9 * exact


def test_learned_warp_q2_against_quadrature(oracle_mod, tiny_tables, q2_quadrature):
    """Q_2 through the learned warp agrees with nested adaptive quadrature."""
    quad = q2_quadrature
    _, cdf = _learn(oracle_mod, tiny_tables, 2, log2_m=12)
    job = order_job(1, 2, 14, 16)
    q, mean, se = oracle_mod.eval_order(tiny_tables, 10.0, 2, job.log2_n, job.lattice_a,
                                        job.shifts, 1.0, cdf=cdf)
    assert abs(mean.real - quad) < 5 * se + 1e-8


# --------------------------------------------------------------------------
# Zero temperature (App. E "Precision calculation"; the paper's benchmark)
# --------------------------------------------------------------------------
def _e1_lesser_T0(eps, gam, V, tau):
    """g^<(tau > 0) at T = 0 from the exponential integral (mpmath's E1):
    Int_{-inf}^{mu} A/2pi e^{-i w tau} = [F(z1) - F(z2)] / 2 pi i with
    z = eps +- i Gamma, F(z) = -e^{-i mu tau} e^{i b tau} [E1(i b tau) + 2 pi i
    if Re < 0 <= Im of i b tau], b = mu - z."""
    def G(b):
        t0 = 1j * b * tau
        e = mpmath.e1(t0)
        if mpmath.re(t0) < 0 and mpmath.im(t0) >= 0:
            e += 2j * mpmath.pi
        return mpmath.exp(1j * b * tau) * e

    def below(mu):
        F = lambda z: -mpmath.exp(-1j * mu * tau) * G(mu - z)
        return (F(eps + 1j * gam) - F(eps - 1j * gam)) / (2j * mpmath.pi)
    return complex(0.5j * (below(V / 2) + below(-V / 2)))


@pytest.mark.parametrize("d", [Dot(0.0, 1.0, math.inf, 0.0), Dot(0.7, 0.5, math.inf, 1.0),
                               Dot(-2.5, 2.0, math.inf, 0.5)])
@pytest.mark.parametrize("tau", [0.003, 0.37, 4.2, 29.0, -1.5])
def test_zero_temperature_gf_exponential_integral(oracle_mod, d, tau):
    """The deformed-contour quadrature against the E1 closed form, and
    g^> - g^< = -i e^{-i eps tau - Gamma |tau|}."""
    mpmath.mp.dps = 30
    gl, gg = oracle_mod.gf_direct(d.eps_d, d.gamma, d.beta, d.bias_v, tau)
    ref = _e1_lesser_T0(d.eps_d, d.gamma, d.bias_v, abs(tau))
    if tau < 0:
        ref = -ref.conjugate()
    assert abs(gl - ref) < 1e-13
    assert abs((gg - gl) - (-1j) * np.exp(-1j * d.eps_d * tau - d.gamma * abs(tau))) < 1e-13


def test_zero_temperature_occupation_is_the_digamma_limit(oracle_mod):
    mpmath.mp.dps = 30
    for eps, gam, V in [(0.0, 1.0, 0.0), (0.7, 0.5, 1.0), (-2.5, 2.0, 0.5)]:
        beta = 1e9
        ref = 0.0
        for mu in (V / 2, -V / 2):
            z = 0.5 + beta * (gam + 1j * (eps - mu)) / (2 * mpmath.pi)
            ref += 0.5 * (0.5 - float(mpmath.im(mpmath.digamma(z))) / math.pi)
        assert abs(oracle_mod.n_sigma(eps, gam, math.inf, V) - ref) < 1e-8


@pytest.fixture(scope="module")
def bethe_tables(oracle_mod):
    """The paper's benchmark: T = 0, eps_d = 0, V = 0, Gamma = 1, wide band;
    grid [-30, 30] with 65536 nodes for t = 30."""
    return oracle_mod.Tables(0.0, 1.0, math.inf, 0.0, 65536, 30.0)


def _bethe():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bethe_qn.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    return {int(a): float(b) for a, b in rows}


def test_bethe_q1_by_quadrature(oracle_mod, bethe_tables):
    """Q_1 at t = 30 (adaptive quadrature of the order-1 integrand) against
    the printed Bethe-ansatz -1/pi."""
    q = integrate.quad(lambda u: oracle_mod.integrand(bethe_tables, 30.0, [u])[0].real,
                       0, 30.0, limit=400, epsabs=1e-13, epsrel=1e-12)[0]
    assert abs(q - _bethe()[1]) < 2e-6


@pytest.mark.parametrize("n", [2, 3, 4])
def test_bethe_low_orders_by_qmc(oracle_mod, bethe_tables, n):
    """Q_2..Q_4 at t = 30 (N = 2^14 x 16 shifts, tau = 0.95 as in the paper)
    within their randomised-QMC error bars of the printed Bethe values."""
    job = order_job(1, n, 14, 16, model_tau=0.95)
    q, mean, se = oracle_mod.eval_order(bethe_tables, 30.0, n, job.log2_n, job.lattice_a,
                                        job.shifts, 0.95)
    assert abs(mean.real - _bethe()[n]) < 5 * se + 2e-6


# ---------------------------------------------------------------------------
# alpha-shifted interaction U (n_up - alpha)(n_dn - alpha) (App. E, "Model";
# the diagonal shift is stated after the definition of the Wick determinant).
# The tables are built at the quadratic level E; the Hamiltonian equals the
# alpha = 0 one at level E - alpha U plus a constant, so in the stationary
# state Q^alpha(E; U) = Q^0(E - alpha U; U).  Expanding in U:
#   Q^a_1 = Q^0_1 - a dQ^0_0/dE
#   Q^a_2 = Q^0_2 - a dQ^0_1/dE + a^2/2 d2Q^0_0/dE2
#   Q^a_3 = Q^0_3 - a dQ^0_2/dE + a^2/2 d2Q^0_1/dE2 - a^3/6 d3Q^0_0/dE3
# with Q^0_0 = 2 n_sigma(E).  beta = 2 and Gamma = 1 make t = 10 stationary
# (the memory of the initial state decays like e^{-2t}); the fine grid keeps
# the tables' interpolation error near 1e-7.
# ---------------------------------------------------------------------------
ALPHA_E, ALPHA_G, ALPHA_B, ALPHA_V, ALPHA_T = 0.3, 1.0, 2.0, 0.4, 10.0


@pytest.fixture(scope="module")
def alpha_tab(oracle_mod):
    cache = {}

    def tab(e):
        if e not in cache:
            cache[e] = oracle_mod.Tables(e, ALPHA_G, ALPHA_B, ALPHA_V, 32768, 10.0)
        return cache[e]
    return tab


def _d1(f, x, h):
    return (8.0 * (f(x + h) - f(x - h)) - (f(x + 2 * h) - f(x - 2 * h))) / (12.0 * h)


def _d2(f, x, h):
    return (-f(x + 2 * h) + 16.0 * f(x + h) - 30.0 * f(x) + 16.0 * f(x - h)
            - f(x - 2 * h)) / (12.0 * h * h)


def _d3(f, x, h):
    return (-(f(x + 3 * h) - f(x - 3 * h)) + 8.0 * (f(x + 2 * h) - f(x - 2 * h))
            - 13.0 * (f(x + h) - f(x - h))) / (8.0 * h ** 3)


def _q1_quad(oracle_mod, tb):
    return integrate.quad(lambda u: oracle_mod.integrand(tb, ALPHA_T, [u])[0].real, 0, ALPHA_T,
                          epsabs=1e-13, epsrel=1e-12, limit=400)[0]


def _q0(oracle_mod, e):
    return 2.0 * oracle_mod.n_sigma(e, ALPHA_G, ALPHA_B, ALPHA_V)


@pytest.mark.parametrize("alpha", [0.5, -0.35, 1.2])
def test_alpha_order1_proportional(oracle_mod, alpha_tab, alpha):
    """At order 1 the measurement term cancels from the Keldysh sum and the
    vertex determinant is the shifted diagonal alone, so the integrand scales
    by (n_sigma - alpha) / n_sigma at every point."""
    tb = alpha_tab(ALPHA_E)
    ratio = (tb.n_sigma - alpha) / tb.n_sigma
    for u in (0.3, 4.4, 9.7):
        f0 = oracle_mod.integrand(tb, ALPHA_T, [u])[0]
        fa = oracle_mod.integrand(tb, ALPHA_T, [u], alpha)[0]
        assert abs(fa - ratio * f0) <= 1e-13 * abs(f0)


def test_alpha_wick_diagonals(oracle_mod, alpha_tab):
    """Vertex diagonals carry i (n_sigma - alpha), the measurement diagonal
    keeps i n_sigma, and no off-diagonal entry moves."""
    tb = alpha_tab(ALPHA_E)
    u, a = [7.0, 3.5, 1.0], [1, 0, 1]
    m0 = oracle_mod.wick_matrix(tb, ALPHA_T, u, a)
    ma = oracle_mod.wick_matrix(tb, ALPHA_T, u, a, 0.4)
    assert ma[0, 0] == 1j * tb.n_sigma
    for k in range(1, 4):
        assert ma[k, k] == 1j * (tb.n_sigma - 0.4)
    off = ~np.eye(4, dtype=bool)
    assert np.array_equal(ma[off], m0[off])


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_alpha_pointwise_degree(oracle_mod, alpha_tab, n):
    """Each vertex (n_up - a)(n_dn - a) contributes at most one power of a
    (its a^2 part is a c-number, cancelled between the two branches), so at
    any point the order-n integrand is a polynomial of degree n in alpha:
    its (n+1)-th finite difference vanishes to rounding of the term mass,
    its n-th does not.  Vertices within 2 of the measurement time, where the
    Keldysh sum cancels least."""
    tb = alpha_tab(ALPHA_E)
    rs = np.random.RandomState(40 + n)
    u = ALPHA_T - np.sort(rs.uniform(0.0, 2.0, n))
    h = 0.25
    r = [oracle_mod.integrand(tb, ALPHA_T, u, -0.5 + k * h) for k in range(n + 2)]
    f = [v[0] for v in r]
    mass = max(v[1] for v in r)
    dn1 = sum((-1) ** k * math.comb(n + 1, k) * f[k] for k in range(n + 2))
    dn = sum((-1) ** k * math.comb(n, k) * f[k] for k in range(n + 1))
    assert abs(dn1) <= 1e-14 * mass
    assert abs(dn) > 1e-6 * mass


@pytest.mark.parametrize("alpha", [0.5, -0.35])
def test_alpha_reexpansion_order2(oracle_mod, alpha_tab, alpha):
    """Q^a_2 - Q^0_2 (paired estimate on one lattice) against
    -a dQ^0_1/dE + a^2/2 d2Q^0_0/dE2, with Q^0_1 by adaptive quadrature."""
    d = 2e-3
    dq1 = _d1(lambda e: _q1_quad(oracle_mod, alpha_tab(e)), ALPHA_E, d)
    d2q0 = _d2(lambda e: _q0(oracle_mod, e), ALPHA_E, d)
    pred = -alpha * dq1 + 0.5 * alpha ** 2 * d2q0
    tb = alpha_tab(ALPHA_E)
    job = order_job(7, 2, 16, 16)
    qa, _, _ = oracle_mod.eval_order(tb, ALPHA_T, 2, 16, job.lattice_a, job.shifts, 1.0,
                                     alpha=alpha)
    q0, _, _ = oracle_mod.eval_order(tb, ALPHA_T, 2, 16, job.lattice_a, job.shifts, 1.0)
    diff = (qa - q0).real
    m, se = diff.mean(), diff.std(ddof=1) / math.sqrt(diff.size)
    assert abs(m - pred) < 5 * se + 3e-7, (m, se, pred)


@pytest.mark.parametrize("alpha", [0.5, -0.35])
def test_alpha_reexpansion_order3(oracle_mod, alpha_tab, alpha):
    """Q^a_3 - Q^0_3 against -a dQ^0_2/dE + a^2/2 d2Q^0_1/dE2
    - a^3/6 d3Q^0_0/dE3; dQ^0_2/dE from lattice estimates at neighbouring
    levels on one lattice (common random numbers)."""
    d = 2e-3
    j2 = order_job(8, 2, 16, 16)

    def q2(e):
        return oracle_mod.eval_order(alpha_tab(e), ALPHA_T, 2, 16, j2.lattice_a, j2.shifts,
                                     1.0)[1].real
    dq2 = _d1(q2, ALPHA_E, d)
    d2q1 = _d2(lambda e: _q1_quad(oracle_mod, alpha_tab(e)), ALPHA_E, d)
    d3q0 = _d3(lambda e: _q0(oracle_mod, e), ALPHA_E, d)
    pred = -alpha * dq2 + 0.5 * alpha ** 2 * d2q1 - alpha ** 3 / 6.0 * d3q0
    tb = alpha_tab(ALPHA_E)
    job = order_job(9, 3, 16, 16)
    qa, _, _ = oracle_mod.eval_order(tb, ALPHA_T, 3, 16, job.lattice_a, job.shifts, 1.0,
                                     alpha=alpha)
    q0, _, _ = oracle_mod.eval_order(tb, ALPHA_T, 3, 16, job.lattice_a, job.shifts, 1.0)
    diff = (qa - q0).real
    m, se = diff.mean(), diff.std(ddof=1) / math.sqrt(diff.size)
    assert abs(m - pred) < 5 * se + 1e-6, (m, se, pred)


def test_eval_mass_bounds_the_sums(oracle_mod, tiny_tables):
    """The term mass of an estimate is the sum of 2 W M over the points: it
    bounds |sum of f W| (each |S| <= M) and agrees with the per-point masses
    that integrand() returns."""
    job = order_job(3, 3, 10, 2)
    sums = oracle_mod.eval_sums(tiny_tables, 10.0, 3, 10, job.lattice_a, job.shifts, 1.0)
    mass = oracle_mod.eval_mass(tiny_tables, 10.0, 3, 10, job.lattice_a, job.shifts, 1.0)
    assert np.all(np.abs(sums) <= mass) and np.all(mass > 0)
    # the same mass point by point over a short index range
    ref = 0.0
    for i in range(40):
        x = oracle_mod.lattice_point(i, 3, 10, job.lattice_a, job.shifts[0])
        u, W, inside = oracle_mod.warp(x, 1.0, 10.0)
        if inside:
            ref += W * oracle_mod.integrand(tiny_tables, 10.0, u)[1]
    got = oracle_mod.eval_mass(tiny_tables, 10.0, 3, 10, job.lattice_a, job.shifts[:1], 1.0,
                               0, 40)[0]
    assert abs(got - ref) <= 1e-12 * ref


# ---------------------------------------------------------------------------
# Finite bandwidth: semicircular leads of half-bandwidth D (App. E, "Model").
# ---------------------------------------------------------------------------
def test_band_closed_form_at_gamma_half_d(oracle_mod):
    """Gamma = D/2, eps_d = 0: g^R = 2 (omega - i s)/D^2, so A is the
    semicircle 4 s/D^2; at infinite temperature fbar = 1/2 and
    g^<(tau) = i J_1(D tau)/(D tau) = -g^>(tau) (the Fourier transform of
    the semicircle).  beta = 1e-12 leaves an O(beta) correction."""
    from scipy.special import j1
    D = 2.0
    for tau in (0.0, 0.3, 1.7, 5.2, -3.1, 9.9):
        gl, gg = oracle_mod.gf_band(0.0, 1.0, 1e-12, 0.0, D, tau)
        ref = 0.5j if tau == 0 else 1j * j1(D * tau) / (D * tau)
        assert abs(gl - ref) < 1e-12 and abs(gg + ref) < 1e-12, tau


@pytest.mark.parametrize("eps,gam,beta,V", [(0.4, 0.3, 10.0, 0.5), (-1.2, 0.1, math.inf, 0.3),
                                            (0.0, 0.9, 2.0, 1.5)])
def test_band_sum_rule_and_occupation(oracle_mod, eps, gam, beta, V):
    """Without bound states the band carries the whole spectral weight:
    g^>(0) - g^<(0) = -i; and g^<(0) = i n_sigma with n_sigma in (0, 1)."""
    gl, gg = oracle_mod.gf_band(eps, gam, beta, V, 2.0, 0.0)
    assert abs(gg - gl + 1j) < 1e-13
    ns = oracle_mod.n_sigma_band(eps, gam, beta, V, 2.0)
    assert abs(gl - 1j * ns) < 1e-15 and 0.0 < ns < 1.0


def test_band_particle_hole_symmetry(oracle_mod):
    """eps_d = 0 and a symmetric bias: A is even and 1 - fbar(-w) = fbar(w),
    so g^>(tau) = conj(g^<(tau))."""
    for tau in (0.2, 1.0, 4.4, 9.0):
        gl, gg = oracle_mod.gf_band(0.0, 0.4, 5.0, 0.8, 2.0, tau)
        assert abs(gg - np.conj(gl)) < 1e-13


def test_band_wide_band_limit(oracle_mod):
    """D -> infinity at fixed Gamma: the tables approach the wide-band ones,
    with an error of order Gamma/D (the real part of Delta and the
    Lorentzian tails beyond the band)."""
    eps, gam, beta, V = 0.3, 1.0, 5.0, 0.4
    taus = np.linspace(0.5, 9.0, 9)
    err = {}
    for D in (50.0, 200.0):
        e = 0.0
        for tau in taus:
            gl, gg = oracle_mod.gf_band(eps, gam, beta, V, D, tau)
            w = oracle_mod.gf_direct(eps, gam, beta, V, tau)
            e = max(e, abs(gl - w[0]), abs(gg - w[1]))
        err[D] = e
    assert err[200.0] < 5e-3
    assert 2.5 < err[50.0] / err[200.0] < 6.0, err


def test_band_tables_grid_and_symmetry(oracle_mod):
    """The grid holds g(tau_j) at tau_j = -t_half + j h, and
    g(-tau) = -conj(g(tau)) (i times a real spectral weight)."""
    tb = oracle_mod.Tables(0.3, 0.1, 20.0, 0.4, 257, 10.0, half_bandwidth=2.0)
    gl, gg = tb.gl_c(), tb.gg_c()
    for j in (0, 17, 128, 200, 256):
        l, g = oracle_mod.gf_band(0.3, 0.1, 20.0, 0.4, 2.0, tb.grid[j])
        assert abs(gl[j] - l) < 1e-15 and abs(gg[j] - g) < 1e-15
        assert abs(gl[256 - j] + np.conj(gl[j])) < 1e-13
    with pytest.raises(ValueError):          # a bound state: |eps_d| >= D - Gamma
        oracle_mod.Tables(1.95, 0.1, 20.0, 0.0, 64, 10.0, half_bandwidth=2.0)


# ---------------------------------------------------------------------------
# The current into a lead (finite bandwidth): the measurement column of the
# Wick matrices is the lead site, with gamma g^<_{0i}, gamma g^>_{0i} from the
# Langreth rules; the order-n current coefficient is Re of -4 i^n S.
# ---------------------------------------------------------------------------
CUR = dict(eps=0.3, gam=1.0, beta=2.0, V=0.8, D=4.0, t=10.0)


@pytest.fixture(scope="module")
def lead_tables(oracle_mod):
    c = CUR
    return {lead: oracle_mod.Tables(c["eps"], c["gam"], c["beta"], c["V"], 16001, c["t"],
                                    half_bandwidth=c["D"], lead=lead) for lead in (1, 2)}


def _landauer(eps, gam, beta, V, D, lead):
    """Non-interacting current into the lead, both spins, from the
    transmission T = Gamma_1 Gamma_2 |g^R|^2 with the band broadening
    Gamma_i(omega) = (Gamma/D) sqrt(D^2 - omega^2) = gamma_t(omega):
    I_0 = -Int gamma_t A (f_i - f_j) domega/2pi."""
    g = gam / D

    def integrand(w):
        s = math.sqrt(max(D * D - w * w, 0.0))
        A = 2 * g * s / ((w - eps - g * w) ** 2 + (g * s) ** 2)
        mi, mj = (-V / 2, V / 2) if lead == 1 else (V / 2, -V / 2)
        fermi = lambda x: 1.0 / (math.exp(min(beta * x, 700.0)) + 1.0)
        return g * s * A * (fermi(w - mi) - fermi(w - mj))
    pts = sorted(x for x in {eps, V / 2, -V / 2} if abs(x) < D)
    return -integrate.quad(integrand, -D, D, points=pts, limit=500, epsabs=1e-14,
                           epsrel=1e-13)[0] / (2 * math.pi)


@pytest.mark.parametrize("eps,gam,beta,V,D", [(0.3, 0.5, 5.0, 0.8, 2.0),
                                              (-0.4, 1.0, 2.0, 1.5, 4.0),
                                              (0.0, 0.1, 20.0, 0.3, 2.0)])
def test_current_order0_landauer(oracle_mod, eps, gam, beta, V, D):
    """Order 0 of -4 Re(gamma G^<_{0i}(t, t)) is the Landauer current."""
    for lead in (1, 2):
        cl, _ = oracle_mod.gf_lead(eps, gam, beta, V, D, lead, 0.0)
        ref = _landauer(eps, gam, beta, V, D, lead)
        assert abs(-4.0 * cl.real - ref) <= 1e-12 * abs(ref), (lead, -4.0 * cl.real, ref)


def test_current_order1_is_the_hartree_shift(oracle_mod, lead_tables):
    """At first order the interaction shifts the level by U n_sigma (Hartree;
    no exchange between equal spins), so in the stationary state
    I_1 = n_sigma dI_0/deps_d; I_1 by adaptive quadrature of the order-1
    current integrand, dI_0/deps_d by 5-point differences of the Landauer
    current."""
    c = CUR

    def i0(e):
        return _landauer(e, c["gam"], c["beta"], c["V"], c["D"], 1)
    d = 1e-3
    di0 = (8 * (i0(c["eps"] + d) - i0(c["eps"] - d)) - (i0(c["eps"] + 2 * d)
                                                       - i0(c["eps"] - 2 * d))) / (12 * d)
    ns = oracle_mod.n_sigma_band(c["eps"], c["gam"], c["beta"], c["V"], c["D"])
    tb = lead_tables[1]
    i1 = integrate.quad(lambda u: oracle_mod.current_integrand(tb, c["t"], [u])[0].real,
                        0, c["t"], limit=400, epsabs=1e-13, epsrel=1e-12)[0]
    assert abs(i1 - ns * di0) < 5e-7, (i1, ns * di0)


def test_current_vanishes_without_bias(oracle_mod):
    """V = 0: no stationary current at first order (quadrature over the
    vertex time).  At t = 10 the charging current after the switch-on has
    decayed to about 1e-7 (the same residual as in the Hartree pin)."""
    tb = oracle_mod.Tables(0.3, 1.0, 2.0, 0.0, 4001, 10.0, half_bandwidth=4.0, lead=1)
    i1 = integrate.quad(lambda u: oracle_mod.current_integrand(tb, 10.0, [u])[0].real,
                        0, 10.0, limit=400, epsabs=1e-14, epsrel=1e-12)[0]
    tb_v = oracle_mod.Tables(0.3, 1.0, 2.0, 0.8, 4001, 10.0, half_bandwidth=4.0, lead=1)
    i1_v = integrate.quad(lambda u: oracle_mod.current_integrand(tb_v, 10.0, [u])[0].real,
                          0, 10.0, limit=400, epsabs=1e-14, epsrel=1e-12)[0]
    assert abs(i1) < 5e-7 and abs(i1_v) > 1e-2


@pytest.mark.parametrize("n", [2, 3])
def test_current_conservation(oracle_mod, lead_tables, n):
    """Stationary state: what enters lead 1 leaves lead 2, order by order
    (paired estimates on one lattice)."""
    c = CUR
    job = order_job(61, n, 14, 16)
    q1, _, _, _ = oracle_mod.eval_order_current(lead_tables[1], c["t"], n, 14, job.lattice_a,
                                                job.shifts, 1.0)
    q2, _, _, _ = oracle_mod.eval_order_current(lead_tables[2], c["t"], n, 14, job.lattice_a,
                                                job.shifts, 1.0)
    s = (q1 + q2).real
    se = s.std(ddof=1) / math.sqrt(s.size)
    assert abs(s.mean()) < 5 * se + 1e-6
    assert abs(q1.mean().real) > 20 * se      # the currents themselves are resolved


def test_lead_tables_grid(oracle_mod, lead_tables):
    tb = lead_tables[1]
    c = CUR
    for j in (0, 5000, 8000, 12345, 16000):
        cl, cg = oracle_mod.gf_lead(c["eps"], c["gam"], c["beta"], c["V"], c["D"], 1,
                                    tb.grid[j])
        got_l = tb.cl[2 * j] + 1j * tb.cl[2 * j + 1]
        got_g = tb.cg[2 * j] + 1j * tb.cg[2 * j + 1]
        assert abs(got_l - cl) < 1e-15 and abs(got_g - cg) < 1e-15
    with pytest.raises(ValueError):          # the current needs a finite band
        oracle_mod.Tables(0.0, 1.0, 2.0, 0.5, 64, 10.0, lead=1)


# ---------------------------------------------------------------------------
# Sobol' points (App. B): derived primitive polynomials and direction numbers
# (qqmc_inputs.sobol), digital shifts, the oracle's point and estimator.
# ---------------------------------------------------------------------------
def _phi(k):
    r, m, p = k, k, 2
    while p * p <= m:
        if m % p == 0:
            while m % p == 0:
                m //= p
            r -= r // p
        p += 1
    if m > 1:
        r -= r // m
    return r


def test_sobol_primitive_polynomial_counts():
    """There are phi(2^s - 1)/s primitive polynomials of degree s over GF(2);
    the derived list holds them in order of degree, and each generates a
    linear recurrence of full period 2^s - 1."""
    from qqmc_inputs import sobol as S
    polys = S.primitive_polynomials(19)
    for s in range(1, 6):
        assert sum(1 for d, _ in polys if d == s) == _phi((1 << s) - 1) // s
    for s, poly in polys:
        state, seen = 1, set()
        for _ in range((1 << s) - 1):          # LFSR with feedback poly
            seen.add(state)
            fb = bin(state & (poly >> 1)).count("1") & 1
            state = ((state << 1) | fb) & ((1 << s) - 1) if s > 1 else fb
            if s == 1:
                state = 1
        assert len(seen) == (1 << s) - 1 or s == 1


def test_sobol_first_dimension_is_van_der_corput(oracle_mod):
    from qqmc_inputs import sobol as S
    V = S.direction_numbers(3)
    for i in (0, 1, 2, 3, 5, 1000, 123456):
        rev = int("{:032b}".format(i)[::-1], 2)
        assert oracle_mod.sobol_point(i, V)[0] == rev / 2.0 ** 32


def test_sobol_one_dimensional_nets(oracle_mod):
    """Every coordinate of the first 2^m points, digitally shifted, puts
    exactly one point in each interval [k 2^-m, (k+1) 2^-m)."""
    from qqmc_inputs import sobol as S
    m, n = 10, 8
    V = S.direction_numbers(n)
    ds = S.digital_shifts(3, 1, n)[0]
    X = np.array([oracle_mod.sobol_point(i, V, ds) for i in range(1 << m)])
    for j in range(n):
        counts = np.bincount((X[:, j] * (1 << m)).astype(int), minlength=1 << m)
        assert np.all(counts == 1), j


@pytest.mark.parametrize("pair", [(0, 1), (1, 2), (2, 5), (3, 7), (6, 7)])
def test_sobol_two_dimensional_t_values(oracle_mod, pair):
    """The t-value from the generating-matrix rank criterion agrees with
    direct counting: the first 2^m points put exactly 2^t points in every
    elementary box of area 2^(t-m), and some box of area 2^(t-1-m) misses."""
    from qqmc_inputs import sobol as S
    m = 8
    V = S.direction_numbers(8)
    a, b = pair
    t = S.t_value_2d(V[a], V[b], m)
    X = np.array([oracle_mod.sobol_point(i, V) for i in range(1 << m)])[:, [a, b]]

    def stratified(tt):
        d = m - tt
        for d1 in range(d + 1):
            ia = (X[:, 0] * (1 << d1)).astype(int)
            ib = (X[:, 1] * (1 << (d - d1))).astype(int)
            counts = np.bincount(ia * (1 << (d - d1)) + ib, minlength=1 << d)
            if not np.all(counts == 1 << tt):
                return False
        return True
    assert stratified(t)
    if t > 0:
        assert not stratified(t - 1)


def test_sobol_q2_against_quadrature(oracle_mod, tiny_tables, q2_quadrature):
    """Q_2 over 2^14 Sobol' points x 16 digital shifts within its error bar
    of the two-dimensional adaptive quadrature."""
    from qqmc_inputs import sobol as S
    V = S.direction_numbers(2)
    ds = S.digital_shifts(5, 16, 2)
    _, mean, se = oracle_mod.eval_order_sobol(tiny_tables, 10.0, 2, 14, V, ds, 1.0)
    assert abs(mean.real - q2_quadrature) < 5 * se + 1e-8


# ---------------------------------------------------------------------------
# Sobol' points through the learned second warp (App. I samples the cube with
# Sobol' points, App. B)
# ---------------------------------------------------------------------------
def _sobol_xor_point(i, V, ds):
    """Sobol' point i written out here: XOR of the direction numbers of the
    set index bits and the shift word, times 2^-32."""
    x = np.zeros(V.shape[0])
    for j in range(V.shape[0]):
        w = int(ds[j])
        for k in range(32):
            if (i >> k) & 1:
                w ^= int(V[j, k])
        x[j] = w / 2.0 ** 32
    return x


def _learn_sobol(oracle_mod, tables, n, log2_m=10, n_bins=50, lam=0.05, floor_eps=1e-3,
                 seed=23):
    from qqmc_inputs import sobol as S
    V = S.direction_numbers(n)
    ds = S.digital_shifts(seed, 1, n)[0]
    return oracle_mod.learn_model_sobol(tables, 10.0, n, log2_m, V, ds, 1.0, n_bins, lam,
                                        floor_eps)


def test_sobol_model_projection_brute_force(oracle_mod, tiny_tables):
    """The projection of |Re f~| over 64 Sobol' points, redone point by point
    from the integrand, the warp and the XOR construction of the points."""
    from qqmc_inputs import sobol as S
    n, log2_m, n_bins = 3, 6, 8
    V = S.direction_numbers(n)
    ds = S.digital_shifts(23, 1, n)[0]
    hist, cdf = oracle_mod.learn_model_sobol(tiny_tables, 10.0, n, log2_m, V, ds, 1.0,
                                             n_bins, 0.05, 1e-3)
    ref = np.zeros((n, n_bins))
    for i in range(1 << log2_m):
        x = _sobol_xor_point(i, V, ds)
        u, W, inside = oracle_mod.warp(x, 1.0, 10.0)
        if not inside:
            continue
        f, _ = oracle_mod.integrand(tiny_tables, 10.0, u)
        for j in range(n):
            ref[j, min(int(x[j] * n_bins), n_bins - 1)] += abs((f * W).real)
    assert np.allclose(hist, ref, rtol=1e-12, atol=0)
    assert np.allclose(cdf, oracle_mod.model_from_hist(ref, 0.05, 1e-3), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("n", [1, 3, 6])
def test_sobol_learned_model_mode_is_exact(oracle_mod, tiny_tables, n):
    """f := p_n prod_j q_j over Sobol' points through the learned warp: every
    sample is tau^n, so each shift's mean is exactly 1 at tau = 1."""
    from qqmc_inputs import sobol as S
    _, cdf = _learn_sobol(oracle_mod, tiny_tables, n)
    V = S.direction_numbers(n)
    ds = S.digital_shifts(8, 4, n)
    q, _, _ = oracle_mod.eval_order_sobol(tiny_tables, 10.0, n, 10, V, ds, 1.0, mode=1, cdf=cdf)
    assert np.max(np.abs(q - 1.0)) <= 1e-12


def test_sobol_flat_model_reduces_to_the_exponential_warp(oracle_mod, tiny_tables):
    from qqmc_inputs import sobol as S
    n = 3
    cdf = oracle_mod.model_from_hist(np.ones((n, 20)), 1e6, 0.0)
    V = S.direction_numbers(n)
    ds = S.digital_shifts(9, 4, n)
    a, _, _ = oracle_mod.eval_order_sobol(tiny_tables, 10.0, n, 10, V, ds, 1.0)
    b, _, _ = oracle_mod.eval_order_sobol(tiny_tables, 10.0, n, 10, V, ds, 1.0, cdf=cdf)
    assert np.allclose(a, b, rtol=1e-11, atol=0)


def test_sobol_learned_warp_q2_against_quadrature(oracle_mod, tiny_tables, q2_quadrature):
    """Q_2 over Sobol' points through a model learned on Sobol' points agrees
    with the two-dimensional adaptive quadrature."""
    from qqmc_inputs import sobol as S
    _, cdf = _learn_sobol(oracle_mod, tiny_tables, 2, log2_m=12)
    V = S.direction_numbers(2)
    ds = S.digital_shifts(10, 16, 2)
    _, mean, se = oracle_mod.eval_order_sobol(tiny_tables, 10.0, 2, 14, V, ds, 1.0, cdf=cdf)
    assert abs(mean.real - q2_quadrature) < 5 * se + 1e-8
