"""Finite-bandwidth semicircular leads (App. E, "Model") on the GPU: the
uploaded tables against the oracle's adaptive quadrature, and order-n
estimates on them against the oracle, including the parameters of the
paper's finite-bandwidth application (D = 2, Gamma = 0.1, E_d = 0.9 Gamma,
alpha = n_sigma, t = 10/Gamma, tau = 1.5/Gamma; the charge, not the
current).  Tolerances as in the other parity tests (tables 1e-13, estimates
1e-9 relative + 1e-15, alpha = n_sigma included).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from qqmc_inputs import Dot, order_job

pytestmark = pytest.mark.gpu

BAND_DOTS = [Dot(0.3, 0.1, 20.0, 0.4, half_bandwidth=2.0),
             Dot(-0.6, 0.5, 8.0, 1.1, half_bandwidth=2.0),
             Dot(0.0, 1.0, float("inf"), 0.6, half_bandwidth=2.0)]
# the paper's finite-bandwidth application, V = 0.05 (one bias of its sweep)
PAPER_BAND = Dot(0.09, 0.1, 200.0, 0.05, t_meas=100.0, n_grid=65536, t_half=100.0,
                 half_bandwidth=2.0)


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_12372_amd import qqmc
    qqmc.lib()
    return qqmc


_CACHE = {}


def _oracle_tables(oracle_mod, d):
    """The oracle's tables, built once per dot (the t = 100 grid takes
    seconds)."""
    key = (d.eps_d, d.gamma, d.beta, d.bias_v, d.n_grid, d.t_half, d.half_bandwidth)
    if key not in _CACHE:
        _CACHE[key] = oracle_mod.Tables(*key[:6], half_bandwidth=d.half_bandwidth)
    return _CACHE[key]


@pytest.mark.parametrize("d", BAND_DOTS + [PAPER_BAND])
def test_band_tables_on_device_match_oracle(q, oracle_mod, d):
    gt = q.make_tables(d)
    gl, gg, ns = q.tables_export(gt)
    tb = _oracle_tables(oracle_mod, d)
    assert abs(ns - tb.n_sigma) < 1e-13
    assert np.max(np.abs(gl - tb.gl)) < 1e-13
    assert np.max(np.abs(gg - tb.gg)) < 1e-13


def _compare(qs, qo, floor, label):
    floor = np.broadcast_to(np.asarray(floor, dtype=float), (len(qo),))
    worst = max((abs(qs[s] - qo[s]) / abs(qo[s]) for s in range(len(qo)) if qo[s] != 0), default=0.0)
    print("%s: worst relative error %.2e" % (label, worst))
    for s in range(len(qo)):
        assert abs(qs[s] - qo[s]) <= 1e-9 * abs(qo[s]) + floor[s], (label, s, qs[s], qo[s])


@pytest.mark.parametrize("d", BAND_DOTS)
@pytest.mark.parametrize("n,log2_n,K", [(1, 13, 4), (2, 12, 4), (4, 11, 3), (8, 10, 2)])
def test_band_estimates_match_oracle(q, oracle_mod, d, n, log2_n, K):
    gt = q.make_tables(d)
    tb = _oracle_tables(oracle_mod, d)
    job = order_job(51, n, log2_n, K)
    qs, _, _ = q.eval_order(gt, job, d.t_meas)
    qo, _, _ = oracle_mod.eval_order(tb, d.t_meas, n, log2_n, job.lattice_a, job.shifts, 1.0)
    _compare(qs, qo, [1e-15] * K, "n=%d" % n)


@pytest.mark.parametrize("n,log2_n", [(1, 12), (2, 11), (3, 10), (4, 10), (5, 9), (6, 9),
                                      (7, 8), (8, 8), (9, 7), (10, 7), (11, 6), (12, 6)])
def test_paper_band_application_charge(q, oracle_mod, n, log2_n):
    """t = 100, tau = 15, alpha = n_sigma (paired tree and its adaptive
    re-evaluation): per-shift estimates against the oracle at orders 1-12."""
    d = PAPER_BAND
    gt = q.make_tables(d)
    tb = _oracle_tables(oracle_mod, d)
    a = tb.n_sigma
    job = order_job(52, n, log2_n, 2, model_tau=15.0, alpha=a)
    qs, _, _ = q.eval_order(gt, job, d.t_meas)
    qo, _, _ = oracle_mod.eval_order(tb, d.t_meas, n, log2_n, job.lattice_a, job.shifts, 15.0,
                                     alpha=a)
    if n == 1:
        # the Hartree term vanishes at alpha = n_sigma: zero to rounding
        assert np.max(np.abs(qs)) <= 1e-15 and np.max(np.abs(qo)) <= 1e-15
        return
    _compare(qs, qo, 1e-15, "paper band n=%d" % n)


def test_band_rejects_bound_state_regime(q):
    with pytest.raises(q.QQMCError):
        q.make_tables(Dot(1.95, 0.1, 20.0, 0.0, half_bandwidth=2.0))
