"""Learned second warp (App. I) on the GPU against the oracle.

The learning pass runs the production integrand kernel; the projection,
smoothing and CDF are the library's own host code.  With the same learning
sample the library's projection must match the oracle's (the per-point
integrand values differ only by rounding), and with the same model (the
oracle's CDF uploaded) the estimates must match the oracle's estimator.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from qqmc_inputs import STRESS_DOT, TINY_DOT, order_job

pytestmark = pytest.mark.gpu

T_MEAS = 10.0


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_12372_amd import qqmc
    qqmc.lib()
    return qqmc


def _tables(oracle_mod, d):
    return oracle_mod.Tables(d.eps_d, d.gamma, d.beta, d.bias_v, d.n_grid, d.t_half)


def _upload(q, tb):
    return q.tables_from_host(tb.gl, tb.gg, tb.n_grid, tb.t_half, tb.n_sigma)


@pytest.mark.parametrize("n,log2_m,n_bins", [(1, 10, 16), (4, 12, 50), (8, 11, 100), (10, 8, 40)])
def test_learning_matches_oracle(q, oracle_mod, n, log2_m, n_bins):
    d = STRESS_DOT if n > 8 else TINY_DOT
    tb = _tables(oracle_mod, d)
    gt = _upload(q, tb)
    job = order_job(31, n, log2_m, 1)
    hist_o, cdf_o = oracle_mod.learn_model(tb, T_MEAS, n, log2_m, job.lattice_a, job.shifts[0],
                                           1.0, n_bins, 0.05, 1e-3)
    m = q.learn_model(gt, n, log2_m, job.lattice_a, job.shifts[0], 1.0, T_MEAS, n_bins, 0.05, 1e-3)
    cdf, hist = m.export()
    assert hist.shape == hist_o.shape and cdf.shape == cdf_o.shape
    scale = hist_o.sum(axis=1, keepdims=True)
    assert np.all(np.abs(hist - hist_o) <= 1e-10 * scale)
    assert np.all(cdf[:, 0] == 0.0) and np.all(cdf[:, -1] == 1.0)
    assert np.max(np.abs(cdf - cdf_o)) <= 1e-10


@pytest.mark.parametrize("n,log2_n,K", [(2, 12, 4), (5, 11, 3), (8, 10, 2), (10, 8, 2)])
def test_estimator_with_model_matches_oracle(q, oracle_mod, n, log2_n, K):
    """The oracle's learned model uploaded as is: per-shift estimates agree."""
    d = STRESS_DOT if n > 8 else TINY_DOT
    tb = _tables(oracle_mod, d)
    gt = _upload(q, tb)
    lj = order_job(32, n, 10, 1)
    _, cdf = oracle_mod.learn_model(tb, T_MEAS, n, 10, lj.lattice_a, lj.shifts[0], 1.0, 64,
                                    0.05, 1e-3)
    m = q.model_from_host(cdf)
    job = order_job(33, n, log2_n, K)
    qs, _, _ = q.eval_order(gt, job, T_MEAS, model=m)
    qo, _, _ = oracle_mod.eval_order(tb, T_MEAS, n, log2_n, job.lattice_a, job.shifts, 1.0,
                                     cdf=cdf)
    for s in range(K):
        assert abs(qs[s] - qo[s]) <= 1e-9 * abs(qo[s]) + 1e-15, (s, qs[s], qo[s])


def test_learned_model_mode_full_size(q, tiny_tables):
    """N = 2^20, 32 shifts, n = 8 with a model learned on the GPU: with
    f := p_n prod_j q_j every sample equals tau^n."""
    gt = q.tables_from_host(tiny_tables.gl, tiny_tables.gg, tiny_tables.n_grid,
                            tiny_tables.t_half, tiny_tables.n_sigma)
    lj = order_job(34, 8, 14, 1)
    m = q.learn_model(gt, 8, 14, lj.lattice_a, lj.shifts[0], 1.0, T_MEAS, 100, 0.05, 1e-3)
    job = order_job(1, 8, 20, 32, mode=q.MODE_MODEL)
    qs, _, _ = q.eval_order(gt, job, T_MEAS, model=m)
    assert np.max(np.abs(qs - 1.0)) <= 1e-12


def test_learned_model_in_plan_is_bitwise_single_launch(q, tiny_tables):
    """Items with and without a model in one plan give the bits of single
    launches at the plan's tile length."""
    gt = q.tables_from_host(tiny_tables.gl, tiny_tables.gg, tiny_tables.n_grid,
                            tiny_tables.t_half, tiny_tables.n_sigma)
    lj = order_job(35, 6, 12, 1)
    m = q.learn_model(gt, 6, 12, lj.lattice_a, lj.shifts[0], 1.0, T_MEAS, 50, 0.05, 1e-3)
    jobs = [order_job(36, 6, 12, 4), order_job(37, 6, 12, 4)]
    plan = q.plan_create([(gt, jobs[0], m), (gt, jobs[1])], T_MEAS, tile_len=256)
    q.plan_run(plan)
    res = q.plan_results(plan)
    for job, model, got in zip(jobs, (m, None), res):
        sums = torch.zeros(8, dtype=torch.float64, device="cuda")
        q.eval_order_async(gt, job, T_MEAS, sums, None, tile_len=256, model=model)
        h = sums.cpu().numpy()
        ref = (h[0::2] + 1j * h[1::2]) / (1 << 12)
        assert np.array_equal(got, ref)


def test_model_rejects_bad_input(q, tiny_tables):
    gt = q.tables_from_host(tiny_tables.gl, tiny_tables.gg, tiny_tables.n_grid,
                            tiny_tables.t_half, tiny_tables.n_sigma)
    cdf = np.tile(np.linspace(0.0, 1.0, 11), (3, 1))
    m = q.model_from_host(cdf)
    with pytest.raises(q.QQMCError):          # model of another order
        q.eval_order(gt, order_job(1, 4, 10, 2), T_MEAS, model=m)
    bad = cdf.copy()
    bad[1, 5] = bad[1, 4]                     # a bin of zero width
    with pytest.raises(q.QQMCError):
        q.model_from_host(bad)
    lj = order_job(1, 3, 10, 1)
    with pytest.raises(q.QQMCError):          # lambda must be positive
        q.learn_model(gt, 3, 10, lj.lattice_a, lj.shifts[0], 1.0, T_MEAS, 10, 0.0, 1e-3)
