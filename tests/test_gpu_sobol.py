"""Sobol' points (App. B) on the GPU against the oracle: the same direction
numbers and digital shifts (qqmc_inputs.sobol) on both sides, per-shift
estimates and sampled tiles, both elimination trees, the charge and the
current; the learned second warp (App. I) over Sobol' points, learning pass
and estimates.  Tolerances as in the lattice parity tests (1e-9 relative;
projections 1e-10 of their sum, CDFs 1e-10)."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from qqmc_inputs import Dot, STRESS_DOT, TINY_DOT, order_job, sobol_job

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_12372_amd import qqmc
    qqmc.lib()
    return qqmc


def _upload(q, tb):
    return q.tables_from_host(tb.gl, tb.gg, tb.n_grid, tb.t_half, tb.n_sigma)


def _compare(qs, qo, label, floor=None):
    for s in range(len(qo)):
        fl = 1e-15 if floor is None else floor
        assert abs(qs[s] - qo[s]) <= 1e-9 * abs(qo[s]) + fl, (label, s, qs[s], qo[s])


@pytest.mark.parametrize("n,log2_n,K", [(1, 14, 8), (2, 12, 4), (4, 11, 3), (6, 11, 2),
                                        (8, 10, 2), (10, 8, 2), (12, 7, 1), (14, 6, 1)])
def test_sobol_estimates_match_oracle(q, oracle_mod, n, log2_n, K):
    d = STRESS_DOT if n > 8 else TINY_DOT
    tb = oracle_mod.Tables(d.eps_d, d.gamma, d.beta, d.bias_v, d.n_grid, d.t_half)
    job = sobol_job(81, n, log2_n, K)
    qs, _, _ = q.eval_order(_upload(q, tb), job, 10.0)
    qo, _, _ = oracle_mod.eval_order_sobol(tb, 10.0, n, log2_n, job.sobol_v, job.sobol_shifts,
                                           1.0)
    _compare(qs, qo, "sobol n=%d" % n)


def test_sobol_paired_tree(q, oracle_mod):
    """alpha = n_sigma (zero vertex diagonal) on Sobol' points."""
    tb = oracle_mod.Tables(0.3, 1.0, 20.0, 0.4)
    a = tb.n_sigma
    job = sobol_job(82, 6, 11, 3, alpha=a)
    qs, _, _ = q.eval_order(_upload(q, tb), job, 10.0)
    qo, _, _ = oracle_mod.eval_order_sobol(tb, 10.0, 6, 11, job.sobol_v, job.sobol_shifts,
                                           1.0, alpha=a)
    _compare(qs, qo, "sobol paired")


def test_sobol_full_size_sampled_tiles(q, oracle_mod, tiny_tables):
    """n = 8, N = 2^20, 32 digital shifts at the default tile length: sampled
    tiles against the oracle over the same index ranges (the kernel steps the
    coordinate words by 64 indices across each tile)."""
    gt = _upload(q, tiny_tables)
    job = sobol_job(1, 8, 20, 32)
    sums = torch.zeros(64, dtype=torch.float64, device="cuda")
    nt = q.eval_order_async(gt, job, 10.0, sums, None)
    torch.cuda.synchronize()
    tile_len = (1 << 20) * 32 // nt
    tiles = torch.zeros(2 * nt, dtype=torch.float64, device="cuda")
    q.eval_order_async(gt, job, 10.0, sums, tiles, tile_len=tile_len)
    torch.cuda.synchronize()
    th = tiles.cpu().numpy()
    tc = th[0::2] + 1j * th[1::2]
    per = (1 << 20) // tile_len
    for k in np.random.default_rng(96).choice(nt, size=8, replace=False):
        s, i0 = divmod(int(k), per)
        ref = oracle_mod.eval_sums_sobol(tiny_tables, 10.0, 8, job.sobol_v,
                                         job.sobol_shifts[s:s + 1], 1.0, i0 * tile_len,
                                         (i0 + 1) * tile_len)[0]
        assert abs(tc[k] - ref) <= 1e-9 * abs(ref) + 1e-13


def test_sobol_and_lattice_agree_full_size(q, tiny_tables):
    """Both point sets estimate the same Q_8 (N = 2^20 x 32)."""
    gt = _upload(q, tiny_tables)
    _, ms, ses = q.eval_order(gt, sobol_job(2, 8, 20, 32), 10.0)
    _, ml, sel = q.eval_order(gt, order_job(2, 8, 20, 32), 10.0)
    print("Q_8 Sobol' %.10f +- %.1e, lattice %.10f +- %.1e" % (ms.real, ses, ml.real, sel))
    assert abs(ms.real - ml.real) < 5 * math.hypot(ses, sel)


def test_sobol_current(q, oracle_mod):
    d = Dot(0.3, 1.0, 2.0, 0.8, n_grid=4001, half_bandwidth=4.0)
    tb = oracle_mod.Tables(d.eps_d, d.gamma, d.beta, d.bias_v, d.n_grid, d.t_half,
                           half_bandwidth=d.half_bandwidth, lead=1)
    gt = _upload(q, tb)
    q.tables_lead_from_host(gt, tb.cl, tb.cg)
    job = sobol_job(83, 3, 11, 3, mode=q.MODE_CURRENT)
    qs, _, _ = q.eval_order(gt, job, 10.0)
    # the oracle's current estimator takes lattice points; the Sobol' one is
    # checked per point: sum of the current integrand over the same points
    # (the terms are summed exactly, by math.fsum per component)
    ref = np.zeros(3, dtype=complex)
    for s in range(3):
        terms = []
        for i in range(1 << 11):
            x = oracle_mod.sobol_point(i, job.sobol_v, job.sobol_shifts[s])
            u, W, inside = oracle_mod.warp(x, 1.0, 10.0)
            if inside:
                terms.append(W * oracle_mod.current_integrand(tb, 10.0, u)[0])
        ref[s] = complex(math.fsum(t.real for t in terms),
                         math.fsum(t.imag for t in terms)) / (1 << 11)
    _compare(qs, ref, "sobol current")


def _solo(q, gt, job, tile_len, model=None):
    K = job.shifts.shape[0]
    sums = torch.zeros(2 * K, dtype=torch.float64, device="cuda")
    q.eval_order_async(gt, job, 10.0, sums, None, tile_len=min(tile_len, 1 << job.log2_n),
                       model=model)
    torch.cuda.synchronize()
    h = sums.cpu().numpy()
    return (h[0::2] + 1j * h[1::2]) / (1 << job.log2_n)


def test_sobol_plan_matches_single_launches_bitwise(q, oracle_mod, tiny_tables):
    """Sobol' items in one plan with lattice items: the charge on both
    trees, through a learned warp, and the current; every graph replay
    gives the single launches' bits; one item against the oracle."""
    gt = _upload(q, tiny_tables)
    tb_a = oracle_mod.Tables(0.3, 1.0, 20.0, 0.4)
    gt_a = _upload(q, tb_a)
    V, ds = _sobol_learn_inputs(5, 94)
    _, cdf = oracle_mod.learn_model_sobol(tiny_tables, 10.0, 5, 10, V, ds, 1.0, 32, 0.05, 1e-3)
    model = q.model_from_host(cdf)
    d = Dot(0.3, 1.0, 2.0, 0.8, 10.0, 4001, 10.0, 4.0, 1)
    gt_c = q.make_tables(d)
    entries = []
    for n in (1, 3, 6, 8, 9):
        entries.append((gt, sobol_job(100 + n, n, 9 + n % 3, 3)))
        entries.append((gt, order_job(110 + n, n, 10, 2)))
    entries.append((gt_a, sobol_job(120, 6, 10, 3, alpha=tb_a.n_sigma)))
    entries.append((gt, sobol_job(121, 5, 11, 3), model))
    entries.append((gt_c, sobol_job(122, 4, 10, 3, mode=q.MODE_CURRENT)))
    plan = q.plan_create(entries, 10.0, tile_len=256)
    for rep in range(3):
        q.plan_run(plan)
        res = q.plan_results(plan)
        for k, (e, got) in enumerate(zip(entries, res)):
            ref = _solo(q, e[0], e[1], 256, e[2] if len(e) > 2 else None)
            assert np.array_equal(got, ref), (k, e[1].order, rep)
    job = entries[4][1]                          # Sobol', order 6, tiny dot
    qo, _, _ = oracle_mod.eval_order_sobol(tiny_tables, 10.0, 6, job.log2_n, job.sobol_v,
                                           job.sobol_shifts, 1.0)
    _compare(res[4], qo, "plan sobol n=6")


def test_sobol_server_equals_solo_runs(q):
    """Sobol' and lattice requests served together: each result is the
    single launch's at the server's tile length."""
    import time
    dots = [Dot(0.0, 1.0, 20.0, 0.0), Dot(-1.2, 0.7, 20.0, 0.5)]
    reqs = []
    for i in range(8):
        n = 2 + (i * 3) % 8
        mk = sobol_job if i % 3 != 2 else order_job
        reqs.append((dots[i % 2], mk(130 + i, n, 10 + i % 2, 3)))
    srv = q.Server(hbm_budget_bytes=1 << 30, max_slots=4)
    tickets = [srv.submit(d, job, 10.0) for d, job in reqs]
    out = {}
    deadline = time.time() + 120
    while len(out) < len(tickets) and time.time() < deadline:
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        time.sleep(0.005)
    assert len(out) == len(tickets)
    tabs = [q.make_tables(d) for d in dots]
    for i, (t, (d, job)) in enumerate(zip(tickets, reqs)):
        assert np.array_equal(out[t]["q_shift"], _solo(q, tabs[i % 2], job, 0))
    srv.close()


# ---------------------------------------------------------------------------
# The learned second warp over Sobol' points (App. I learns from Sobol'
# samples of the cube; App. B)
# ---------------------------------------------------------------------------
def _sobol_learn_inputs(n, seed):
    from qqmc_inputs import sobol as S
    return S.direction_numbers(n), S.digital_shifts(seed, 1, n)[0]


@pytest.mark.parametrize("n,log2_m,n_bins", [(1, 10, 16), (4, 12, 50), (8, 11, 100),
                                             (10, 8, 40)])
def test_sobol_learning_matches_oracle(q, oracle_mod, n, log2_m, n_bins):
    d = STRESS_DOT if n > 8 else TINY_DOT
    tb = oracle_mod.Tables(d.eps_d, d.gamma, d.beta, d.bias_v, d.n_grid, d.t_half)
    V, ds = _sobol_learn_inputs(n, 85)
    hist_o, cdf_o = oracle_mod.learn_model_sobol(tb, 10.0, n, log2_m, V, ds, 1.0, n_bins,
                                                 0.05, 1e-3)
    m = q.learn_model(_upload(q, tb), n, log2_m, 0, None, 1.0, 10.0, n_bins, 0.05, 1e-3,
                      sobol_v=V, sobol_shift=ds)
    cdf, hist = m.export()
    assert hist.shape == hist_o.shape and cdf.shape == cdf_o.shape
    scale = hist_o.sum(axis=1, keepdims=True)
    assert np.all(np.abs(hist - hist_o) <= 1e-10 * scale)
    assert np.all(cdf[:, 0] == 0.0) and np.all(cdf[:, -1] == 1.0)
    assert np.max(np.abs(cdf - cdf_o)) <= 1e-10


def test_sobol_learning_paired_tree(q, oracle_mod):
    """The learning pass at alpha = n_sigma (zero vertex diagonal)."""
    tb = oracle_mod.Tables(0.3, 1.0, 20.0, 0.4)
    a = tb.n_sigma
    V, ds = _sobol_learn_inputs(5, 86)
    hist_o, cdf_o = oracle_mod.learn_model_sobol(tb, 10.0, 5, 11, V, ds, 1.0, 50, 0.05, 1e-3,
                                                 alpha=a)
    m = q.learn_model(_upload(q, tb), 5, 11, 0, None, 1.0, 10.0, 50, 0.05, 1e-3, alpha=a,
                      sobol_v=V, sobol_shift=ds)
    cdf, hist = m.export()
    scale = hist_o.sum(axis=1, keepdims=True)
    assert np.all(np.abs(hist - hist_o) <= 1e-10 * scale)
    assert np.max(np.abs(cdf - cdf_o)) <= 1e-10


@pytest.mark.parametrize("n,log2_n,K", [(1, 13, 4), (2, 12, 4), (5, 11, 3), (8, 10, 2),
                                        (10, 8, 2), (12, 7, 1)])
def test_sobol_estimates_with_model_match_oracle(q, oracle_mod, n, log2_n, K):
    """The oracle's model (learned on Sobol' points) uploaded as is: per-shift
    estimates over Sobol' points through both warps agree."""
    d = STRESS_DOT if n > 8 else TINY_DOT
    tb = oracle_mod.Tables(d.eps_d, d.gamma, d.beta, d.bias_v, d.n_grid, d.t_half)
    V, ds = _sobol_learn_inputs(n, 87)
    _, cdf = oracle_mod.learn_model_sobol(tb, 10.0, n, 10, V, ds, 1.0, 64, 0.05, 1e-3)
    job = sobol_job(88, n, log2_n, K)
    qs, _, _ = q.eval_order(_upload(q, tb), job, 10.0, model=q.model_from_host(cdf))
    qo, _, _ = oracle_mod.eval_order_sobol(tb, 10.0, n, log2_n, job.sobol_v, job.sobol_shifts,
                                           1.0, cdf=cdf)
    _compare(qs, qo, "sobol model n=%d" % n)


def test_sobol_model_paired_tree(q, oracle_mod):
    tb = oracle_mod.Tables(0.3, 1.0, 20.0, 0.4)
    a = tb.n_sigma
    V, ds = _sobol_learn_inputs(6, 89)
    _, cdf = oracle_mod.learn_model_sobol(tb, 10.0, 6, 10, V, ds, 1.0, 64, 0.05, 1e-3, alpha=a)
    job = sobol_job(90, 6, 11, 3, alpha=a)
    qs, _, _ = q.eval_order(_upload(q, tb), job, 10.0, model=q.model_from_host(cdf))
    qo, _, _ = oracle_mod.eval_order_sobol(tb, 10.0, 6, 11, job.sobol_v, job.sobol_shifts,
                                           1.0, alpha=a, cdf=cdf)
    _compare(qs, qo, "sobol model paired")


def test_sobol_model_full_size_sampled_tiles(q, oracle_mod, tiny_tables):
    """n = 8, N = 2^20 x 32 digital shifts, a model learned on the GPU from
    2^14 Sobol' points: sampled tiles against the oracle with that model."""
    gt = _upload(q, tiny_tables)
    V, ds = _sobol_learn_inputs(8, 91)
    m = q.learn_model(gt, 8, 14, 0, None, 1.0, 10.0, 100, 0.05, 1e-3, sobol_v=V,
                      sobol_shift=ds)
    cdf, _ = m.export()
    job = sobol_job(3, 8, 20, 32)
    sums = torch.zeros(64, dtype=torch.float64, device="cuda")
    nt = q.eval_order_async(gt, job, 10.0, sums, None, model=m)
    torch.cuda.synchronize()
    tile_len = (1 << 20) * 32 // nt
    tiles = torch.zeros(2 * nt, dtype=torch.float64, device="cuda")
    q.eval_order_async(gt, job, 10.0, sums, tiles, tile_len=tile_len, model=m)
    torch.cuda.synchronize()
    th = tiles.cpu().numpy()
    tc = th[0::2] + 1j * th[1::2]
    per = (1 << 20) // tile_len
    for k in np.random.default_rng(98).choice(nt, size=8, replace=False):
        s, i0 = divmod(int(k), per)
        ref = oracle_mod.eval_sums_sobol(tiny_tables, 10.0, 8, job.sobol_v,
                                         job.sobol_shifts[s:s + 1], 1.0, i0 * tile_len,
                                         (i0 + 1) * tile_len, cdf=cdf)[0]
        assert abs(tc[k] - ref) <= 1e-9 * abs(ref) + 1e-13


def test_sobol_model_mode_and_estimate_full_size(q, tiny_tables):
    """N = 2^20 x 32, n = 8, a model learned on the GPU from Sobol' points:
    with f := p_n prod_j q_j every sample is tau^n; the charge estimate
    through the learned warp agrees with the exponential warp alone."""
    gt = _upload(q, tiny_tables)
    V, ds = _sobol_learn_inputs(8, 92)
    m = q.learn_model(gt, 8, 14, 0, None, 1.0, 10.0, 100, 0.05, 1e-3, sobol_v=V,
                      sobol_shift=ds)
    qs, _, _ = q.eval_order(gt, sobol_job(4, 8, 20, 32, mode=q.MODE_MODEL), 10.0, model=m)
    assert np.max(np.abs(qs - 1.0)) <= 1e-12
    job = sobol_job(5, 8, 20, 32)
    _, ml, sel = q.eval_order(gt, job, 10.0, model=m)
    _, me, see = q.eval_order(gt, job, 10.0)
    print("Q_8 Sobol' learned warp %.10f +- %.1e, exponential %.10f +- %.1e"
          % (ml.real, sel, me.real, see))
    assert abs(ml.real - me.real) < 5 * math.hypot(sel, see)


def test_sobol_learning_rejects_half_inputs(q, tiny_tables):
    """Direction numbers without the digital shift: EINVAL at the C ABI."""
    import ctypes
    gt = _upload(q, tiny_tables)
    V = np.ascontiguousarray(_sobol_learn_inputs(3, 93)[0])
    sh = np.zeros(3)
    p = q.qqmc_learn_params(3, 10, 3, sh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1.0,
                            10.0, 16, 0.05, 1e-3, 0.0,
                            V.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), None)
    h = ctypes.c_void_p()
    st = q.lib().qqmc_learn_model(gt.handle, ctypes.byref(p), None, ctypes.byref(h))
    assert st == q.EINVAL and not h.value


def test_sobol_largest_size_sampled_tiles(q, oracle_mod, tiny_tables):
    """N = 2^24 (the largest lattice size), order 3, two digital shifts:
    sampled tiles, each shift's last tile among them, against the oracle
    (the coordinate words are stepped through every index bit up to 23)."""
    gt = _upload(q, tiny_tables)
    log2_n, K = 24, 2
    job = sobol_job(6, 3, log2_n, K)
    sums = torch.zeros(2 * K, dtype=torch.float64, device="cuda")
    nt = q.eval_order_async(gt, job, 10.0, sums, None)
    torch.cuda.synchronize()
    tile_len = (1 << log2_n) * K // nt
    tiles = torch.zeros(2 * nt, dtype=torch.float64, device="cuda")
    q.eval_order_async(gt, job, 10.0, sums, tiles, tile_len=tile_len)
    torch.cuda.synchronize()
    th = tiles.cpu().numpy()
    tc = th[0::2] + 1j * th[1::2]
    per = (1 << log2_n) // tile_len
    picks = set(int(k) for k in np.random.default_rng(99).choice(nt, size=6, replace=False))
    picks |= {per - 1, 2 * per - 1}
    for k in sorted(picks):
        s, i0 = divmod(k, per)
        ref = oracle_mod.eval_sums_sobol(tiny_tables, 10.0, 3, job.sobol_v,
                                         job.sobol_shifts[s:s + 1], 1.0, i0 * tile_len,
                                         (i0 + 1) * tile_len)[0]
        assert abs(tc[k] - ref) <= 1e-9 * abs(ref) + 1e-13, (k, tc[k], ref)
    total = sums.cpu().numpy()
    assert np.allclose(total[0::2], [th[0::2][s * per:(s + 1) * per].sum() for s in range(K)],
                       rtol=1e-12, atol=1e-15)
