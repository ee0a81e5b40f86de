"""The current into a lead (finite bandwidth) on the GPU, through the C ABI:
the measurement column of the Wick matrices is the lead site, with the
lead's dot-lead functions.  Kernel parity uses the oracle's tables uploaded
as they are (dot and lead); one end-to-end case builds them in the library.
Per point: tree and direct methods against the oracle's current integrand;
per shift: estimates against the oracle's; at full size: sampled tiles, and
two stationary-state laws (current conservation between the leads at order
2, the Hartree shift at order 1).

Plans and the server run the current as they run the charge: per-shift sums
equal, bit for bit, those of single launches at the same tile length.

Tolerances as in the charge parity tests, alpha = n_sigma included (per value
1e-10 relative or 1e-13 of the term mass, estimates and tiles 1e-9 relative
+1e-15).  At alpha = n_sigma the paired tree runs with a zero vertex
diagonal; points whose pair steps grow (a 2x2 pivot block spanning a long
gap) are evaluated again with data-chosen elimination blocks.  The one
comparison between tables built by the library and by the oracle (which
agree to 1e-13, not bit for bit) carries a floor of 1e-12 of the term mass.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from qqmc_inputs import Dot, order_job

pytestmark = pytest.mark.gpu

T = 10.0
CUR_DOT = Dot(0.3, 1.0, 2.0, 0.8, t_meas=T, n_grid=16001, t_half=T, half_bandwidth=4.0)


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_12372_amd import qqmc
    qqmc.lib()
    return qqmc


@pytest.fixture(scope="module")
def otab(oracle_mod):
    d = CUR_DOT
    return {lead: oracle_mod.Tables(d.eps_d, d.gamma, d.beta, d.bias_v, d.n_grid, d.t_half,
                                    half_bandwidth=d.half_bandwidth, lead=lead)
            for lead in (1, 2)}


def _upload(q, tb):
    gt = q.tables_from_host(tb.gl, tb.gg, tb.n_grid, tb.t_half, tb.n_sigma)
    q.tables_lead_from_host(gt, tb.cl, tb.cg)
    return gt


def _points(rng, n, count):
    out = []
    while len(out) < count:
        u = T - np.cumsum(-np.log1p(-rng.random(n)))
        if u[-1] > 0:
            out.append(u)
    return np.array(out)


def _eval_points(q, gt, n, u, method, alpha):
    ut = torch.tensor(u, dtype=torch.float64, device="cuda")
    f = torch.zeros((u.shape[0], 2), dtype=torch.float64, device="cuda")
    q.eval_points(gt, n, T, ut, f, method=method, alpha=alpha, current=True)
    torch.cuda.synchronize()
    fh = f.cpu().numpy()
    return fh[:, 0] + 1j * fh[:, 1]


def _check(f_gpu, ref, mass_rel, label):
    f_or = np.array([r[0] for r in ref])
    mass = np.array([r[1] for r in ref])
    err = np.abs(f_gpu - f_or)
    ok = (err <= 1e-10 * np.abs(f_or)) | (err <= mass_rel * mass)
    assert ok.all(), "%s: %d/%d off" % (label, int((~ok).sum()), ok.size)


@pytest.mark.parametrize("alpha", [0.0, "ns"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 14])
def test_points_tree_current(q, oracle_mod, otab, n, alpha):
    tb = otab[1]
    a = tb.n_sigma if alpha == "ns" else alpha
    gt = _upload(q, tb)
    u = _points(np.random.default_rng(4000 + n), n, 48 if n <= 8 else (6 if n <= 10 else 2))
    f = _eval_points(q, gt, n, u, q.METHOD_TREE, a)
    _check(f, [oracle_mod.current_integrand(tb, T, row, a) for row in u],
           1e-13, "tree n=%d" % n)


@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_points_direct_current(q, oracle_mod, otab, n):
    tb = otab[2]
    gt = _upload(q, tb)
    u = _points(np.random.default_rng(4100 + n), n, 16)
    f = _eval_points(q, gt, n, u, q.METHOD_DIRECT, 0.0)
    _check(f, [oracle_mod.current_integrand(tb, T, row, 0.0) for row in u], 1e-13,
           "direct n=%d" % n)


def test_points_direct_current_term_mass(q, oracle_mod, otab):
    """The current's term mass 4 sum_a |det_up det_dn| (lead site in the
    measurement column) against the oracle's, per point."""
    tb = otab[2]
    gt = _upload(q, tb)
    u = _points(np.random.default_rng(4200), 5, 16)
    ut = torch.tensor(u, dtype=torch.float64, device="cuda")
    f = torch.zeros((u.shape[0], 2), dtype=torch.float64, device="cuda")
    m = torch.zeros(u.shape[0], dtype=torch.float64, device="cuda")
    q.eval_points(gt, 5, T, ut, f, method=q.METHOD_DIRECT, current=True, mass=m)
    torch.cuda.synchronize()
    ref = np.array([oracle_mod.current_integrand(tb, T, row)[1] for row in u])
    assert np.all(np.abs(m.cpu().numpy() - ref) <= 1e-11 * ref)


def _compare(qs, qo, floor, label):
    floor = np.broadcast_to(np.asarray(floor, dtype=float), (len(qo),))
    worst = max((abs(qs[s] - qo[s]) / abs(qo[s]) for s in range(len(qo)) if qo[s] != 0), default=0.0)
    print("%s: worst relative error %.2e" % (label, worst))
    for s in range(len(qo)):
        assert abs(qs[s] - qo[s]) <= 1e-9 * abs(qo[s]) + floor[s], (label, s, qs[s], qo[s])


@pytest.mark.parametrize("alpha", [0.0, "ns"])
@pytest.mark.parametrize("n,log2_n,K", [(1, 13, 4), (2, 12, 4), (3, 11, 3), (5, 10, 3),
                                        (8, 9, 2), (10, 8, 2), (11, 7, 1), (12, 7, 1),
                                        (14, 6, 1)])
def test_eval_order_current(q, oracle_mod, otab, n, log2_n, K, alpha):
    tb = otab[1]
    a = tb.n_sigma if alpha == "ns" else alpha
    gt = _upload(q, tb)
    job = order_job(71, n, log2_n, K, mode=q.MODE_CURRENT, alpha=a)
    qs, _, _ = q.eval_order(gt, job, T)
    qo, _, _, mass = oracle_mod.eval_order_current(tb, T, n, log2_n, job.lattice_a, job.shifts,
                                                   1.0, alpha=a)
    _compare(qs, qo, 1e-15, "n=%d alpha=%g" % (n, a))


def test_current_library_tables_end_to_end(q, oracle_mod, otab):
    """Tables and lead functions built by the library (host band rule), the
    estimate against the oracle's on its own tables."""
    d = Dot(CUR_DOT.eps_d, CUR_DOT.gamma, CUR_DOT.beta, CUR_DOT.bias_v, T, CUR_DOT.n_grid, T,
            CUR_DOT.half_bandwidth, 1)
    gt = q.make_tables(d)
    job = order_job(72, 4, 11, 4, mode=q.MODE_CURRENT)
    qs, _, _ = q.eval_order(gt, job, T)
    qo, _, _, mass = oracle_mod.eval_order_current(otab[1], T, 4, 11, job.lattice_a,
                                                   job.shifts, 1.0)
    _compare(qs, qo, 1e-12 * mass + 1e-14, "library tables")


def test_current_full_size_sampled_tiles(q, oracle_mod, otab):
    """n = 8, N = 2^20, 32 shifts at the default tile length: sampled tile
    sums against the oracle over the same index ranges."""
    tb = otab[1]
    gt = _upload(q, tb)
    job = order_job(1, 8, 20, 32, mode=q.MODE_CURRENT)
    sums = torch.zeros(64, dtype=torch.float64, device="cuda")
    nt = q.eval_order_async(gt, job, T, sums, None)
    torch.cuda.synchronize()
    tile_len = (1 << 20) * 32 // nt
    tiles = torch.zeros(2 * nt, dtype=torch.float64, device="cuda")
    q.eval_order_async(gt, job, T, sums, tiles, tile_len=tile_len)
    torch.cuda.synchronize()
    th = tiles.cpu().numpy()
    tc = th[0::2] + 1j * th[1::2]
    per = (1 << 20) // tile_len
    for k in np.random.default_rng(97).choice(nt, size=8, replace=False):
        s, i0 = divmod(int(k), per)
        ref, mass = oracle_mod.eval_current(tb, T, 8, 20, job.lattice_a, job.shifts[s:s + 1],
                                            1.0, i0 * tile_len, (i0 + 1) * tile_len)
        assert abs(tc[k] - ref[0]) <= 1e-9 * abs(ref[0]) + 1e-15


def test_current_conservation_full_size(q, otab):
    """N = 2^20 x 32, order 2: what enters lead 1 leaves lead 2 (paired
    estimates on one lattice; the stationary state holds to about 1e-7 at
    t = 10)."""
    job = order_job(73, 2, 20, 32, mode=q.MODE_CURRENT)
    q1, _, _ = q.eval_order(_upload(q, otab[1]), job, T)
    q2, _, _ = q.eval_order(_upload(q, otab[2]), job, T)
    s = (q1 + q2).real
    se = s.std(ddof=1) / math.sqrt(s.size)
    print("I_2 into lead 1: %.9f, sum of both leads %.2e +- %.1e" % (q1.real.mean(), s.mean(), se))
    assert abs(s.mean()) < 5 * se + 1e-6
    assert abs(q1.real.mean()) > 1e3 * (5 * se + 1e-6)


def test_current_order1_hartree_full_size(q, oracle_mod, otab):
    """N = 2^20 x 32, order 1: I_1 = n_sigma dI_0/deps_d (Hartree shift;
    I_0 from the oracle's lead function at tau = 0, the Landauer current)."""
    d = CUR_DOT
    job = order_job(74, 1, 20, 32, mode=q.MODE_CURRENT)
    qs, mean, se = q.eval_order(_upload(q, otab[1]), job, T)

    def i0(e):
        return -4.0 * oracle_mod.gf_lead(e, d.gamma, d.beta, d.bias_v, d.half_bandwidth, 1,
                                         0.0)[0].real
    h = 1e-3
    di0 = (8 * (i0(d.eps_d + h) - i0(d.eps_d - h)) - (i0(d.eps_d + 2 * h)
                                                     - i0(d.eps_d - 2 * h))) / (12 * h)
    pred = otab[1].n_sigma * di0
    print("I_1 = %.10f +- %.1e, Hartree %.10f" % (mean.real, se, pred))
    assert abs(mean.real - pred) < 5 * se + 5e-7


def test_current_rejections(q, otab, tiny_tables):
    gt_plain = q.tables_from_host(tiny_tables.gl, tiny_tables.gg, tiny_tables.n_grid,
                                  tiny_tables.t_half, tiny_tables.n_sigma)
    job = order_job(75, 3, 10, 2, mode=q.MODE_CURRENT)
    with pytest.raises(q.QQMCError):           # no lead functions
        q.eval_order(gt_plain, job, T)
    with pytest.raises(q.QQMCError):           # plans need the lead functions too
        q.plan_create([(gt_plain, job)], T, tile_len=256)
    gt = _upload(q, otab[1])
    cdf = np.tile(np.linspace(0.0, 1.0, 9), (3, 1))
    with pytest.raises(q.QQMCError):           # no learned warp for the current
        q.eval_order(gt, job, T, model=q.model_from_host(cdf))


# ---------------------------------------------------------------------------
# The current in plans (persistent batched launch) and in the server
# ---------------------------------------------------------------------------
def _solo(q, gt, job, tile_len):
    K = job.shifts.shape[0]
    sums = torch.zeros(2 * K, dtype=torch.float64, device="cuda")
    q.eval_order_async(gt, job, T, sums, None, tile_len=min(tile_len, 1 << job.log2_n))
    torch.cuda.synchronize()
    h = sums.cpu().numpy()
    return (h[0::2] + 1j * h[1::2]) / (1 << job.log2_n)


def _band_dots():
    return [Dot(0.3, 1.0, 2.0, 0.8, T, 4001, T, 4.0, 1),
            Dot(0.3, 1.0, 2.0, 0.8, T, 4001, T, 4.0, 2),
            Dot(-0.6, 0.7, 5.0, 0.4, T, 4001, T, 3.0, 1)]


def test_current_plan_matches_single_launches_bitwise(q, oracle_mod, otab):
    """Current and charge items of three band dots (two leads of one), both
    trees (alpha = 0 and alpha = n_sigma), orders 1..9, in one plan: every
    replay gives the single launches' bits; one item against the oracle."""
    dots = _band_dots()
    tabs = [q.make_tables(d) for d in dots]
    entries = []
    for p, (d, gt) in enumerate(zip(dots, tabs)):
        a_ns = otab[1].n_sigma if p < 2 else 0.0
        for n in (1, 3, 5, 8, 9):
            for alpha in (0.0, a_ns):
                entries.append((gt, order_job(60 + p, n, 9 + (n % 3), 3, mode=q.MODE_CURRENT,
                                              alpha=alpha)))
        entries.append((gt, order_job(70 + p, 4, 10, 3)))
    tb = otab[1]                                # the oracle's tables, uploaded as they are
    entries.append((_upload(q, tb), order_job(75, 5, 10, 3, mode=q.MODE_CURRENT)))
    plan = q.plan_create(entries, T, tile_len=256)
    for rep in range(3):
        q.plan_run(plan)
        res = q.plan_results(plan)
        for k, ((gt, job), got) in enumerate(zip(entries, res)):
            assert np.array_equal(got, _solo(q, gt, job, 256)), (k, job.order, job.mode, rep)
    job = entries[-1][1]
    qo, _, _, mass = oracle_mod.eval_order_current(tb, T, 5, job.log2_n, job.lattice_a,
                                                   job.shifts, 1.0)
    assert np.all(np.abs(res[-1] - qo) <= 1e-9 * np.abs(qo) + 1e-15)


def test_current_plan_autotuned(q):
    dots = _band_dots()
    gt = q.make_tables(dots[0])
    entries = [(gt, order_job(80 + n, n, 10, 2, mode=q.MODE_CURRENT)) for n in (2, 6, 8)]
    plan = q.plan_create(entries, T)
    info = q.plan_info(plan)
    q.plan_run(plan)
    for (g, job), got in zip(entries, q.plan_results(plan)):
        assert np.array_equal(got, _solo(q, g, job, info["tile_len"]))


def test_current_server_equals_solo_runs(q):
    """Current and charge requests on band dots with leads, served together:
    each result is the single launch's at the server's tile length."""
    import time
    dots = _band_dots()
    reqs = []
    for i in range(10):
        d = dots[i % 3]
        n = 2 + (i * 3) % 7
        mode = q.MODE_CURRENT if i % 4 != 3 else q.MODE_CHARGE
        reqs.append((d, order_job(90 + i, n, 10 + i % 2, 3, mode=mode)))
    srv = q.Server(hbm_budget_bytes=1 << 30, max_slots=4)
    tickets = [srv.submit(d, job, T) for d, job in reqs]
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
    cache = {}
    for t, (d, job) in zip(tickets, reqs):
        key = (d.eps_d, d.beta, d.lead)
        if key not in cache:
            cache[key] = q.make_tables(d)
        assert np.array_equal(out[t]["q_shift"], _solo(q, cache[key], job, 0))
    with pytest.raises(q.QQMCError):           # the current needs a dot with a lead
        srv.submit(Dot(0.3, 1.0, 2.0, 0.8, T, 4001, T, 4.0, 0),
                   order_job(99, 3, 10, 2, mode=q.MODE_CURRENT), T)
    srv.close()
