"""Batched persistent launch (HIP graph) and the continuous-batching server.

Each batched item and each served request must give exactly the bits of the
single-order launch with the same tile length (the tiles are identical and
every reduction runs in a fixed order), hence the same result alone and in
the mix.  The single-order launch itself is checked against the oracle in
test_gpu_parity.py; here one batched item is also checked against the
oracle directly.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from qqmc_inputs import Dot, order_job, serving_trace

pytestmark = pytest.mark.gpu

T_MEAS = 10.0


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_12372_amd import qqmc
    qqmc.lib()
    return qqmc


def _solo(q, tables, job, tile_len):
    K = job.shifts.shape[0]
    sums = torch.zeros(2 * K, dtype=torch.float64, device="cuda")
    q.eval_order_async(tables, job, T_MEAS, sums, None, tile_len=min(tile_len, 1 << job.log2_n))
    torch.cuda.synchronize()
    s = sums.cpu().numpy()
    return (s[0::2] + 1j * s[1::2]) / (1 << job.log2_n)


def _entries(q):
    dots = [Dot(0.0, 1.0, 20.0, 0.0), Dot(-1.7, 0.5, 20.0, 1.0), Dot(2.2, 1.0, 20.0, 0.5)]
    tabs = [q.make_tables(d) for d in dots]
    entries = []
    for p, tb in enumerate(tabs):
        for n in (1, 3, 5, 8, 9):
            entries.append((tb, order_job(50 + p, n, 10 + (n % 3), 4)))
    return dots, tabs, entries


def test_plan_matches_single_launches_bitwise(q, oracle_mod):
    dots, tabs, entries = _entries(q)
    plan = q.plan_create(entries, T_MEAS, tile_len=256)
    info = q.plan_info(plan)
    assert info["tile_len"] == 256
    for rep in range(3):          # graph replays, with eager work in between
        q.plan_run(plan)
        res = q.plan_results(plan)
        for (tb, job), got in zip(entries, res):
            assert np.array_equal(got, _solo(q, tb, job, 256)), (job.order, rep)
    # one item straight against the oracle
    d = dots[1]
    tb = oracle_mod.Tables(d.eps_d, d.gamma, d.beta, d.bias_v, d.n_grid, d.t_half)
    job = entries[8][1]
    qo = oracle_mod.eval_sums(tb, T_MEAS, job.order, job.log2_n, job.lattice_a, job.shifts,
                              1.0) / (1 << job.log2_n)
    assert np.max(np.abs(res[8] - qo) / np.abs(qo)) < 1e-9


def _geometry(n, alt):
    """(lanes per item, cooperative top levels) of the scalar-tree charge
    kernel's default mapping (a depth-5 register tree: 2^(n-5) lanes per
    point up to order 10, 8 lanes per top-level prefix above; at orders 5
    and 6 a depth-4 tree, 2^(n-4) lanes) or its alternative (a depth-5 tree
    at orders 5 and 6, a depth-4 tree at orders 7, 8 and 11-14, cooperative
    top levels at 9 and 10)."""
    if n < 5:
        return (1, 0)
    if n in (5, 6):
        return (1 << (n - 5), 0) if alt else (1 << (n - 4), 0)
    if not alt:
        return (1 << (n - 5), 0) if n <= 10 else (8, n - 8)
    if n in (9, 10):
        return (8, n - 8)
    return (1 << (n - 4), 0) if n <= 8 else (16, n - 8)


def test_plan_autotuned(q):
    dots, tabs, entries = _entries(q)
    plan = q.plan_create(entries, T_MEAS)
    info = q.plan_info(plan)
    # 0: every item at its own default tile length
    assert info["tile_len"] in (0, 64, 128, 256, 512, 1024, 2048) and info["grid_blocks"] >= 0
    geo = info["geometry"]
    assert sorted(geo) == [1, 3, 5, 8, 9]
    for n, g in geo.items():
        assert g in (_geometry(n, False), _geometry(n, True)), (n, g)
    print("autotuned lane mappings:", geo)
    q.plan_run(plan)
    res = q.plan_results(plan)
    for (tb, job), got in zip(entries, res):
        ref = _solo(q, tb, job, info["tile_len"])
        if geo[job.order] == _geometry(job.order, False):
            assert np.array_equal(got, ref)
        else:
            # the other lane mapping: the same estimate to rounding (the
            # per-shift sums cancel, so the relative difference grows with
            # the order; 1e-10 is ten times tighter than the parity bar)
            assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-10, job.order


@pytest.mark.parametrize("n", [5, 6, 7, 8, 9, 10, 11, 12])
def test_plan_lane_mappings_match_each_other_and_oracle(q, oracle_mod, n):
    """Both lane mappings of the scalar-tree charge kernel against each
    other (rounding) and the alternative against the oracle (parity bar)."""
    d = Dot(-0.4, 1.0, 20.0, 0.3)
    tb = q.make_tables(d)
    log2_n, K = (11, 3) if n <= 8 else (9, 2) if n <= 10 else (8, 1)
    job = order_job(700 + n, n, log2_n, K)
    plan = q.plan_create([(tb, job)], T_MEAS, tile_len=64)
    assert q.plan_info(plan)["geometry"] == {n: _geometry(n, False)}
    q.plan_run(plan)
    r0 = q.plan_results(plan)[0]
    assert np.array_equal(r0, _solo(q, tb, job, 64))
    q.plan_set_geometry(plan, n, *_geometry(n, True))
    assert q.plan_info(plan)["geometry"] == {n: _geometry(n, True)}
    with pytest.raises(q.QQMCError):
        q.plan_set_geometry(plan, n, 3, 0)
    q.plan_run(plan)
    r1 = q.plan_results(plan)[0]
    rel = np.max(np.abs(r1 - r0) / np.abs(r0))
    to = oracle_mod.Tables(d.eps_d, d.gamma, d.beta, d.bias_v, d.n_grid, d.t_half)
    qo = oracle_mod.eval_sums(to, T_MEAS, n, job.log2_n, job.lattice_a, job.shifts,
                              1.0) / (1 << job.log2_n)
    worst = np.max(np.abs(r1 - qo) / np.abs(qo))
    print("n=%d alternative vs default mapping: %.2e, vs oracle: %.2e" % (n, rel, worst))
    # rounding only: the per-shift sums cancel (to 1e-12 relative at n = 11),
    # so the mappings are held ten times tighter than the parity bar
    assert rel < 1e-10
    assert worst < 1e-9
    # and back to the default: the single-order launch's bits again
    q.plan_set_geometry(plan, n, *_geometry(n, False))
    q.plan_run(plan)
    assert np.array_equal(q.plan_results(plan)[0], r0)


def test_server_results_equal_solo_runs(q):
    trace = serving_trace(seed=11, n_requests=12, k_min=10, k_max=12, n_min=2, n_max=9)
    srv = q.Server(hbm_budget_bytes=1 << 30, max_slots=4)
    tickets = [srv.submit(r.dot, r.job, T_MEAS) for r in trace]
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
    for t, r in zip(tickets, trace):
        tb = q.make_tables(r.dot)
        ref = _solo(q, tb, r.job, 0)
        assert np.array_equal(out[t]["q_shift"], ref)
        assert out[t]["t_done"] >= out[t]["t_submit"]
    with pytest.raises(q.QQMCError):
        srv.poll(tickets[0])          # already collected
    srv.close()


def test_server_admission_and_alone_vs_mix(q):
    trace = serving_trace(seed=12, n_requests=6, k_min=10, k_max=11, n_min=3, n_max=7)
    # alone: a fresh server per request
    alone = []
    for r in trace:
        srv = q.Server(hbm_budget_bytes=1 << 28, max_slots=1)
        t = srv.submit(r.dot, r.job, T_MEAS)
        srv.drain()
        alone.append(srv.poll(t)["q_shift"])
        srv.close()
    # in the mix: all at once on one server
    srv = q.Server(hbm_budget_bytes=1 << 28, max_slots=3)
    ts = [srv.submit(r.dot, r.job, T_MEAS) for r in trace]
    srv.drain()
    for t, a in zip(ts, alone):
        assert np.array_equal(srv.poll(t)["q_shift"], a)
    # a budget smaller than one request's footprint is refused at submission
    tiny = q.Server(hbm_budget_bytes=4096, max_slots=2)
    with pytest.raises(q.QQMCError) as e:
        tiny.submit(trace[0].dot, trace[0].job, T_MEAS)
    assert e.value.status == q.EADMIT
    with pytest.raises(q.QQMCError) as e:
        tiny.poll(12345)
    assert e.value.status == q.ENOTICKET
    tiny.close()
    srv.close()


def _c4_draws():
    """16 requests from the serving ranges (eps_d in [-3, 3], Gamma in
    [0.5, 2], V in [0, 1], beta = 20), orders 2..12, the corners of slow
    decay (Gamma = 0.5, |eps_d| = 3, where n_sigma is near 0.05 or 0.95)
    first; lattices of 2^10..2^12 points."""
    rng = np.random.default_rng(404)
    fixed = [(3.0, 0.5, 0.0), (-3.0, 0.5, 1.0), (2.9, 0.5, 0.6), (3.0, 2.0, 1.0)]
    out = []
    for i in range(16):
        if i < len(fixed):
            e, g, v = fixed[i]
        else:
            e, g, v = rng.uniform(-3, 3), rng.uniform(0.5, 2.0), rng.uniform(0, 1)
        n = 2 + (i * 7) % 11
        log2_n = 12 if n <= 6 else (11 if n <= 9 else 10)
        K = 4 if n <= 9 else 2
        out.append((Dot(float(e), float(g), 20.0, float(v)), order_job(900 + i, n, log2_n, K)))
    return out


def test_server_against_oracle_over_serving_ranges(q, oracle_mod):
    """Every per-shift Q of 16 served requests drawn from the serving ranges.
    The served results equal, bit for bit, the plain evaluation on the
    library's tables; the plain evaluation on the oracle's own tables (the
    same inputs) matches the oracle to 1e-9 relative, plus one tenth of the
    FP64 unit roundoff of the per-point term mass M (1e-17 M): some draws
    cancel by up to eleven orders of magnitude (|Q| / M = 1e-11 at order 11
    with eps_d = -2.8), where the oracle's own sum of 2^n pivoted-LU terms
    carries rounding of about 3e-19 M (2e-8 of Q against a long-double
    evaluation of the same sum, the tree 20 times closer), while a wrong or
    missing term would move Q by a sizeable fraction of M.  This covers the
    elimination tree without pivoting over the whole parameter range.  The
    served results against the oracle on its own tables (the two table
    builders agree to about 1e-13, not bit for bit) are printed."""
    draws = _c4_draws()
    srv = q.Server(hbm_budget_bytes=1 << 30, max_slots=6)
    tickets = [srv.submit(d, job, T_MEAS) for d, job in draws]
    srv.drain()
    worst_tree, worst_served, floor_used, cmp = 0.0, 0.0, 0, 0
    for t, (d, job) in zip(tickets, draws):
        served = srv.poll(t)["q_shift"]
        n, l2 = job.order, job.log2_n
        tb = oracle_mod.Tables(d.eps_d, d.gamma, d.beta, d.bias_v, d.n_grid, d.t_half)
        qo, _, _ = oracle_mod.eval_order(tb, T_MEAS, n, l2, job.lattice_a, job.shifts, 1.0)
        mass = oracle_mod.eval_mass(tb, T_MEAS, n, l2, job.lattice_a, job.shifts, 1.0)
        up = q.tables_from_host(tb.gl, tb.gg, tb.n_grid, tb.t_half, tb.n_sigma)
        plain_or = _solo(q, up, job, 0)
        plain_lib = _solo(q, q.make_tables(d), job, 0)
        assert np.array_equal(served, plain_lib), (d, n)
        for s in range(len(qo)):
            m = mass[s] / (1 << l2)
            e_tree = abs(plain_or[s] - qo[s])
            worst_tree = max(worst_tree, e_tree / abs(qo[s]))
            worst_served = max(worst_served, abs(served[s] - qo[s]) / abs(qo[s]))
            cmp += 1
            floor_used += e_tree > 1e-9 * abs(qo[s]) + 1e-15
            assert e_tree <= 1e-9 * abs(qo[s]) + 1e-17 * m + 1e-15, \
                ("tree", d, n, s, plain_or[s], qo[s], m)
    print("serving ranges: tree on the oracle's tables worst relative error %.2e (%d of %d "
          "comparisons beyond 1e-9 relative, within 1e-17 of the term mass); served against "
          "the oracle on its own tables worst relative difference %.2e"
          % (worst_tree, floor_used, cmp, worst_served))
    srv.close()
