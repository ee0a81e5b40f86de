"""Throughput of the QQMC hot path on one MI355X.

Workload (one step): the order-8 charge coefficient of the wide-band dot
(Gamma = 1, eps_d = 0, beta = 20, V = 0, t = 10), N = 2^20 Korobov lattice
points x 32 random shifts (33,554,432 points), warped with h(v) = exp(-v),
Keldysh sum over all 2^8 index vectors per point, reduced per shift on the
device.  Tables are built and resident in HBM before timing.

Prints one JSON line: points/s (all lattice points, in or out of the domain),
the roofline of the integrand kernel (FP64 vector ALU: algorithmic
operations of the elimination tree per point inside the domain, see
paper_2002_12372_amd/flops.py), the CPU oracle timed on a bounded sample,
and the serving trace (512 Poisson sweep requests at 200/s): p50 and p99
latency and points/s of the continuous-batching server beside one plain
launch per request in arrival order.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Keldysh-summed integrand points/s at n=8 FP64, % FP64 peak; p99 sweep latency"
FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CUs x 128 FP64 flop/clk x 2.4 GHz


KERNEL_SOURCES = ["paper_2002_12372_amd/csrc/qqmc_kernels.hip",
                  "paper_2002_12372_amd/csrc/qqmc_kernels.h",
                  "paper_2002_12372_amd/csrc/qqmc_tree.h",
                  "paper_2002_12372_amd/csrc/qqmc_adapt.h",
                  "paper_2002_12372_amd/csrc/qqmc_gf.h",
                  "paper_2002_12372_amd/csrc/qqmc_internal.h",
                  "paper_2002_12372_amd/csrc/qqmc_api.cpp"]


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(order):
    """HBM bytes per launch from the committed rocprofv3 counter summary, only
    if it was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_order%d.json" % order)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return rec.get("bytes_per_launch")


def inside_fraction(n, t_over_tau):
    from scipy.special import gammainc
    return float(gammainc(n, t_over_tau))


def counted_inside_fraction(job, t_meas, tau):
    """Fraction of the job's lattice points inside the domain (u_n > 0),
    counted on the host with the kernel's arithmetic: m = i a^j mod N,
    y = m / N + shift (minus 1 past 1), v = -tau log1p(-y), u_j = u_{j-1} - v
    in sequence.  (The host's log1p may differ from the device's in the last
    place, which can move only points within about 1e-15 of the boundary.)"""
    import numpy as np
    n, N = job.order, 1 << job.log2_n
    z = [pow(int(job.lattice_a), j, N) for j in range(n)]
    idx = np.arange(N, dtype=np.uint64)
    inside = 0
    for s in range(job.shifts.shape[0]):
        u = np.full(N, float(t_meas))
        for j in range(n):
            m = (idx * np.uint64(z[j])) & np.uint64(N - 1)
            y = m.astype(np.float64) / N + job.shifts[s, j]
            y[y >= 1.0] -= 1.0
            u -= -tau * np.log1p(-y)
        inside += int(np.count_nonzero(u > 0.0))
    return inside / (N * job.shifts.shape[0])


def cpu_baseline(order, log2_n, lattice_a, shifts, count):
    import oracle
    from qqmc_inputs import TINY_DOT as d
    tb = oracle.Tables(d.eps_d, d.gamma, d.beta, d.bias_v, d.n_grid, d.t_half)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.eval_sums(tb, d.t_meas, order, log2_n, lattice_a, shifts[:1], 1.0, 0, 0, count,
                     n_threads=threads)
    dt = time.perf_counter() - t0
    one = max(count // 64, 64)
    t0 = time.perf_counter()
    oracle.eval_sums(tb, d.t_meas, order, log2_n, lattice_a, shifts[:1], 1.0, 0, 0, one,
                     n_threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": count / dt, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": "lattice indices 0..%d of shift 0 (order %d, same dot and lattice), "
                      "%d OpenMP threads, %.1f s" % (count - 1, order, threads, dt),
            "one_core": {"value": one / dt1, "sample": "indices 0..%d, 1 thread, %.1f s"
                                                      % (one - 1, dt1)}}


def timed_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [a.elapsed_time(b) for a, b in ev]


def run_plain(args):
    import torch
    from paper_2002_12372_amd import qqmc
    from paper_2002_12372_amd.flops import pair_tree_flops, tree_flops, warp_flops
    from qqmc_inputs import Dot, TINY_DOT, order_job, sobol_job

    stream = torch.cuda.current_stream()
    n = args.order
    alpha = 0.0
    tau = 1.0
    mode = qqmc.MODE_CHARGE
    d = TINY_DOT
    if args.current:
        # the paper's current application (semicircular leads D = 2,
        # Gamma = 0.1, E_d = 0.9 Gamma, alpha = n_sigma, t = 10/Gamma,
        # tau = 1.5/Gamma): the current into lead 1
        d = Dot(0.09, 0.1, 200.0, 0.05, t_meas=100.0, n_grid=65536, t_half=100.0,
                half_bandwidth=2.0, lead=1)
        args.alpha = "ns"
        tau = 15.0
        mode = qqmc.MODE_CURRENT
    elif args.band:
        # the paper's finite-bandwidth application: semicircular leads D = 2,
        # Gamma = 0.1, E_d = 0.9 Gamma, alpha = n_sigma, t = 10/Gamma,
        # tau = 1.5/Gamma (bias 0.05, low temperature)
        d = Dot(0.09, 0.1, 200.0, 0.05, t_meas=100.0, n_grid=65536, t_half=100.0,
                half_bandwidth=2.0)
        args.alpha = "ns"
        tau = 15.0
    elif args.alpha is not None:
        # the alpha-shifted interaction away from particle-hole symmetry;
        # "ns" is the paper's choice alpha = n_sigma (zero vertex diagonal)
        d = Dot(0.3, 1.0, 20.0, 0.4)
    tables = qqmc.make_tables(d)
    if args.alpha is not None:
        alpha = qqmc.tables_export(tables)[2] if args.alpha == "ns" else float(args.alpha)
    make_job = sobol_job if args.sobol else order_job
    job = make_job(1, n, args.log2n, args.shifts, model_tau=tau, mode=mode, alpha=alpha)
    # the library runs the paired tree when |n_sigma - alpha| < 0.05
    paired = abs(qqmc.tables_export(tables)[2] - alpha) < 0.05
    tflops = pair_tree_flops(n) if paired else tree_flops(n)
    if mode == qqmc.MODE_CURRENT:
        tflops += 16 * n        # the lead-function lookups of the measurement column
    N = 1 << args.log2n
    points = N * args.shifts
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    sums = torch.zeros(2 * args.shifts, dtype=torch.float64, device="cuda")

    def step():
        qqmc.eval_order_async(tables, job, d.t_meas, sums, None, tile_len=args.tile, stream=stream)

    wall, launch_ms = timed_steps(step, args.steps, args.warmup, stream)
    ms_per_step = wall * 1e3 / args.steps
    value = points * args.steps / wall
    frac_model = inside_fraction(n, d.t_meas / job.model_tau)
    frac_in = frac_model if args.sobol else counted_inside_fraction(job, d.t_meas, job.model_tau)
    alg_flops = points * (frac_in * tflops + warp_flops(n))
    avg_launch_s = sum(launch_ms) / len(launch_ms) * 1e-3
    achieved = alg_flops / avg_launch_s / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s of the %s Anderson dot "
                               "(Gamma=%g, eps_d=%g, beta=%g, V=%g, t=%g%s), order %d, "
                               "%s N=2^%d x %d random shifts, tau=%g"
                               % ("current coefficient I_n into lead 1"
                                  if mode == qqmc.MODE_CURRENT else "charge coefficient Q_n",
                                  "semicircular-lead (D=%g)" % d.half_bandwidth
                                  if d.half_bandwidth else "wide-band",
                                  d.gamma, d.eps_d, d.beta, d.bias_v, d.t_meas,
                                  (", alpha=%.6g, %s tree" % (alpha, "paired" if paired else "scalar"))
                                  if alpha else "",
                                  n, "Sobol' points (digital shifts)" if args.sobol
                                  else "Korobov lattice", args.log2n, args.shifts, tau),
                   "order": n, "lattice_points": N, "shifts": args.shifts,
                   "inside_fraction": frac_in,
                   "inside_fraction_source": "model P(n, t/tau)" if args.sobol
                                             else "counted over the lattice",
                   "inside_fraction_model": frac_model,
                   "inside_points_per_s": value * frac_in},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": measured_traffic(n) if alpha == 0.0 else None,
                     "flops_per_inside_point": tflops,
                     "avg_launch_ms": avg_launch_s * 1e3},
    }
    if not args.no_serving and alpha == 0.0 and not args.sobol and n == 8:
        # the metric's second half: p99 sweep latency of the serving trace,
        # served by continuous batching and by plain launches (before the
        # CPU leg, whose worker threads would share the host with the
        # server's scheduling thread)
        out["serving"] = serving_measure(args)[0]
    if not args.no_cpu and alpha == 0.0 and not args.sobol:
        out["cpu_baseline"] = cpu_baseline(n, args.log2n, job.lattice_a, job.shifts,
                                           args.cpu_sample)
    print(json.dumps(out), flush=True)


def run_geometry(args):
    """Both lane mappings of the scalar-tree charge kernel, order by order:
    one plan per order (Gamma=1, eps_d=0, beta=20, V=0, t=10; 32 shifts;
    N = 2^(16+floor(2(n-1)/3)) up to order 10, 2^(30-n) above), forced to
    each mapping in turn, timed over the same steps.  One JSON line per
    order; a mapping is (lanes per item, cooperative top levels)."""
    import torch
    from paper_2002_12372_amd import qqmc
    from paper_2002_12372_amd.flops import geometry, tree_flops
    from qqmc_inputs import Dot, batched_log2_n, order_job

    def shape(n, alt):
        _, off, t = geometry(n, alt)
        return (1 << t, off)

    stream = torch.cuda.current_stream()
    tb = qqmc.make_tables(Dot(0.0, 1.0, 20.0, 0.0))
    for n in range(5, 15):
        log2_n = batched_log2_n(n) if n <= 10 else 20 - (n - 10)
        job = order_job(900 + n, n, log2_n, 32)
        plan = qqmc.plan_create([(tb, job)], 10.0)
        info = qqmc.plan_info(plan)
        auto = info["geometry"][n]
        pts = (1 << log2_n) * 32
        flops = pts * inside_fraction(n, 10.0) * tree_flops(n)
        default, other = shape(n, False), shape(n, True)
        row = {"order": n, "lattice_points": 1 << log2_n, "shifts": 32,
               "tile_len": info["tile_len"], "autotuned": list(auto)}
        for name, g in (("default", default), ("alternative", other)):
            qqmc.plan_set_geometry(plan, n, *g)
            _, ms = timed_steps(lambda: qqmc.plan_run(plan, stream), args.steps, args.warmup, stream)
            t = sum(ms) / len(ms) * 1e-3
            row[name] = {"lanes_per_item": g[0], "top_levels": g[1], "ms_per_step": t * 1e3,
                         "points_per_s": pts / t,
                         "frac_fp64_peak": flops / t / 1e12 / FP64_VECTOR_PEAK_TFLOPS}
        print(json.dumps(row), flush=True)


def run_batched(args):
    """64 dots x orders 1..10 x 16 shifts, lattice sizes 2^(16+floor(2(n-1)/3)-shrink):
    one autotuned persistent launch (HIP graph) against one launch per item."""
    import numpy as np
    import torch
    from paper_2002_12372_amd import qqmc
    from paper_2002_12372_amd.flops import tree_flops
    from qqmc_inputs import batched_dots, batched_jobs

    stream = torch.cuda.current_stream()
    dots = batched_dots(count=args.params)
    tables = [qqmc.make_tables(d) for d in dots]
    jobs = batched_jobs(count=args.params, log2_offset=args.shrink)
    entries = [(tables[p], job) for p, job in jobs]
    t0 = time.perf_counter()
    plan = qqmc.plan_create(entries, 10.0)
    t_plan = time.perf_counter() - t0
    info = qqmc.plan_info(plan)
    points = info["n_points"]
    print("batched: %d items, %d points, %d tiles, tile_len %d, grid %d, plan %.2f s"
          % (len(entries), points, info["n_tiles"], info["tile_len"], info["grid_blocks"], t_plan),
          file=sys.stderr, flush=True)
    wall_b, ms_b = timed_steps(lambda: qqmc.plan_run(plan, stream), args.steps, args.warmup, stream)
    res_b = qqmc.plan_results(plan)
    sums = [torch.zeros(2 * job.shifts.shape[0], dtype=torch.float64, device="cuda")
            for _, job in entries]

    def per_item():
        for (tb, job), buf in zip(entries, sums):
            qqmc.eval_order_async(tb, job, 10.0, buf, None,
                                  tile_len=min(info["tile_len"], 1 << job.log2_n), stream=stream)

    wall_p, ms_p = timed_steps(per_item, args.steps, args.warmup, stream)
    solo = [(lambda h: (h[0::2] + 1j * h[1::2]) / (1 << job.log2_n))(buf.cpu().numpy())
            for buf, (_, job) in zip(sums, entries)]
    same = all(np.array_equal(rb, rs) for rb, rs in zip(res_b, solo))
    agree = max(float(np.max(np.abs(rb - rs) / np.abs(rs))) for rb, rs in zip(res_b, solo))
    flops = 0.0
    for _, job in entries:
        flops += (1 << job.log2_n) * job.shifts.shape[0] * inside_fraction(job.order, 10.0) * \
            tree_flops(job.order)
    tb_s = sum(ms_b) / len(ms_b) * 1e-3
    tp_s = sum(ms_p) / len(ms_p) * 1e-3
    print(json.dumps({
        "metric": "batched Keldysh-summed integrand points/s (64 parameter points x orders 1..10)",
        "value": points / tb_s, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": tb_s * 1e3, "higher_is_better": True,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "64 wide-band dots (eps_d~U[-3,3], V in {0,.5,1}, Gamma in {.5,1}, "
                               "beta=20) x orders 1..10 x 16 shifts, N_n = 2^(16+floor(2(n-1)/3)-%d)"
                               % args.shrink,
                   "items": len(entries), "points": points, "tile_len": info["tile_len"],
                   "grid_blocks": info["grid_blocks"], "plan_create_s": t_plan,
                   "lane_mappings": {n: list(g) for n, g in info["geometry"].items()}},
        "per_order_launches": {"value": points / tp_s, "unit": "points/s",
                               "ms_per_step": tp_s * 1e3},
        "speedup_vs_per_order": tp_s / tb_s,
        "bitwise_equal_to_per_order": bool(same),
        "max_rel_diff_vs_per_order": agree,
        "roofline": {"bound": "alu", "achieved": flops / tb_s / 1e12,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": flops / tb_s / 1e12 / FP64_VECTOR_PEAK_TFLOPS},
    }), flush=True)


def serving_measure(args):
    """Poisson sweep requests through the continuous-batching server, then the
    same trace through one plain launch per request in arrival order (first
    come first served, the library's default tile length: the plain path at
    its own best setting, whose per-shift sums the served results equal bit
    for bit).  Returns the figures as a dict."""
    import numpy as np
    import torch
    from paper_2002_12372_amd import qqmc
    from qqmc_inputs import serving_trace

    trace = serving_trace(seed=3, n_requests=args.requests, rate_hz=args.rate)
    pts = [(1 << r.job.log2_n) * r.job.shifts.shape[0] for r in trace]

    def serve(rate_scale):
        srv = qqmc.Server(hbm_budget_bytes=args.budget_gb << 30, max_slots=args.slots)
        t0 = srv.now()
        pending, done = {}, {}
        k = 0
        while k < len(trace) or pending:
            now = srv.now() - t0
            while k < len(trace) and trace[k].arrival_s / rate_scale <= now:
                pending[srv.submit(trace[k].dot, trace[k].job, 10.0)] = k
                k += 1
            for tk in list(pending):
                r = srv.poll(tk)
                if r is not None:
                    done[pending.pop(tk)] = r
            # completion times are the server's own clock: polling only
            # collects them, so it need not be frequent
            time.sleep(0.002)
        lat = np.array([done[i]["t_done"] - (t0 + trace[i].arrival_s / rate_scale)
                        for i in range(len(trace))])
        span = max(done[i]["t_done"] for i in done) - t0
        srv.close()
        return lat, span, done

    lat_s, span_s, done = serve(1.0)
    print("served %d requests in %.2f s" % (len(trace), span_s), file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    lat_p = []
    same = True
    busy = 0.0
    for i, r in enumerate(trace):
        now = time.perf_counter() - t0
        if now < r.arrival_s:
            time.sleep(r.arrival_s - now)
        ts = time.perf_counter()
        tb = qqmc.make_tables(r.dot)
        K = r.job.shifts.shape[0]
        buf = torch.zeros(2 * K, dtype=torch.float64, device="cuda")
        qqmc.eval_order_async(tb, r.job, 10.0, buf, None, tile_len=0, stream=stream)
        h = buf.cpu().numpy()
        q = (h[0::2] + 1j * h[1::2]) / (1 << r.job.log2_n)
        te = time.perf_counter()
        busy += te - ts
        lat_p.append(te - t0 - r.arrival_s)
        same = same and np.array_equal(q, done[i]["q_shift"])
    span_p = time.perf_counter() - t0
    print("plain launches: %d requests in %.2f s" % (len(trace), span_p), file=sys.stderr,
          flush=True)
    lat_p = np.array(lat_p)
    capacity = len(trace) / busy
    out = {
        "workload": "Poisson %.0f req/s, %d requests: eps_d~U[-3,3], Gamma~U[.5,2], "
                    "V~U[0,1], n~U{2..12}, N=2^k k~U{14..22}, 16 shifts, beta=20, t=10"
                    % (args.rate, args.requests),
        "slots": args.slots, "budget_gb": args.budget_gb,
        "p50_s": float(np.percentile(lat_s, 50)), "p99_s": float(np.percentile(lat_s, 99)),
        "makespan_s": span_s, "points_per_s": sum(pts) / span_s,
        "plain_per_request": {"p50_s": float(np.percentile(lat_p, 50)),
                              "p99_s": float(np.percentile(lat_p, 99)),
                              "makespan_s": span_p, "points_per_s": sum(pts) / span_p,
                              "busy_s": busy},
        "capacity_req_per_s_estimate": capacity,
        "results_bitwise_equal_served_vs_plain": bool(same),
    }
    return out, serve, trace, capacity


def run_serving(args):
    import numpy as np
    sv, serve, trace, capacity = serving_measure(args)
    out = {
        "metric": "p99 sweep latency (served), s",
        "value": sv["p99_s"], "unit": "s", "n_gpus": 1,
        "higher_is_better": False, "dtype": "f64", "data": "synthetic",
        "config": {"workload": sv["workload"], "slots": sv["slots"],
                   "budget_gb": sv["budget_gb"]},
        "served": {k: sv[k] for k in ("p50_s", "p99_s", "makespan_s", "points_per_s")},
        "plain_per_request": sv["plain_per_request"],
        "capacity_req_per_s_estimate": capacity,
        "results_bitwise_equal_served_vs_plain": sv["results_bitwise_equal_served_vs_plain"],
    }
    if args.find_capacity > 0:
        # bisection on the arrival rate: a rate is sustained when the queue
        # drains within 10% of the arrival window after the last arrival
        lo, hi = 0.25 * capacity, 1.5 * capacity
        steps = []
        for _ in range(args.find_capacity):
            mid = 0.5 * (lo + hi)
            scale = mid / args.rate
            lat_b, span_b, _ = serve(scale)
            window = trace[-1].arrival_s / scale
            ok = span_b - window <= 0.1 * window
            steps.append({"rate_req_per_s": mid, "p99_s": float(np.percentile(lat_b, 99)),
                          "drain_s": span_b - window, "sustained": bool(ok)})
            print("capacity probe %.2f req/s: drain %.2f s of %.2f s window -> %s"
                  % (mid, span_b - window, window, ok), file=sys.stderr, flush=True)
            if ok:
                lo = mid
            else:
                hi = mid
        scale = 0.8 * lo / args.rate
        lat_c, span_c, _ = serve(scale)
        out["max_sustained_rate"] = {
            "rate_req_per_s": lo, "bisection": steps,
            "at_0.8x": {"rate_req_per_s": 0.8 * lo, "p50_s": float(np.percentile(lat_c, 50)),
                        "p99_s": float(np.percentile(lat_c, 99)), "makespan_s": span_c}}
    if args.serve_at_fraction > 0:
        scale = capacity * args.serve_at_fraction / args.rate
        lat_f, span_f, _ = serve(scale)
        out["served_at_fraction_of_capacity"] = {
            "fraction": args.serve_at_fraction, "rate_req_per_s": args.rate * scale,
            "p50_s": float(np.percentile(lat_f, 50)), "p99_s": float(np.percentile(lat_f, 99)),
            "makespan_s": span_f}
    print(json.dumps(out), flush=True)


def run_stress(args):
    """Orders 11..14 (eps_d=-0.5, V=0.2), N = 2^18 x 16 shifts, with the
    model-function exactness check on device."""
    import numpy as np
    import torch
    from paper_2002_12372_amd import qqmc
    from paper_2002_12372_amd.flops import tree_flops, warp_flops
    from qqmc_inputs import STRESS_DOT as d, order_job

    stream = torch.cuda.current_stream()
    tables = qqmc.make_tables(d)
    rows = []
    for n in range(11, 15):
        job = order_job(4, n, args.stress_log2n, 16)
        # one untimed call, then the mean of three (each call is synchronous)
        q, mean, se = qqmc.eval_order(tables, job, 10.0)
        t0 = time.perf_counter()
        for _ in range(3):
            q, mean, se = qqmc.eval_order(tables, job, 10.0)
        dt = (time.perf_counter() - t0) / 3
        jm = order_job(4, n, args.stress_log2n, 16, mode=qqmc.MODE_MODEL)
        qm, _, _ = qqmc.eval_order(tables, jm, 10.0)
        pts = (1 << job.log2_n) * 16
        frac_in = counted_inside_fraction(job, 10.0, job.model_tau)
        fl = pts * (frac_in * tree_flops(n) + warp_flops(n))
        rows.append({"order": n, "Q": mean.real, "stderr": se, "seconds": dt,
                     "points_per_s": pts / dt, "inside_fraction": frac_in,
                     "tflops": fl / dt / 1e12,
                     "frac_fp64_peak": fl / dt / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                     "model_mode_max_dev": float(np.max(np.abs(qm - 1.0)))})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    print(json.dumps({"metric": "stress orders 11..14", "rows": rows,
                      "config": {"workload": "eps_d=-0.5, V=0.2, Gamma=1, beta=20, t=10, "
                                             "N=2^%d x 16 shifts" % args.stress_log2n}}),
          flush=True)


def run_learned(args):
    """The learned second warp (App. I) on the plain workload: learning cost,
    throughput through the learned warp, and the spread of the shift
    estimates against the exponential warp alone, for two first-warp taus."""
    import torch
    from paper_2002_12372_amd import qqmc
    from qqmc_inputs import TINY_DOT as d, order_job, sobol_job
    from qqmc_inputs import sobol as S

    n = args.order
    stream = torch.cuda.current_stream()
    tables = qqmc.make_tables(d)
    points = (1 << args.log2n) * args.shifts
    rows = []
    for tau in (1.0, 1.5):
        lj = order_job(41, n, args.learn_log2m, 1, model_tau=tau)
        sob = {}
        if args.sobol:
            sob = {"sobol_v": S.direction_numbers(n), "sobol_shift": S.digital_shifts(41, 1, n)[0]}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        model = qqmc.learn_model(tables, n, args.learn_log2m, lj.lattice_a, lj.shifts[0], tau,
                                 d.t_meas, args.learn_bins, args.learn_lambda, 1e-3, **sob)
        t_learn = time.perf_counter() - t0
        job = (sobol_job if args.sobol else order_job)(1, n, args.log2n, args.shifts,
                                                       model_tau=tau)
        sums = torch.zeros(2 * args.shifts, dtype=torch.float64, device="cuda")

        def step(m):
            qqmc.eval_order_async(tables, job, d.t_meas, sums, None, stream=stream, model=m)

        wall_e, _ = timed_steps(lambda: step(None), args.steps, args.warmup, stream)
        qe, me, se_e = qqmc.eval_order(tables, job, d.t_meas)
        wall_l, _ = timed_steps(lambda: step(model), args.steps, args.warmup, stream)
        ql, ml, se_l = qqmc.eval_order(tables, job, d.t_meas, model=model)
        rows.append({"tau": tau, "learn_s": t_learn,
                     "exponential": {"points_per_s": points * args.steps / wall_e,
                                     "Q": me.real, "stderr": se_e},
                     "learned": {"points_per_s": points * args.steps / wall_l,
                                 "Q": ml.real, "stderr": se_l},
                     "stderr_ratio": se_e / se_l})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        model.close()
    print(json.dumps({
        "metric": "learned-warp Keldysh-summed integrand points/s at n=%d FP64; stderr vs "
                  "exponential warp" % n,
        "value": rows[0]["learned"]["points_per_s"], "unit": "points/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic", "rows": rows,
        "config": {"workload": "plain dot (Gamma=1, eps_d=0, beta=20, V=0, t=10), order %d, "
                               "%s N=2^%d x %d shifts; model learned from 2^%d of those points, "
                               "%d bins, lambda %.3g, floor 1e-3"
                               % (n, "Sobol' points (digital shifts)," if args.sobol
                                  else "Korobov lattice", args.log2n, args.shifts,
                                  args.learn_log2m, args.learn_bins, args.learn_lambda)}}),
          flush=True)


def run_bethe(args):
    """The paper's benchmark (T = 0, eps_d = 0, V = 0, Gamma = 1, t = 30,
    tau = 0.95): Q_n for n = 1..12 against the printed Bethe-ansatz
    coefficients (tests/golden/bethe_qn.txt)."""
    from paper_2002_12372_amd import qqmc
    from qqmc_inputs import BETHE_DOT as d, order_job

    with open(os.path.join(ROOT, "tests", "golden", "bethe_qn.txt")) as f:
        bethe = {int(a): float(b) for a, b in (l.split() for l in f
                                               if l.strip() and not l.startswith("#"))}
    t0 = time.perf_counter()
    tables = qqmc.make_tables(d)
    t_tab = time.perf_counter() - t0
    rows = []
    for n in range(1, 13):
        job = order_job(1, n, args.log2n, 16, model_tau=0.95)
        t0 = time.perf_counter()
        q, mean, se = qqmc.eval_order(tables, job, d.t_meas)
        dt = time.perf_counter() - t0
        rows.append({"order": n, "Q": mean.real, "stderr": se, "bethe": bethe[n],
                     "rel_err": abs(mean.real - bethe[n]) / abs(bethe[n]),
                     "sigmas": (mean.real - bethe[n]) / se, "seconds": dt})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    print(json.dumps({"metric": "Bethe-ansatz benchmark Q_n, n=1..12", "rows": rows,
                      "tables_s": t_tab,
                      "config": {"workload": "T=0, eps_d=0, V=0, Gamma=1, t=30, tau=0.95, "
                                             "N=2^%d x 16 shifts, grid 65536 on [-30, 30]"
                                             % args.log2n}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload",
                    choices=["plain", "batched", "serving", "stress", "learned", "bethe", "geometry"],
                    default="plain")
    ap.add_argument("--order", type=int, default=8)
    ap.add_argument("--sobol", action="store_true",
                    help="plain workload on Sobol' points instead of the lattice")
    ap.add_argument("--current", action="store_true",
                    help="plain workload: the current on the paper's finite-bandwidth "
                         "parameters")
    ap.add_argument("--band", action="store_true",
                    help="plain workload on the paper's finite-bandwidth parameters")
    ap.add_argument("--alpha", default=None,
                    help="plain workload with the alpha-shifted interaction (a number, "
                         "or ns for alpha = n_sigma), on eps_d=0.3, V=0.4")
    ap.add_argument("--log2n", type=int, default=20)
    ap.add_argument("--shifts", type=int, default=32)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=1 << 19)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="plain workload: skip the serving trace (p99 sweep latency)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="run one plain device copy of this many bytes first (a reference "
                         "for hardware byte counters)")
    ap.add_argument("--params", type=int, default=64)
    ap.add_argument("--shrink", type=int, default=10,
                    help="batched: lattice sizes divided by 2^shrink")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--budget-gb", type=int, default=16)
    ap.add_argument("--serve-at-fraction", type=float, default=0.0)
    ap.add_argument("--find-capacity", type=int, default=0,
                    help="serving: bisection steps for the highest sustained arrival rate")
    ap.add_argument("--stress-log2n", type=int, default=18)
    ap.add_argument("--learn-log2m", type=int, default=16)
    ap.add_argument("--learn-bins", type=int, default=100)
    ap.add_argument("--learn-lambda", type=float, default=0.05)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    {"plain": run_plain, "batched": run_batched, "serving": run_serving,
     "stress": run_stress, "learned": run_learned, "bethe": run_bethe,
     "geometry": run_geometry}[args.workload](args)


if __name__ == "__main__":
    main()
