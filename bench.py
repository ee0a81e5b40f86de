"""Throughput of the QQMC hot path on one MI355X.

Workload (one step): the order-8 charge coefficient of the wide-band dot
(Gamma = 1, eps_d = 0, beta = 20, V = 0, t = 10), N = 2^20 Korobov lattice
points x 32 random shifts (33,554,432 points), warped with h(v) = exp(-v),
Keldysh sum over all 2^8 index vectors per point, reduced per shift on the
device.  Tables are built and resident in HBM before timing.

Prints one JSON line: points/s (all lattice points, in or out of the domain),
the roofline of the integrand kernel (FP64 vector ALU: algorithmic
operations of the elimination tree per point inside the domain, see
paper_2002_12372_amd/flops.py), and the CPU oracle timed on a bounded sample.
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
                  "paper_2002_12372_amd/csrc/qqmc_tree.h"]


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


def cpu_baseline(order, log2_n, lattice_a, shifts, count):
    import oracle
    from qqmc_inputs import TINY_DOT as d
    tb = oracle.Tables(d.eps_d, d.gamma, d.beta, d.bias_v, d.n_grid, d.t_half)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.eval_sums(tb, d.t_meas, order, log2_n, lattice_a, shifts[:1], 1.0, 0, 0, count,
                     n_threads=threads)
    dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": "lattice indices 0..%d of shift 0 (order %d, same dot and lattice), "
                      "%d OpenMP threads, %.1f s" % (count - 1, order, threads, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--order", type=int, default=8)
    ap.add_argument("--log2n", type=int, default=20)
    ap.add_argument("--shifts", type=int, default=32)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=1 << 15)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="run one plain device copy of this many bytes first (a reference "
                         "for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2002_12372_amd import qqmc
    from paper_2002_12372_amd.flops import tree_flops, warp_flops
    from qqmc_inputs import TINY_DOT as d, order_job

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n = args.order
    job = order_job(1, n, args.log2n, args.shifts)
    N = 1 << args.log2n
    points = N * args.shifts
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tables = qqmc.make_tables(d)
    sums = torch.zeros(2 * args.shifts, dtype=torch.float64, device="cuda")

    def step():
        qqmc.eval_order_async(tables, job, d.t_meas, sums, None, tile_len=args.tile, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1e3 / args.steps
    value = points * args.steps / wall

    frac_in = inside_fraction(n, d.t_meas / job.model_tau)
    alg_flops = points * (frac_in * tree_flops(n) + warp_flops(n))
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
        "config": {"workload": "charge coefficient Q_n of the wide-band Anderson dot "
                               "(Gamma=1, eps_d=0, beta=20, V=0, t=10), order %d, "
                               "Korobov lattice N=2^%d x %d random shifts, tau=1"
                               % (n, args.log2n, args.shifts),
                   "order": n, "lattice_points": N, "shifts": args.shifts,
                   "inside_fraction": frac_in,
                   "inside_points_per_s": value * frac_in},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": measured_traffic(n),
                     "flops_per_inside_point": tree_flops(n),
                     "avg_launch_ms": avg_launch_s * 1e3},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, args.log2n, job.lattice_a, job.shifts,
                                           args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
