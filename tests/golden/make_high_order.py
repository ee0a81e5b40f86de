"""Writes high_order_q.json: the oracle's per-shift estimates Q^{(s)}
(Eq. (warped_int2)) for orders 10..14 on the stress dot (eps_d = -0.5,
V = 0.2, Gamma = 1, beta = 20, t = 10, tau = 1), Korobov lattice N = 2^14,
two random shifts drawn by order_job(seed 11, ...).

Calls only the oracle and the seeded input recipes; run from the repository
root:  python tests/golden/make_high_order.py   (a few minutes on 8 cores).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from qqmc_inputs import STRESS_DOT, order_job  # noqa: E402

SEED, LOG2_N, K, T_MEAS = 11, 14, 2, 10.0


def main():
    d = STRESS_DOT
    tb = oracle.Tables(d.eps_d, d.gamma, d.beta, d.bias_v, d.n_grid, d.t_half)
    out = {"dot": {"eps_d": d.eps_d, "gamma": d.gamma, "beta": d.beta, "bias_v": d.bias_v,
                   "n_grid": d.n_grid, "t_half": d.t_half},
           "t_meas": T_MEAS, "seed": SEED, "log2_n": LOG2_N, "n_shifts": K, "orders": []}
    for n in range(10, 15):
        job = order_job(SEED, n, LOG2_N, K)
        q, _, _ = oracle.eval_order(tb, T_MEAS, n, job.log2_n, job.lattice_a, job.shifts,
                                    job.model_tau)
        out["orders"].append({"order": n, "lattice_a": int(job.lattice_a),
                              "shifts": job.shifts.tolist(), "model_tau": job.model_tau,
                              "q_shift": [[float(v.real), float(v.imag)] for v in q]})
        print("order", n, q, flush=True)
    with open(os.path.join(HERE, "high_order_q.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
