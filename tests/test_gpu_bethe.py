"""The paper's benchmark on the GPU path: T = 0, eps_d = 0, V = 0, Gamma = 1,
t = 30, exponential model tau = 0.95 (main text, "Benchmark"), against the
Bethe-ansatz coefficients the paper prints (tests/golden/bethe_qn.txt).

The estimates carry a randomised-QMC error bar (16 shifts) and the finite-t
and grid-interpolation bias of about 1e-6 relative measured on Q_1 by
quadrature in the oracle pins."""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from qqmc_inputs import BETHE_DOT, order_job

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_12372_amd import qqmc
    qqmc.lib()
    return qqmc


@pytest.fixture(scope="module")
def tables(q):
    return q.make_tables(BETHE_DOT)


def _bethe():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bethe_qn.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    return {int(a): float(b) for a, b in rows}


@pytest.mark.parametrize("n", list(range(1, 13)))
def test_bethe_coefficients(q, tables, n):
    log2_n = 16 if n <= 6 else (18 if n <= 10 else 20)
    job = order_job(1, n, log2_n, 16, model_tau=0.95)
    qs, mean, se = q.eval_order(tables, job, BETHE_DOT.t_meas)
    ref = _bethe()[n]
    print("n=%d Q=%.10g +- %.2g Bethe %.10g (%.2f sigma)"
          % (n, mean.real, se, ref, (mean.real - ref) / se))
    assert abs(mean.real - ref) < 5 * se + 3e-6 * abs(ref) + 1e-9
    assert abs(mean.imag) < 1e-10
