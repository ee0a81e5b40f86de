"""qqmc_eval_order_noalloc (the entry point for callers that cannot
allocate device memory) against qqmc_eval_order_async, through the C ABI:
two calls in a row on the same device scratch, the second with a smaller
input, each equal bit for bit to the allocating entry point's per-shift
sums (the same tiles and the same fixed-order reductions); a call that
needs more than the scratch holds is refused with a clear error."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from qqmc_inputs import TINY_DOT, STRESS_DOT, order_job, sobol_job

pytestmark = pytest.mark.gpu

T_MEAS = 10.0


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_12372_amd import qqmc
    qqmc.lib()
    return qqmc


def _pair(q, gt, job, tile_len=0):
    K = job.shifts.shape[0]
    a = torch.zeros(2 * K, dtype=torch.float64, device="cuda")
    b = torch.full((2 * K,), float("nan"), dtype=torch.float64, device="cuda")
    na = q.eval_order_async(gt, job, T_MEAS, a, None, tile_len=tile_len)
    nb = q.eval_order_noalloc(gt, job, T_MEAS, b, tile_len=tile_len)
    torch.cuda.synchronize()
    return na, nb, a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_equals_async_two_calls_second_smaller(q):
    gt = q.make_tables(TINY_DOT)
    big = order_job(61, 8, 18, 16)          # 2^18 x 16 points, default tiles
    small = order_job(62, 5, 12, 4)         # a smaller call after it
    for job in (big, small):
        na, nb, a, b = _pair(q, gt, job)
        assert na == nb
        assert np.array_equal(a, b), job.order
    # and again the large one, after the small one left its data behind
    na, nb, a, b = _pair(q, gt, big)
    assert np.array_equal(a, b)


def test_noalloc_other_forms(q):
    """Sobol' points, the paired tree (alpha = n_sigma) and a high order."""
    gt = q.make_tables(TINY_DOT)
    for job in (sobol_job(63, 6, 14, 8), order_job(64, 7, 13, 4, alpha=0.5)):
        _, _, a, b = _pair(q, gt, job)
        assert np.array_equal(a, b)
    gs = q.make_tables(STRESS_DOT)
    _, _, a, b = _pair(q, gs, order_job(65, 11, 12, 2))
    assert np.array_equal(a, b)


def test_noalloc_refuses_beyond_scratch(q):
    gt = q.make_tables(TINY_DOT)
    job = order_job(66, 2, 22, 64)          # 2^22 / 64 x 64 tiles of 64: 64 MiB of tile sums
    buf = torch.zeros(128, dtype=torch.float64, device="cuda")
    with pytest.raises(q.QQMCError) as e:
        q.eval_order_noalloc(gt, job, T_MEAS, buf, tile_len=64)
    assert e.value.status == q.EINVAL and "MiB" in str(e.value)
