"""ri_pd_residual_noalloc (the entry point for callers that cannot allocate) against
ri_pd_residual: Eq. 13 at the primal iterate for every block, bitwise the same FP64 sums,
on two calls in a row, the second on a smaller problem, so that what the first call left
in the static scratch cannot leak into the second."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from helpers import problem, to_plan

pytestmark = pytest.mark.gpu


def _pd(R, n, M, d, seed):
    x, uv, off = problem(n, M, d, "lognormal", seed)
    plan = R.Plan(n, uv, off)
    rng = np.random.default_rng(seed)
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    pd = R.PD(plan, R.Sara(n), torch.tensor(to_plan(y, plan.order()), dtype=torch.complex64, device="cuda"),
              np.ones(d), 0.49, 1.0 / 9.0, 1e-6, 1e-3, 3.0, 100.0)
    pd.set(0, torch.tensor(np.abs(synth.sky(n, 5, 10, rng)), dtype=torch.float32, device="cuda"))
    v = 0.01 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    pd.set(3, torch.tensor(v, dtype=torch.complex64, device="cuda"))
    return plan, pd


def _noalloc(pd, d):
    from paper_1610_08895_amd import _lib as L

    out = torch.full((d, 2), float("nan"), dtype=torch.float64, device="cuda")
    L.check(L.load().ri_pd_residual_noalloc(pd._h, ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return out


def test_noalloc_residual_matches_the_allocating_entry_point():
    import paper_1610_08895_amd as R

    assert torch.cuda.is_available()
    for n, M, d, seed in [(128, 60000, 9, 1), (64, 5000, 3, 2)]:  # the second call is smaller
        plan, pd = _pd(R, n, M, d, seed)
        got = _noalloc(pd, d).cpu().numpy()
        want = pd.residual().cpu().numpy()
        assert np.array_equal(got, want), (n, M, d)
        assert np.all(np.isfinite(got)) and np.all(got > 0)
        # the state is untouched: a second evaluation gives the same sums
        assert np.array_equal(_noalloc(pd, d).cpu().numpy(), want)


def test_noalloc_residual_rejects_bad_arguments():
    from paper_1610_08895_amd import _lib as L

    assert L.load().ri_pd_residual_noalloc(None, None, None) == L.RI_EINVAL
