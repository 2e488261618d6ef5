"""The allocation-free Jacobi SVD (tt_svd_small_noalloc) against the
allocating one (tt_svd_small), through the C ABI: the same factors, on two
calls in a row on one context, the second with a smaller input (the
per-GPU static counters keep the first call's contents and must be
cleared by the second), and the blocked and single-workgroup forms."""
import numpy as np
import pytest

from gpu_util import make_ctx
from paper_2403_04946_amd import tt

pytestmark = pytest.mark.gpu


def _svd(ctx, b, noalloc):
    import torch

    m, k = b.shape
    B = torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()
    U = torch.empty(m * k, dtype=torch.complex128, device="cuda")
    s = torch.empty(k, dtype=torch.float64, device="cuda")
    sweeps = tt.tt_svd_small(ctx, B, U, s, noalloc=noalloc)
    torch.cuda.synchronize()
    return U.cpu().numpy().reshape(k, m).T, s.cpu().numpy(), sweeps


def test_noalloc_svd_matches_the_allocating_one():
    ctx = make_ctx()
    rng = np.random.default_rng(42)
    try:
        for m, k in [(320, 320), (96, 64), (40, 24)]:
            b = rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k))
            u0, s0, w0 = _svd(ctx, b, False)
            u1, s1, w1 = _svd(ctx, b, True)
            r = min(m, k)
            assert 0 < w1 < 60
            assert np.abs(s1 - s0).max() <= 1e-12 * s0[0]
            # singular vectors agree up to a phase per column (distinct sigma)
            ph = np.sum(u1[:, :r].conj() * u0[:, :r], axis=0)
            assert np.abs(np.abs(ph) - 1.0).max() < 1e-10
            w = u1[:, :r].conj().T @ b
            assert np.linalg.norm(w @ w.conj().T - np.diag(s1[:r] ** 2)) < 1e-11 * s1[0] ** 2
        with pytest.raises(tt.TTError):
            ctx.set_profiling(True)
            try:
                _svd(ctx, rng.standard_normal((8, 8)) + 0j, True)
            finally:
                ctx.set_profiling(False)
        null = tt.P(0)
        assert tt.lib().tt_svd_small_noalloc(ctx.h, 1537, 4, null, null, null, None) == -1
    finally:
        ctx.sync()
        ctx.close()
