"""GPU checks of the dense building blocks of TT rounding, through the C
ABI: the QR factorisation behind every orthogonalisation (block
Gram-Schmidt with Cholesky / Householder panels and its checked fallbacks)
and the one-sided Jacobi SVD of the small truncation factor, against numpy
and against the defining identities (A = QR, Q^H Q = I, B = U S V^H)."""
import numpy as np
import pytest

from gpu_util import make_ctx
from paper_2403_04946_amd import inputs, tt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    yield c
    c.sync()
    c.close()


def _cplx(rng, m, k):
    return rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k))


def _dev(a):
    import torch

    # column-major device copy: the transpose of a C-ordered tensor
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


def _qr(ctx, a):
    import torch

    m, k = a.shape
    A = _dev(a)
    Q = torch.empty((k, m), dtype=torch.complex128, device="cuda")
    R = torch.empty((k, k), dtype=torch.complex128, device="cuda")
    tt.tt_qr(ctx, A, Q, R)
    torch.cuda.synchronize()
    return Q.cpu().numpy().T, R.cpu().numpy().T


def _fallbacks(ctx):
    return ctx.dump_stats()["qr_fallbacks"]["launches"]


def _check_qr(a, q, r, tol=1e-12):
    k = a.shape[1]
    orth = np.linalg.norm(q.conj().T @ q - np.eye(k))
    res = np.linalg.norm(q @ r - a) / max(np.linalg.norm(a), 1e-300)
    assert orth < tol * max(1, k) ** 0.5, orth
    assert res < tol, res
    assert np.abs(np.tril(r, -1)).max() == 0.0


def _cases(rng, m, k):
    x = _cplx(rng, m, (k + 1) // 2)
    yield "random", _cplx(rng, m, k)
    yield "duplicate", np.hstack([x, x])[:, :k]
    yield "zero half", np.hstack([x, 0 * x])[:, :k]
    yield "rank 3", (_cplx(rng, m, 3) @ _cplx(rng, 3, k))
    yield "unit columns", np.eye(m, k, dtype=complex)[:, ::-1].copy()
    scaled = _cplx(rng, m, k) * np.logspace(0, -14, k)[None, :]
    yield "graded columns", scaled


@pytest.mark.parametrize("m,k", [(1, 1), (5, 3), (64, 64), (300, 32), (1000, 70), (2049, 100), (320, 320),
                                 (700, 200), (16384, 40)])
def test_qr_identities(ctx, m, k):
    rng = np.random.default_rng(m * 1000 + k)
    for name, a in _cases(rng, m, k):
        q, r = _qr(ctx, a)
        try:
            _check_qr(a, q, r)
        except AssertionError as e:
            raise AssertionError(f"{name}: {e}") from None


def test_qr_matches_numpy_up_to_phases(ctx):
    rng = np.random.default_rng(7)
    a = _cplx(rng, 3000, 96)
    q, r = _qr(ctx, a)
    qn, rn = np.linalg.qr(a)
    # unique up to a unit complex scaling of each column: Q = Qn D, R = D^H Rn
    dph = np.diag(qn.conj().T @ q)
    assert np.allclose(np.abs(dph), 1.0, atol=1e-11)
    assert np.linalg.norm(q - qn * dph[None, :]) < 1e-11
    assert np.linalg.norm(r - dph.conj()[:, None] * rn) / np.linalg.norm(rn) < 1e-12


def test_qr_fast_path_and_fallback(ctx):
    rng = np.random.default_rng(11)
    ctx.reset_stats()
    a = _cplx(rng, 4000, 64)
    q, r = _qr(ctx, a)
    _check_qr(a, q, r)
    assert _fallbacks(ctx) == 0  # well conditioned: Cholesky QR panels suffice
    # two columns of one panel that differ by 1e-9: the Cholesky pivot test
    # fails and the factorisation is redone with Householder panels
    b = _cplx(rng, 4000, 64)
    b[:, 5] = b[:, 4] + 1e-9 * _cplx(rng, 4000, 1)[:, 0]
    ctx.reset_stats()
    q, r = _qr(ctx, b)
    _check_qr(b, q, r)
    assert _fallbacks(ctx) >= 1


def test_qr_and_svd_reject_bad_shapes(ctx):
    null = tt.P(0)
    assert tt.lib().tt_qr(ctx.h, 4, 8, null, 4, null, null) == -1  # m < k
    assert tt.lib().tt_qr(ctx.h, 8, 0, null, 8, null, null) == -1  # k < 1
    assert tt.lib().tt_svd_small(ctx.h, 1537, 4, null, null, null, None) == -1  # beyond 1536 rows
    ctx.sync()


def _svd(ctx, b):
    import torch

    m, k = b.shape
    B = torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()  # column-major m x k
    U = torch.empty(m * k, dtype=torch.complex128, device="cuda")
    s = torch.empty(k, dtype=torch.float64, device="cuda")
    sweeps = tt.tt_svd_small(ctx, B, U, s)
    torch.cuda.synchronize()
    return U.cpu().numpy().reshape(k, m).T, s.cpu().numpy(), sweeps


@pytest.mark.parametrize("m,k", [(1, 1), (16, 16), (33, 33), (80, 80), (128, 128), (320, 320), (500, 500), (200, 50),
                                 (64, 100), (640, 640), (700, 24), (1000, 1000), (1024, 300), (1344, 1344),
                                 (1536, 200)])
def test_svd_small_matches_numpy(ctx, m, k):
    rng = np.random.default_rng(m + 7 * k)
    b = _cplx(rng, m, k)
    u, s, sweeps = _svd(ctx, b)
    sn = np.linalg.svd(b, compute_uv=False)
    r = min(m, k)
    assert sweeps < 60
    assert np.abs(s[:r] - sn).max() < 1e-12 * sn[0]
    assert np.all(np.diff(s) <= 0)
    if k > m:  # the extra singular values are zero, their U columns zero
        assert np.abs(s[r:]).max() < 1e-12 * sn[0]
    ur = u[:, :r]
    assert np.linalg.norm(ur.conj().T @ ur - np.eye(r)) < 1e-11
    # U^H B B^H U = S^2 (B = U S V^H)
    w = ur.conj().T @ b
    assert np.linalg.norm(w @ w.conj().T - np.diag(s[:r] ** 2)) < 1e-11 * sn[0] ** 2


def test_svd_small_graded_and_rank_deficient(ctx):
    rng = np.random.default_rng(3)
    m = 96
    uq, _ = np.linalg.qr(_cplx(rng, m, m))
    vq, _ = np.linalg.qr(_cplx(rng, m, m))
    spec = np.logspace(0, -10, m)
    spec[60:] = 0.0  # exact rank 60
    b = (uq * spec) @ vq.conj().T
    u, s, _ = _svd(ctx, b)
    assert np.abs(s[:60] - spec[:60]).max() < 1e-13
    assert np.abs(s[60:]).max() < 1e-13
    # the leading singular vectors span the constructed subspace: every
    # principal angle between the two 50-dimensional spaces is tiny
    cosines = np.linalg.svd(uq[:, :50].conj().T @ u[:, :50], compute_uv=False)
    assert cosines.min() > 1 - 1e-10


def test_jacobi_ends_on_the_all_pairs_test(ctx):
    """The blocked Jacobi SVD stops when one all-pairs application of the
    rotation test finds nothing to rotate, instead of running a sweep that
    rotates nothing.  The same matrix twice: the same sweep count and
    bitwise the same factors; the second run's first batch is as long as
    the first run needed, so it ends on that test and launches no sweep
    more than it needs."""
    rng = np.random.default_rng(11)
    b = _cplx(rng, 128, 128)
    ctx.reset_stats()
    u1, s1, w1 = _svd(ctx, b)
    st1 = ctx.dump_stats()
    u2, s2, w2 = _svd(ctx, b)
    st = ctx.dump_stats()
    assert st["jacobi_svds"]["launches"] == 2
    assert st["jacobi_check_passed"]["launches"] - st1["jacobi_check_passed"]["launches"] == 1
    assert w1 == w2 and 1 < w1 < 60
    assert np.array_equal(s1, s2) and np.array_equal(u1, u2)
    second_launched = st["jacobi_sweeps_launched"]["launches"] - st1["jacobi_sweeps_launched"]["launches"]
    second_needed = st["jacobi_sweeps_needed"]["launches"] - st1["jacobi_sweeps_needed"]["launches"]
    assert second_launched == second_needed == w1
    ctx.reset_stats()


def test_jacobi_sweep_limit_is_an_error(ctx):
    """A Jacobi SVD that reaches its sweep limit unconverged fails with
    TT_ENOCONV instead of handing back unorthogonal factors; the limit is
    forced from the host (one sweep), so every kernel still ends normally.
    Both the blocked form and the single-workgroup form (k <= 32), and a
    TT rounding whose truncation SVD stops unconverged."""
    rng = np.random.default_rng(5)
    ctx.set_option(tt.TT_OPT_JACOBI_MAX_SWEEPS, 1)
    try:
        for m, k in [(128, 128), (40, 24)]:
            with pytest.raises(tt.TTError) as e:
                _svd(ctx, _cplx(rng, m, k))
            assert e.value.code == tt.TT_ENOCONV
        x = tt.Tensor(ctx, 4, 16, 64)
        x.set_cores(inputs.random_tt(4, 16, [1, 16, 64, 16, 1], 3))
        with pytest.raises(tt.TTError) as e:
            tt.tt_round(ctx, x, 1e-6, 16)
        assert e.value.code == tt.TT_ENOCONV
        x.close()
    finally:
        ctx.set_option(tt.TT_OPT_JACOBI_MAX_SWEEPS, 60)
    # the default limit converges on the same kind of input
    _, s, sweeps = _svd(ctx, _cplx(rng, 128, 128))
    assert 1 < sweeps < 60
    with pytest.raises(tt.TTError):
        ctx.set_option(tt.TT_OPT_JACOBI_MAX_SWEEPS, 0)


@pytest.mark.parametrize("m,k", [(40, 200), (64, 64), (150, 133), (320, 320), (500, 257), (640, 640), (256, 1024)])
def test_fused_sweeps_match_the_launch_per_round_form(ctx, m, k):
    """The sweeps of one batch in one launch (workgroups meeting at grid
    barriers between rounds) against one launch per round: the same
    rotations in the same order, so bitwise the same factors and sweep
    count, on a graded matrix."""
    rng = np.random.default_rng(3 * m + k)
    b = _cplx(rng, m, k) * np.logspace(0, -6, k)[None, :]
    ctx.set_option(tt.TT_OPT_JACOBI_FUSED, 0)
    try:
        u0, s0, w0 = _svd(ctx, b)
    finally:
        ctx.set_option(tt.TT_OPT_JACOBI_FUSED, 1)
    u1, s1, w1 = _svd(ctx, b)
    # the count says where convergence was seen (a sweep without rotations,
    # or the all-pairs test after a batch), which depends on the batch
    # lengths (taken from the previous SVD of the size), not on the rotations
    assert abs(w0 - w1) <= 1 and 1 < w1 < 60
    assert np.array_equal(s0, s1) and np.array_equal(u0, u1)
    sn = np.linalg.svd(b, compute_uv=False)
    r = min(m, k)
    assert np.abs(s1[:r] - sn).max() < 1e-12 * sn[0]


def test_fused_barrier_wait_is_bounded(ctx):
    """A workgroup of the fused form polls a bounded number of times at each
    grid barrier.  With the limit forced to 0 from the host the workgroups
    give up, every kernel returns normally and the SVD fails with
    TT_ENOCONV; with the default limit the same context then computes the
    SVD."""
    rng = np.random.default_rng(9)
    b = _cplx(rng, 256, 256)
    ctx.set_option(tt.TT_OPT_JACOBI_WAIT_LIMIT, 0)
    try:
        with pytest.raises(tt.TTError) as e:
            _svd(ctx, b)
        assert e.value.code == tt.TT_ENOCONV
    finally:
        ctx.set_option(tt.TT_OPT_JACOBI_WAIT_LIMIT, 1 << 20)
    _, s, w = _svd(ctx, b)
    sn = np.linalg.svd(b, compute_uv=False)
    assert 1 < w < 60 and np.abs(s - sn).max() < 1e-12 * sn[0]
    with pytest.raises(tt.TTError):
        ctx.set_option(tt.TT_OPT_JACOBI_FUSED, 2)


@pytest.mark.parametrize("m,k", [(8192, 64), (10240, 80), (16384, 128), (4096, 320), (300, 300), (2000, 17)])
def test_wide_panels_match_narrow_panels(ctx, m, k):
    """The Cholesky form with panels of 64 columns (one factor and inverse
    per pass) against panels of 32, on the shapes of the benchmark's
    factorisations and on a square and a narrow one: both satisfy the
    defining identities, and their R factors agree to rounding (the QR of a
    full-rank matrix is unique up to column phases, fixed here by R's real
    positive diagonal)."""
    rng = np.random.default_rng(m + k)
    a = _cplx(rng, m, k) * np.logspace(0, -4, k)[None, :]
    out = {}
    for wide in (1, 0):
        ctx.set_option(tt.TT_OPT_QR_WIDE_PANELS, wide)
        try:
            ctx.reset_stats()
            q, r = _qr(ctx, a)
            out[wide] = (q, r, _fallbacks(ctx))
        finally:
            ctx.set_option(tt.TT_OPT_QR_WIDE_PANELS, 0)
        _check_qr(a, q, r)
        assert np.all(np.abs(np.diag(r).imag) < 1e-12 * np.abs(np.diag(r)).max())
        assert np.all(np.diag(r).real > 0)
    assert out[1][2] == 0 and out[0][2] == 0  # the fast form sufficed
    rn = np.abs(out[0][1]).max()
    assert np.abs(out[1][1] - out[0][1]).max() < 1e-11 * rn
    with pytest.raises(tt.TTError):
        ctx.set_option(tt.TT_OPT_QR_WIDE_PANELS, 2)
