"""The explicit step-truncation schemes of Sec. 4.1 on the device, through
tt_step's scheme option: truncated Euler (eq. (adaptive-euler-method)) and
truncated explicit midpoint (eq. (adaptive-midpoint-method_2)), against the
CPU oracle's full-grid versions of the same schemes, plus the paper's order
study (local error against the Richardson extrapolation, Sec. 5.2) run on
the device path."""
import numpy as np
import pytest

from gpu_util import full, make_ctx, rel
from oracle import fullgrid, galerkin
from paper_2403_04946_amd import inputs, tt

pytestmark = pytest.mark.gpu
D, N, L, NU = 4, 32, 4.0, 0.05
SCHEMES = {"euler": (tt.TT_STEP_EULER, fullgrid.truncated_euler_step, 1),
           "midpoint": (tt.TT_STEP_MIDPOINT, fullgrid.truncated_midpoint_step, 2)}


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    yield c
    c.sync()
    c.close()


def _problem(d, n):
    return fullgrid.Problem(galerkin.coefficient_B(d), galerkin.coefficient_D(d), NU, n, L)


def _run(ctx, op, d, n, scheme, dt, steps, eps, cap, mode=tt.TT_APPLY_EXACT, ell=0, f=None):
    if f is None:
        mu, sig = inputs.ic_params(d, 0)
        f = tt.Tensor(ctx, d, n, cap)
        f.set_gaussian(mu, sig, L)
    rep = None
    for s in range(steps):
        rep = tt.tt_step(ctx, op, f, dt, cap, eps, mode, ell, 11 + s, scheme=scheme)
    return f, rep


@pytest.mark.parametrize("name", sorted(SCHEMES))
def test_uncapped_scheme_matches_oracle(ctx, name):
    scheme, ostep, _ = SCHEMES[name]
    d, n, dt, steps = 3, 32, 1e-3, 10
    op = tt.Operator(ctx, d, n, L, NU)
    f, rep = _run(ctx, op, d, n, scheme, dt, steps, 1e-13, n)
    mu, sig = inputs.ic_params(d, 0)
    g = fullgrid.gaussian_ic(mu, sig, n, L)
    prob = _problem(d, n)
    for _ in range(steps):
        g = ostep(g, dt, prob.apply, 0.0)
    err = rel(full(f), g)
    print(f"{name} d=3 uncapped, {steps} steps: rel L2 {err:.2e}")
    assert err < 1e-10, err
    assert rep["stages"] == {"euler": 1, "midpoint": 2}[name]
    f.close()
    op.close()


@pytest.mark.parametrize("name", sorted(SCHEMES))
@pytest.mark.parametrize("mode,ell", [(tt.TT_APPLY_EXACT, 0), (tt.TT_APPLY_SKETCH, 96)])
def test_capped_scheme_matches_truncation_aware_oracle(ctx, name, mode, ell):
    """d=4, n=32, cap 8, eps 1e-12: the truncations bind and the device
    must make the same choices as the oracle (the midpoint stage input,
    untruncated, reaches rank 16 before its operator application)."""
    scheme, ostep, _ = SCHEMES[name]
    dt, steps, cap = 1e-3, 8, 8
    op = tt.Operator(ctx, D, N, L, NU)
    f, rep = _run(ctx, op, D, N, scheme, dt, steps, 1e-12, cap, mode, ell)
    mu, sig = inputs.ic_params(D, 0)
    g = fullgrid.gaussian_ic(mu, sig, N, L)
    prob = _problem(D, N)
    for _ in range(steps):
        g = ostep(g, dt, prob.apply, 1e-12, cap)
    err = rel(full(f), g)
    print(f"{name} d=4 cap 8 mode {mode}: rel L2 {err:.2e}, ranks {f.ranks()}, step max rank {rep['max_rank']}")
    assert max(f.ranks()) <= cap
    assert err < 1e-10, err
    f.close()
    op.close()


def _device_richardson(ctx, op, d, scheme, order, dt):
    """||y_dt - R|| with R the Richardson extrapolation from two steps of
    dt/2, on the device (d = 3: a cap of n never binds; no truncation)."""
    cap = N
    y_full, _ = _run(ctx, op, d, N, scheme, dt, 1, 0.0, cap)
    y_half, _ = _run(ctx, op, d, N, scheme, 0.5 * dt, 2, 0.0, cap)
    diff = tt.Tensor(ctx, d, N, 2 * cap)
    tt.tt_axpy(ctx, 1.0, y_full, -1.0, y_half, diff)
    w = 2.0 ** order
    err = w / (w - 1.0) * tt.tt_norm(ctx, diff)
    for t in (y_full, y_half, diff):
        t.close()
    return err


@pytest.mark.parametrize("name", sorted(SCHEMES))
def test_order_study_on_device(ctx, name):
    """Local errors against the Richardson extrapolation fall like dt^(p+1)
    and agree with the oracle's values of the same estimate."""
    scheme, ostep, order = SCHEMES[name]
    d = 3
    op = tt.Operator(ctx, d, N, L, NU)
    prob = _problem(d, N)
    mu, sig = inputs.ic_params(d, 0)
    f0 = fullgrid.gaussian_ic(mu, sig, N, L)
    dts = [4e-3, 2e-3, 1e-3]
    dev = [_device_richardson(ctx, op, d, scheme, order, h) for h in dts]
    ora = [fullgrid.richardson_local_error(lambda f, h: ostep(f, h, prob.apply, 0.0), f0, h, order) for h in dts]
    slopes = [np.log2(dev[i] / dev[i + 1]) for i in range(2)]
    print(f"{name}: device local errors {dev}, slopes {slopes}")
    assert all(order + 1 - 0.3 < s < order + 1 + 0.3 for s in slopes), slopes
    # agreement to 1e-6 relative, up to FP64 rounding in the step
    # difference (about 1e-12 of the state's norm)
    scale = np.linalg.norm(f0)
    for a, b in zip(dev, ora):
        assert abs(a - b) <= 1e-6 * b + 1e-12 * scale, (a, b)
    op.close()


def test_unknown_scheme_is_rejected(ctx):
    op = tt.Operator(ctx, 3, 8, L, NU)
    f = tt.Tensor(ctx, 3, 8, 4)
    mu, sig = inputs.ic_params(3, 0)
    f.set_gaussian(mu, sig, L)
    with pytest.raises(tt.TTError):
        tt.tt_step(ctx, op, f, 1e-3, 4, 1e-8, tt.TT_APPLY_EXACT, 0, 1, scheme=9)
    f.close()
    op.close()


def test_midpoint_at_benchmark_shape(ctx):
    """d=50, n=128, cap 64, sketched apply: the midpoint step keeps the
    rank cap, phi stays bounded by 1 on sampled points and the midpoint and
    RK4 steps from the same state agree to second order in dt."""
    import torch

    d, n, length, nu, dt = 50, 128, 8.0, 0.01, 2e-4
    op = tt.Operator(ctx, d, n, length, nu)
    mu, sig = inputs.ic_params(d, 0)
    a = tt.Tensor(ctx, d, n, 64)
    a.set_gaussian(mu, sig, length)
    b = tt.Tensor(ctx, d, n, 64)
    b.copy_from(a)
    rep = tt.tt_step(ctx, op, a, dt, 64, 1e-6, tt.TT_APPLY_SKETCH, 80, 5, scheme=tt.TT_STEP_MIDPOINT)
    tt.tt_step(ctx, op, b, dt, 64, 1e-6, tt.TT_APPLY_SKETCH, 80, 5, scheme=tt.TT_STEP_RK4)
    assert rep["stages"] == 2 and max(a.ranks()) <= 64
    diff = tt.Tensor(ctx, d, n, 128)
    tt.tt_axpy(ctx, 1.0, a, -1.0, b, diff)
    gap = tt.tt_norm(ctx, diff) / tt.tt_norm(ctx, b)
    print(f"midpoint vs RK4, one step at d=50: rel L2 {gap:.2e}")
    assert gap < 1e-3
    idx = torch.from_numpy(inputs.random_points(d, n, 2048, 3)).cuda()
    out = torch.empty(2048, dtype=torch.complex128, device="cuda")
    tt.tt_eval(ctx, a, idx, out)
    assert float(out.abs().max()) <= 1.0 + 1e-6
    for t in (a, b, diff):
        t.close()
    op.close()


def test_round_with_zero_tolerance_keeps_the_tensor(ctx):
    """Rounding at eps = 0 of a TT whose bond ranks exceed the unfolding
    ranks (a sum, as the midpoint stage input is): the unfoldings have
    roundoff-level singular values, which must count as zero so that the
    rounded TT is still the same tensor (regression: they were kept with
    non-orthogonal singular vectors)."""
    from gpu_util import upload

    d, n = 3, 8
    a = inputs.random_tt(d, n, [1, 8, 8, 1], 4)
    b = inputs.random_tt(d, n, [1, 8, 8, 1], 5)
    x = upload(ctx, a, caps=16)
    y = upload(ctx, b, caps=16)
    z = tt.Tensor(ctx, d, n, 16)
    tt.tt_axpy(ctx, 1.0, x, 0.5, y, z)  # bond ranks 16 > n = 8
    ref = full(z)
    tt.tt_round(ctx, z, 0.0, 16, report=False)
    err = rel(full(z), ref)
    assert err < 1e-13, err
    assert max(z.ranks()) <= 8
    for t in (x, y, z):
        t.close()
