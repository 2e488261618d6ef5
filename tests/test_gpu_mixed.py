"""GPU checks of the mixed-precision form: the operator application's
sketch contractions in a split 16-bit form on the matrix cores (FP32
accumulation), QR, SVD, truncation test and sums in FP64.

The gate is relative L2 <= 1e-5 against the plain FP64 form, per RK4 stage
from identical inputs: a stage is one operator application, its rounding
and the stage combination y = f + c dt k (rounded), so every stage below
starts from the FP64 path's own stage input.  Split-FP16x3 meets it;
split-BF16x3 (about 17 significant bits) does not, and its larger error is
pinned separately."""
import numpy as np
import pytest

from gpu_util import full, make_ctx, rel, upload
from oracle import fullgrid, galerkin
from paper_2403_04946_amd import inputs, tt

pytestmark = pytest.mark.gpu

GATE = 1e-5
D, N, LENGTH, NU, CAP, ELL, EPS, DT = 50, 128, 8.0, 0.01, 64, 80, 1e-6, 2e-4


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    yield c
    c.sync()
    c.close()


@pytest.fixture(scope="module")
def op(ctx):
    o = tt.Operator(ctx, D, N, LENGTH, NU)
    yield o
    o.close()


def _rel_tt(ctx, a, b):
    """||a - b|| / ||b|| for device TTs, via the difference TT."""
    caps = np.array(a.ranks()) + np.array(b.ranks())
    caps[0] = caps[-1] = 1
    diff = tt.Tensor(ctx, a.d, a.n, caps)
    tt.tt_axpy(ctx, 1.0, a, -1.0, b, diff)
    num = tt.tt_norm(ctx, diff)
    den = tt.tt_norm(ctx, b)
    diff.close()
    return num / den


def _apply_round(ctx, op, x, prec, seed):
    y = tt.Tensor(ctx, D, N, max(ELL, CAP))
    tt.tt_apply(ctx, op, x, y, tt.TT_APPLY_SKETCH, ELL, seed, precision=prec)
    tt.tt_round(ctx, y, EPS, CAP, report=False)
    return y


def _combine(ctx, coefs, xs, caps):
    z = tt.Tensor(ctx, D, N, caps)
    tt.tt_sum(ctx, coefs, xs, z)
    tt.tt_round(ctx, z, EPS, CAP, report=False)
    return z


@pytest.mark.parametrize("prec,bound", [(tt.TT_PREC_FP16X3, GATE), (tt.TT_PREC_BF16X3, 1e-3), (tt.TT_PREC_FP32, GATE)])
def test_mixed_sketched_apply_saturated(ctx, op, prec, bound):
    """The timed regime: a seeded random TT with every interior rank 64.
    FP16x3 and FP32 are within the gate of FP64; BF16x3 within 1e-3."""
    x = upload(ctx, inputs.random_tt(D, N, CAP, 0), caps=CAP)
    y64 = tt.Tensor(ctx, D, N, ELL)
    ymx = tt.Tensor(ctx, D, N, ELL)
    tt.tt_apply(ctx, op, x, y64, tt.TT_APPLY_SKETCH, ELL, 99, precision=tt.TT_PREC_FP64)
    tt.tt_apply(ctx, op, x, ymx, tt.TT_APPLY_SKETCH, ELL, 99, precision=prec)
    err = _rel_tt(ctx, ymx, y64)
    print(f"precision {prec} vs FP64 sketched apply, d=50 rank 64: rel L2 {err:.2e}")
    assert 0.0 < err < bound, err  # > 0: the split path really ran
    for t in (x, y64, ymx):
        t.close()


def test_mixed_stages_from_identical_inputs(ctx, op):
    """Two RK4 steps from the seeded Gaussian initial condition: every stage
    of the FP16x3 form, started from the FP64 path's stage input, gives a
    stage output within the gate of the FP64 one; the stage derivatives k
    themselves stay within 2e-4 (at sketch width 80 the sketch's own error
    against the exact product is about 4e-4 here)."""
    mu, sig = inputs.ic_params(D, 0)
    f = tt.Tensor(ctx, D, N, CAP)
    f.set_gaussian(mu, sig, LENGTH)
    cst = [0.5 * DT, 0.5 * DT, DT]
    worst = 0.0
    for step in range(2):
        y = f
        k64, kmx = [], []
        for s in range(4):
            seed = 1000 * step + s
            k64.append(_apply_round(ctx, op, y, tt.TT_PREC_FP64, seed))
            kmx.append(_apply_round(ctx, op, y, tt.TT_PREC_FP16X3, seed))
            kerr = _rel_tt(ctx, kmx[-1], k64[-1])
            assert kerr < 2e-4, (step, s, kerr)
            if s < 3:
                y64 = _combine(ctx, [1.0, cst[s]], [f, k64[-1]], 2 * CAP)
                ymx = _combine(ctx, [1.0, cst[s]], [f, kmx[-1]], 2 * CAP)
            else:
                w = [1.0, DT / 6, DT / 3, DT / 3, DT / 6]
                y64 = _combine(ctx, w, [f] + k64, 5 * CAP)
                ymx = _combine(ctx, w, [f] + kmx, 5 * CAP)
            err = _rel_tt(ctx, ymx, y64)
            print(f"step {step} stage {s}: k {kerr:.2e}  stage output {err:.2e}")
            worst = max(worst, err)
            assert err < GATE, (step, s, err)
            ymx.close()
            if y is not f:
                y.close()
            y = y64
        for t in k64 + kmx:
            t.close()
        f.copy_from(y)
        y.close()
    assert worst > 0.0
    f.close()


@pytest.mark.parametrize("prec", [tt.TT_PREC_FP16X3, tt.TT_PREC_FP32])
def test_mixed_step_from_identical_input(ctx, op, prec):
    """Whole RK4 steps through tt_step from the same Gaussian initial state."""
    mu, sig = inputs.ic_params(D, 1)
    f64 = tt.Tensor(ctx, D, N, CAP)
    f64.set_gaussian(mu, sig, LENGTH)
    fmx = tt.Tensor(ctx, D, N, CAP)
    fmx.copy_from(f64)
    tt.tt_step(ctx, op, f64, DT, CAP, EPS, tt.TT_APPLY_SKETCH, ELL, 12345, precision=tt.TT_PREC_FP64)
    tt.tt_step(ctx, op, fmx, DT, CAP, EPS, tt.TT_APPLY_SKETCH, ELL, 12345, precision=prec)
    err = _rel_tt(ctx, fmx, f64)
    print(f"precision {prec} vs FP64 RK4 step from the initial condition, d=50: rel L2 {err:.2e}")
    assert 0.0 < err < GATE, err
    for t in (f64, fmx):
        t.close()


def test_fp32_form_at_the_fp32_configuration(ctx):
    """The FP32 form at its own configuration (d=20, n=64 on [-6, 6],
    nu=0.02, cap 32, tolerance 1e-8, dt 5e-4, sketched apply of width 48):
    three RK4 steps from the Gaussian initial condition, each from the FP64
    path's input, within the gate of the FP64 step."""
    d, n, length, nu, cap, eps, dt, ell = 20, 64, 6.0, 0.02, 32, 1e-8, 5e-4, 48
    op2 = tt.Operator(ctx, d, n, length, nu)
    mu, sig = inputs.ic_params(d, 0)
    f64 = tt.Tensor(ctx, d, n, cap)
    f64.set_gaussian(mu, sig, length)
    f32 = tt.Tensor(ctx, d, n, cap)
    for s in range(3):
        f32.copy_from(f64)
        tt.tt_step(ctx, op2, f64, dt, cap, eps, tt.TT_APPLY_SKETCH, ell, 50 + s, precision=tt.TT_PREC_FP64)
        tt.tt_step(ctx, op2, f32, dt, cap, eps, tt.TT_APPLY_SKETCH, ell, 50 + s, precision=tt.TT_PREC_FP32)
        err = _rel_tt(ctx, f32, f64)
        print(f"FP32 vs FP64 step {s} at d=20: rel L2 {err:.2e}, ranks {max(f64.ranks())}")
        assert 0.0 < err < GATE, (s, err)
    for t in (f64, f32):
        t.close()
    op2.close()


def test_mixed_d4_n32_trajectory_against_oracle(ctx):
    """d=4, n=32, cap 8 for 20 steps with the sketched apply in the FP16x3
    form: within the gate of the truncation-aware FP64 oracle."""
    d, n, length, nu, dt, steps, eps, cap = 4, 32, 4.0, 0.05, 1e-3, 20, 1e-12, 8
    op = tt.Operator(ctx, d, n, length, nu)
    f = tt.Tensor(ctx, d, n, cap)
    mu, sig = inputs.ic_params(d, 0)
    f.set_gaussian(mu, sig, length)
    for s in range(steps):
        tt.tt_step(ctx, op, f, dt, cap, eps, tt.TT_APPLY_SKETCH, 96, 777 + s, precision=tt.TT_PREC_FP16X3)
    got = full(f)
    prob = fullgrid.Problem(galerkin.coefficient_B(d), galerkin.coefficient_D(d), nu, n, length)
    ref = fullgrid.gaussian_ic(mu, sig, n, length)
    for _ in range(steps):
        ref = fullgrid.truncated_rk4_step(ref, dt, prob.apply, eps, cap)
    err = rel(got, ref)
    print(f"FP16x3 d=4, {steps} steps: rel L2 vs oracle {err:.2e}")
    assert err < GATE, err
    f.close()
    op.close()


def test_mixed_precision_is_rejected_when_unknown(ctx):
    d, n = 3, 8
    op = tt.Operator(ctx, d, n, 4.0, 0.05)
    x = upload(ctx, inputs.random_tt(d, n, 2, 0), caps=4)
    y = tt.Tensor(ctx, d, n, 16)
    with pytest.raises(tt.TTError):
        tt.tt_apply(ctx, op, x, y, tt.TT_APPLY_SKETCH, 8, 1, precision=7)
    f = upload(ctx, inputs.random_tt(d, n, 2, 0), caps=4)
    with pytest.raises(tt.TTError):
        tt.tt_step(ctx, op, f, 1e-3, 4, 1e-8, tt.TT_APPLY_SKETCH, 8, 1, precision=4)
    for t in (x, y, f):
        t.close()
    op.close()


@pytest.mark.parametrize("mixed_passes", [1, 0])
def test_mixed_power_pass_stage_within_gate(ctx, op, mixed_passes):
    """The plain form's sketched apply has one power pass; in the mixed form
    the split-FP16x3 products cover the Gaussian sketch pass and (option 1,
    the default) the power pass, the last pass being FP64.  One stage from
    the saturated input at d=50 (derivative rounded, combination rounded)
    against the FP64 form from the same input and seeds: within the gate."""
    x = tt.Tensor(ctx, D, N, CAP)
    x.set_cores(inputs.random_tt(D, N, CAP, 0))
    ctx.set_option(tt.TT_OPT_SKETCH_MIXED_PASSES, mixed_passes)
    outs = {}
    try:
        for prec in (tt.TT_PREC_FP64, tt.TT_PREC_FP16X3):
            k = tt.Tensor(ctx, D, N, max(ELL, CAP))
            tt.tt_apply(ctx, op, x, k, tt.TT_APPLY_SKETCH, ELL, 5, precision=prec, power=1)
            tt.tt_round(ctx, k, EPS, CAP, report=False)
            y = tt.Tensor(ctx, D, N, 2 * CAP)
            tt.tt_axpy(ctx, 1.0, x, 0.5 * DT, k, y)
            tt.tt_round(ctx, y, EPS, CAP, report=False)
            outs[prec] = (k, y)
    finally:
        ctx.set_option(tt.TT_OPT_SKETCH_MIXED_PASSES, 1)
    ek = _rel_tt(ctx, outs[tt.TT_PREC_FP16X3][0], outs[tt.TT_PREC_FP64][0])
    ey = _rel_tt(ctx, outs[tt.TT_PREC_FP16X3][1], outs[tt.TT_PREC_FP64][1])
    print(f"mixed passes {mixed_passes}: derivative {ek:.2e}, stage output {ey:.2e}")
    assert ey < GATE
    assert ek < 1e-3
    for pair in outs.values():
        for t in pair:
            t.close()
    x.close()
    with pytest.raises(tt.TTError):
        ctx.set_option(tt.TT_OPT_SKETCH_MIXED_PASSES, 2)
