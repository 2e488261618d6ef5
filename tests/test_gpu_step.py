"""RK4 step-truncation on the device against the CPU oracle.

Config-1 workload (d = 4 modes, n = 32 points on [-4, 4], nu = 0.05,
Gaussian IC from seed 0, dt = 1e-3): the device TT is compared with the
oracle's full-grid arrays over all 32^4 points; tolerance 1e-10 relative L2
(the FP64 target).  Larger shapes are checked against exact solutions
(viscous-only: per-axis matrix exponential) and pointwise oracle values.
"""
import os

import numpy as np
import pytest

from gpu_util import full, make_ctx, rel, upload
from oracle import closed_forms, fd, fullgrid, galerkin, tt_ref
from paper_2403_04946_amd import inputs, tt

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "d4_n32_cap8_100steps.npz")
GOLDEN_UNCAPPED = os.path.join(os.path.dirname(__file__), "golden", "d4_n32_uncapped_100steps.npz")
D, N, L, NU, DT = 4, 32, 4.0, 0.05, 1e-3


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    yield c
    c.sync()
    c.close()


def gpu_run(ctx, d, n, length, nu, mu, sig, dt, steps, eps, rmax, mode=tt.TT_APPLY_EXACT, ell=0, adv=1.0,
            seed=1):
    op = tt.Operator(ctx, d, n, length, nu, advection=adv)
    f = tt.Tensor(ctx, d, n, rmax)
    f.set_gaussian(mu, sig, length)
    rep = None
    for _ in range(steps):
        rep = tt.tt_step(ctx, op, f, dt, rmax, eps, mode, ell, seed)
    op.close()
    return f, rep


def oracle_problem(d=D, n=N, length=L, nu=NU):
    return fullgrid.Problem(galerkin.coefficient_B(d), galerkin.coefficient_D(d), nu, n, length)


@pytest.mark.parametrize("d,n", [(3, 32), (3, 48)])
def test_uncapped_matches_plain_oracle(ctx, d, n):
    # with d = 3 every unfolding rank is at most n, so a cap of n never binds
    # and the only truncation is the 1e-13 tolerance
    mu, sig = inputs.ic_params(d, 0)
    f, rep = gpu_run(ctx, d, n, L, NU, mu, sig, DT, 10, 1e-13, n)
    prob = oracle_problem(d=d, n=n)
    g = fullgrid.gaussian_ic(mu, sig, n, L)
    for _ in range(10):
        g = fullgrid.rk4_step(g, DT, prob.apply)
    err = rel(full(f), g)
    assert err < 1e-10, float(err)


def test_d4_n32_uncapped_100_steps_matches_plain_oracle(ctx):
    """The first workload without a rank cap: tolerance 1e-13, rank cap n^2
    (the largest unfolding rank at d = 4, so it never binds), exact operator
    application, 100 RK4 steps of dt = 1e-3; all 32^4 points against the
    oracle's plain full-grid RK4 (golden written by
    tests/golden/make_d4_n32_uncapped_golden.py, stored as a TT-SVD within
    1e-13 of the oracle's array).  Target 1e-10 relative L2."""
    z = np.load(GOLDEN_UNCAPPED, allow_pickle=False)
    mu, sig = z["mu"], z["sigma"]
    ref = fullgrid.tt_to_full([z[f"core{k}"] for k in range(D)])
    assert float(z["store_err"]) < 1e-12
    caps = [1, N, N * N, N, 1]
    op = tt.Operator(ctx, D, N, L, NU)
    f = tt.Tensor(ctx, D, N, caps)
    f.set_gaussian(mu, sig, L)
    maxr = 0
    for _ in range(100):
        rep = tt.tt_step(ctx, op, f, DT, N * N, 1e-13, tt.TT_APPLY_EXACT)
        maxr = max(maxr, rep["max_rank"])
    op.close()
    err = rel(full(f), ref)
    print(f"d=4 n=32 uncapped (eps 1e-13), 100 steps: rel L2 {err:.3e} vs plain RK4, ranks {f.ranks()}, "
          f"largest truncated rank {maxr}")
    assert abs(np.linalg.norm(full(f)) / float(z["norm"]) - 1) < 1e-10
    assert err < 1e-10
    f.close()


def test_d4_n32_capped_matches_truncation_aware_oracle(ctx):
    mu, sig = inputs.ic_params(D, 0)
    f, _ = gpu_run(ctx, D, N, L, NU, mu, sig, DT, 5, 1e-12, 8)
    prob = oracle_problem()
    g = fullgrid.gaussian_ic(mu, sig, N, L)
    for _ in range(5):
        g = fullgrid.truncated_rk4_step(g, DT, prob.apply, 1e-12, 8)
    assert max(f.ranks()) <= 8
    assert rel(full(f), g) < 1e-10


def test_d4_n32_cap8_100_steps_matches_golden(ctx):
    z = np.load(GOLDEN, allow_pickle=False)
    mu, sig = z["mu"], z["sigma"]
    ref = fullgrid.tt_to_full([z[f"core{k}"] for k in range(D)])
    f, _ = gpu_run(ctx, D, N, L, NU, mu, sig, DT, 100, 1e-12, 8)
    err = rel(full(f), ref)
    print(f"d=4 n=32 cap 8, 100 steps: rel L2 {err:.3e}, ranks {f.ranks()}, min gap {float(z['min_gap']):.4f}")
    assert err < 1e-10


def test_d4_n32_sketched_apply_matches_exact(ctx):
    mu, sig = inputs.ic_params(D, 0)
    a, _ = gpu_run(ctx, D, N, L, NU, mu, sig, DT, 10, 1e-12, 8)
    b, _ = gpu_run(ctx, D, N, L, NU, mu, sig, DT, 10, 1e-12, 8, mode=tt.TT_APPLY_SKETCH, ell=96)
    assert rel(full(b), full(a)) < 1e-10


def test_origin_value_and_hermitian_symmetry(ctx):
    import torch

    # phi(0) = 1 holds for the semi-discrete solution on odd-n grids (every
    # term of the operator carries a factor a_k); a binding rank cap would
    # perturb it by the truncation error, so d = 3 with cap n
    d, n = 3, 33
    mu, sig = inputs.ic_params(d, 3)
    f, rep = gpu_run(ctx, d, n, L, NU, mu, sig, DT, 20, 1e-13, n)
    c = (n - 1) // 2
    idx = inputs.random_points(d, n, 200, 4)
    idx[0] = c
    mirror = (n - 1 - idx).astype(np.int32)
    both = torch.from_numpy(np.concatenate([idx, mirror])).cuda()
    out = torch.zeros(400, dtype=torch.complex128, device="cuda")
    tt.tt_eval(ctx, f, both, out)
    v = out.cpu().numpy()
    assert abs(v[0] - 1.0) < 1e-10, float(abs(v[0] - 1.0))
    assert float(np.abs(v[:200] - np.conj(v[200:])).max()) < 1e-10
    assert float(np.abs(v).max()) <= 1.0 + 1e-6


@pytest.mark.parametrize("d,n,length,nu,dt,steps", [(20, 64, 6.0, 0.02, 5e-4, 40), (50, 128, 8.0, 0.01, 2e-4, 20)])
def test_viscous_only_matches_exponential(ctx, d, n, length, nu, dt, steps):
    mu, sig = inputs.ic_params(d, 0)
    f, _ = gpu_run(ctx, d, n, length, nu, mu, sig, dt, steps, 1e-13, 8, mode=tt.TT_APPLY_SKETCH, ell=8,
                   adv=0.0)
    facs = fullgrid.gaussian_ic_factors(mu, sig, n, length)
    ex = closed_forms.viscous_semidiscrete_cores([fa.reshape(1, n, 1) for fa in facs],
                                                 np.diag(galerkin.coefficient_D(d)), nu, dt * steps, n, length)
    got = f.get_cores()
    err = tt_ref.tt_diff_norm(got, ex) / tt_ref.tt_norm(ex)
    assert err < 1e-10, err


@pytest.mark.parametrize("rank,ell,prec,tol", [(1, 128, tt.TT_PREC_FP64, 1e-10), (2, 256, tt.TT_PREC_FP64, 1e-10),
                                               (1, 128, tt.TT_PREC_FP16X3, 3e-5), (2, 256, tt.TT_PREC_FP16X3, 3e-5),
                                               (1, 128, tt.TT_PREC_FP32, 3e-5)])
def test_sketched_apply_at_benchmark_shape_matches_pointwise_oracle(ctx, rank, ell, prec, tol):
    """The benchmark's operator (d=50, n=128) applied by the sketch in the
    plain, mixed and FP32 forms to inputs whose product the sketch width
    covers, against the oracle's operator evaluated point by point (the
    worst sampled point relative to the largest sampled |L x|: for the
    16-bit products about 1.5e-5, against their 1e-5 relative-L2 gate on
    whole stages)."""
    import torch

    d, n, length, nu = 50, 128, 8.0, 0.01
    op = tt.Operator(ctx, d, n, length, nu)
    x = inputs.random_tt(d, n, rank, 20 + rank)
    tx = upload(ctx, x)
    ty = tt.Tensor(ctx, d, n, ell)
    tt.tt_apply(ctx, op, tx, ty, tt.TT_APPLY_SKETCH, sketch_rank=ell, seed=9, precision=prec)
    idx = inputs.random_points(d, n, 12, 21)
    out = torch.zeros(12, dtype=torch.complex128, device="cuda")
    tt.tt_eval(ctx, ty, torch.from_numpy(idx).cuda(), out)
    ref = tt_ref.operator_at_points(x, idx, galerkin.coefficient_B(d), galerkin.coefficient_D(d), nu, n, length)
    scale = np.abs(ref).max()
    err = np.abs(out.cpu().numpy() - ref).max() / scale
    print(f"precision {prec}, rank {rank}: max pointwise error {err:.2e} of max |L x|")
    assert err < tol
    op.close()


def test_round_at_benchmark_shape(ctx):
    import torch

    d, n, r = 50, 128, 64
    x = inputs.random_tt(d, n, r, 30)
    t = upload(ctx, x)
    idx = inputs.random_points(d, n, 16, 31)
    tt.tt_round(ctx, t, 0.0, 0)
    out = torch.zeros(16, dtype=torch.complex128, device="cuda")
    tt.tt_eval(ctx, t, torch.from_numpy(idx).cuda(), out)
    ref = tt_ref.tt_eval(x, idx)
    assert np.abs(out.cpu().numpy() - ref).max() < 1e-10 * np.abs(ref).max()
    cores = t.get_cores()
    for c in cores[:-1]:
        v = c.reshape(-1, c.shape[2], order="F")
        assert np.abs(v.conj().T @ v - np.eye(v.shape[1])).max() < 1e-12
    # truncation to rank 32: error bounded by the discarded tails
    rep = tt.tt_round(ctx, t, 1e-6, 32)
    assert max(t.ranks()) <= 32
    err = tt_ref.tt_diff_norm(t.get_cores(), x)
    assert err <= np.sqrt(np.sum(np.square(rep["tail"]))) * (1 + 1e-8) + 1e-12 * rep["norm"]


def _near_origin_pairs(d, n, npts, seed):
    # points near the origin, where |phi| is of order one (far out in 50
    # dimensions the Gaussian factors make entries far smaller than the
    # pointwise resolution of the representation), and their mirror images
    idx = (n // 2 - 3 + inputs.random_points(d, 6, npts, seed)).astype(np.int32)
    return idx, (n - 1 - idx).astype(np.int32)


def test_apply_round_at_benchmark_shape_is_hermitian(ctx):
    import torch

    # T[L f] for the rank-one Gaussian IC: the sketch of width 128 exceeds the
    # operator's bond dimension (<= 102), so it is exact, and rounding is
    # equivariant under the reflection a -> -a with conjugation
    d, n, length, nu = 50, 128, 8.0, 0.01
    op = tt.Operator(ctx, d, n, length, nu)
    mu, sig = inputs.ic_params(d, 0)
    f = tt.Tensor(ctx, d, n, 1)
    f.set_gaussian(mu, sig, length)
    y = tt.Tensor(ctx, d, n, 128)
    tt.tt_apply(ctx, op, f, y, tt.TT_APPLY_SKETCH, sketch_rank=128, seed=3)
    tt.tt_round(ctx, y, 1e-6, 64)
    idx, mirror = _near_origin_pairs(d, n, 100, 5)
    out = torch.zeros(200, dtype=torch.complex128, device="cuda")
    tt.tt_eval(ctx, y, torch.from_numpy(np.concatenate([idx, mirror])).cuda(), out)
    v = out.cpu().numpy()
    assert float(np.abs(v[:100] - np.conj(v[100:])).max()) < 1e-10 * float(np.abs(v).max())
    op.close()


def test_step_at_benchmark_shape_properties(ctx):
    import torch

    d, n, length, nu = 50, 128, 8.0, 0.01
    mu, sig = inputs.ic_params(d, 0)
    f, rep = gpu_run(ctx, d, n, length, nu, mu, sig, 2e-4, 1, 1e-6, 64, mode=tt.TT_APPLY_SKETCH, ell=128)
    assert rep["max_rank"] <= 128 and max(f.ranks()) <= 64
    idx, mirror = _near_origin_pairs(d, n, 100, 6)
    out = torch.zeros(200, dtype=torch.complex128, device="cuda")
    tt.tt_eval(ctx, f, torch.from_numpy(np.concatenate([idx, mirror])).cuda(), out)
    v = out.cpu().numpy()
    assert np.isfinite(v).all()
    assert float(np.abs(v).max()) <= 1.0 + 1e-6
    # later stages apply the operator to inputs of rank > 1, where a width-128
    # sketch is no longer exact; the reflection symmetry then holds to the
    # sketch accuracy only
    asym = float(np.abs(v[:100] - np.conj(v[100:])).max() / np.abs(v).max())
    assert asym < 1e-4, asym


def test_tridiagonal_ic_matches_oracle_rounding(ctx):
    """The rank-3 initial condition with tridiagonal covariance at d=20,
    n=64 on [-6, 6] (seed 0): the device builds the exact nearest-neighbour
    product (bond ranks 64) and rounds it to rank 3, against the oracle's
    rounding of its own exact TT; the discarded tails are printed."""
    d, n, length = 20, 64, 6.0
    mu, sig, rho = inputs.ic_params_tridiag(d, 0)
    f = tt.Tensor(ctx, d, n, 3)
    rep = f.set_gaussian_tridiag(mu, sig, rho, length, 0.0, 3)
    ref, info = tt_ref.tt_round(closed_forms.tridiag_gaussian_tt(mu, sig, rho, n, length), 0.0, 3)
    tails = [np.sqrt(np.sum(s[3:] ** 2)) / info["norm"] for s in info["sigma"]]
    gaps = [s[2] / s[3] for s in info["sigma"]]
    print(f"rank-3 IC: largest discarded tail {max(tails):.2e} (relative), smallest gap {min(gaps):.1f}; "
          f"device tails {max(rep['tail']) / rep['norm']:.2e}")
    assert f.ranks() == [1] + [3] * (d - 1) + [1]
    err = tt_ref.tt_diff_norm(f.get_cores(), ref) / tt_ref.tt_norm(ref)
    assert err < 1e-10, err
    assert max(tails) < 1e-2
    f.close()


def test_viscous_only_from_tridiagonal_ic_matches_exponential(ctx):
    """Viscous-only RK4 (B = 0) at d=20, n=64, nu=0.02, dt=5e-4 from the
    rank-3 tridiagonal-covariance IC: the semi-discrete exact solution is the
    per-axis matrix exponential applied to the IC's cores (ranks kept)."""
    d, n, length, nu, dt, steps = 20, 64, 6.0, 0.02, 5e-4, 40
    mu, sig, rho = inputs.ic_params_tridiag(d, 0)
    op = tt.Operator(ctx, d, n, length, nu, advection=0.0)
    f = tt.Tensor(ctx, d, n, 8)
    f.set_gaussian_tridiag(mu, sig, rho, length, 0.0, 3)
    for _ in range(steps):
        tt.tt_step(ctx, op, f, dt, 8, 1e-13, tt.TT_APPLY_SKETCH, 16, 1)
    ic, _ = tt_ref.tt_round(closed_forms.tridiag_gaussian_tt(mu, sig, rho, n, length), 0.0, 3)
    ex = closed_forms.viscous_semidiscrete_cores(ic, np.diag(galerkin.coefficient_D(d)), nu, dt * steps, n, length)
    err = tt_ref.tt_diff_norm(f.get_cores(), ex) / tt_ref.tt_norm(ex)
    print(f"viscous-only from the rank-3 IC, {steps} steps: ranks {max(f.ranks())}, error {err:.2e}")
    assert err < 1e-10, err
    f.close()
    op.close()


def test_step_temporaries_follow_the_operator_ranks(ctx):
    """The step's cached temporaries are keyed by the operator's bond ranks:
    stepping with the viscous-only operator (ranks 2) and then, on the same
    context and shape, with the full operator (ranks up to 2d + 2) in exact
    mode works, and matches the same full step on a fresh context."""
    d, n, length, nu, dt, cap = 5, 16, 4.0, 0.05, 1e-3, 8
    mu, sig = inputs.ic_params(d, 2)
    visc = tt.Operator(ctx, d, n, length, nu, advection=0.0)
    full_op = tt.Operator(ctx, d, n, length, nu)
    a = tt.Tensor(ctx, d, n, cap)
    a.set_gaussian(mu, sig, length)
    tt.tt_step(ctx, visc, a, dt, cap, 1e-12, tt.TT_APPLY_EXACT)
    b = tt.Tensor(ctx, d, n, cap)
    b.set_gaussian(mu, sig, length)
    tt.tt_step(ctx, full_op, b, dt, cap, 1e-12, tt.TT_APPLY_EXACT)
    fresh = make_ctx()
    op2 = tt.Operator(fresh, d, n, length, nu)
    c = tt.Tensor(fresh, d, n, cap)
    c.set_gaussian(mu, sig, length)
    tt.tt_step(fresh, op2, c, dt, cap, 1e-12, tt.TT_APPLY_EXACT)
    assert b.ranks() == c.ranks()
    assert tt_ref.tt_diff_norm(b.get_cores(), c.get_cores()) <= 1e-13 * tt_ref.tt_norm(c.get_cores())
    for t in (a, b, visc, full_op, c, op2):
        t.close()
    fresh.sync()
    fresh.close()
