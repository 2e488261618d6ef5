"""Pins for oracle.fullgrid and oracle.closed_forms."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import closed_forms, fd, fullgrid, galerkin, tt_ref
from paper_2403_04946_amd import inputs


def kron_operator(b, dm, nu, d, n, length):
    """The grid operator assembled as a sparse matrix from Kronecker products
    (an independent route to the same semi-discrete operator)."""
    eye = sp.identity(n, format="csr")
    x = sp.csr_matrix(fd.position(n, length))
    g = sp.csr_matrix(fd.first_derivative(n, length))
    l2 = sp.csr_matrix(fd.second_derivative(n, length))

    def on_axis(mats):
        out = None
        for k in range(d):
            m = mats.get(k, eye)
            out = m if out is None else sp.kron(out, m, format="csr")
        return out

    total = sp.csr_matrix((n**d, n**d), dtype=np.complex128)
    for k in range(d):
        for j in range(d):
            for l in range(d):
                c = b[k, j, l]
                if c == 0.0:
                    continue
                if j == l:
                    deriv = on_axis({j: l2})
                else:
                    deriv = on_axis({j: g}) @ on_axis({l: g})
                total = total + (0.5j * c) * (on_axis({k: x}) @ deriv)
            if dm[k, j] != 0.0:
                total = total + (nu * dm[k, j]) * (on_axis({k: x}) @ on_axis({j: g}))
    return total.tocsr()


@pytest.mark.parametrize("d,n", [(3, 7), (4, 5), (5, 4)])
def test_assembly_matches_kronecker_matrix(d, n):
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    prob = fullgrid.Problem(b, dm, 0.05, n, 4.0)
    mat = kron_operator(b, dm, 0.05, d, n, 4.0)
    rng = np.random.default_rng(7)
    f = rng.standard_normal((n,) * d) + 1j * rng.standard_normal((n,) * d)
    got = prob.apply(f).ravel()
    ref = mat @ f.ravel()
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_rk4_fourth_order_against_matrix_exponential():
    d, n, length, nu = 3, 7, 4.0, 0.05
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    prob = fullgrid.Problem(b, dm, nu, n, length)
    mat = kron_operator(b, dm, nu, d, n, length)
    mu, sig = inputs.ic_params(d, 3)
    f0 = fullgrid.gaussian_ic(mu, sig, n, length)
    tend = 0.4
    exact = spla.expm_multiply(tend * mat, f0.ravel()).reshape(f0.shape)
    errs = []
    for steps in (4, 8, 16):
        f = f0.copy()
        for _ in range(steps):
            f = fullgrid.rk4_step(f, tend / steps, prob.apply)
        errs.append(fullgrid.rel_l2(f, exact))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.6 < r < 4.4 for r in rates), (errs, rates)


def test_truncated_euler_and_midpoint_are_the_matrix_polynomials():
    """Without truncation the two explicit schemes are the Taylor polynomials
    of exp(dt M) of degree one and two, M the independently assembled
    Kronecker-product matrix."""
    d, n, length, nu, dt = 3, 6, 4.0, 0.05, 3e-2
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    prob = fullgrid.Problem(b, dm, nu, n, length)
    mat = kron_operator(b, dm, nu, d, n, length)
    rng = np.random.default_rng(5)
    f = rng.standard_normal((n,) * d) + 1j * rng.standard_normal((n,) * d)
    v = f.ravel()
    mv = mat @ v
    euler = v + dt * mv
    midpoint = v + dt * mv + 0.5 * dt * dt * (mat @ mv)
    got_e = fullgrid.truncated_euler_step(f, dt, prob.apply, 0.0).ravel()
    got_m = fullgrid.truncated_midpoint_step(f, dt, prob.apply, 0.0).ravel()
    assert np.linalg.norm(got_e - euler) <= 1e-13 * np.linalg.norm(euler)
    assert np.linalg.norm(got_m - midpoint) <= 1e-13 * np.linalg.norm(midpoint)
    # a dropped half in the midpoint stage is caught: it would equal Euler
    # applied twice less a term of size dt^2/2 |M^2 f|
    assert np.linalg.norm(got_m - euler) > 1e-3 * np.linalg.norm(euler)


@pytest.mark.parametrize("scheme,order", [("euler", 1), ("midpoint", 2)])
def test_explicit_scheme_global_order_against_matrix_exponential(scheme, order):
    d, n, length, nu, tend = 3, 7, 4.0, 0.05, 0.2
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    prob = fullgrid.Problem(b, dm, nu, n, length)
    mat = kron_operator(b, dm, nu, d, n, length)
    mu, sig = inputs.ic_params(d, 3)
    f0 = fullgrid.gaussian_ic(mu, sig, n, length)
    exact = spla.expm_multiply(tend * mat, f0.ravel()).reshape(f0.shape)
    step = {"euler": fullgrid.truncated_euler_step, "midpoint": fullgrid.truncated_midpoint_step}[scheme]
    errs = []
    for steps in (40, 80, 160):
        f = f0.copy()
        for _ in range(steps):
            f = step(f, tend / steps, prob.apply, 0.0)
        errs.append(fullgrid.rel_l2(f, exact))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(order - 0.25 < r < order + 0.25 for r in rates), (errs, rates)


@pytest.mark.parametrize("scheme,order", [("euler", 1), ("midpoint", 2), ("rk4", 4)])
def test_richardson_local_error_slopes(scheme, order):
    """The paper's order study: the local error against the Richardson
    extrapolation falls like dt^(p+1) for a method of order p."""
    d, n, length, nu = 3, 6, 4.0, 0.05
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    prob = fullgrid.Problem(b, dm, nu, n, length)
    mu, sig = inputs.ic_params(d, 2)
    f0 = fullgrid.gaussian_ic(mu, sig, n, length)
    step = {"euler": lambda f, h: fullgrid.truncated_euler_step(f, h, prob.apply, 0.0),
            "midpoint": lambda f, h: fullgrid.truncated_midpoint_step(f, h, prob.apply, 0.0),
            "rk4": lambda f, h: fullgrid.rk4_step(f, h, prob.apply)}[scheme]
    dts = [2e-2, 1e-2, 5e-3]
    errs = [fullgrid.richardson_local_error(step, f0, h, order) for h in dts]
    slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(order + 1 - 0.3 < s < order + 1 + 0.3 for s in slopes), (errs, slopes)


def test_richardson_estimate_matches_exact_local_error():
    """For Euler the Richardson estimate equals the true local error to
    leading order: both are dt^2/2 |M^2 f| (pins the extrapolation weights)."""
    d, n, length, nu, dt = 3, 6, 4.0, 0.05, 1e-3
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    prob = fullgrid.Problem(b, dm, nu, n, length)
    mat = kron_operator(b, dm, nu, d, n, length)
    mu, sig = inputs.ic_params(d, 2)
    f0 = fullgrid.gaussian_ic(mu, sig, n, length)
    est = fullgrid.richardson_local_error(lambda f, h: fullgrid.truncated_euler_step(f, h, prob.apply, 0.0), f0, dt, 1)
    true = np.linalg.norm(spla.expm_multiply(dt * mat, f0.ravel()) - (f0.ravel() + dt * (mat @ f0.ravel())))
    assert abs(est / true - 1.0) < 0.05, (est, true)


def test_numerical_diffusion_term():
    """The stabilisation term kappa sum_k d^2/da_k^2: the grid operator with
    it equals the Kronecker assembly plus kappa sum_k L2_k, and on its own
    (B = D = 0) its semi-discrete flow is the per-axis matrix exponential of
    kappa L2 (a product of one-dimensional heat flows)."""
    d, n, length, nu, kappa = 3, 7, 4.0, 0.05, 0.02
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    prob = fullgrid.Problem(b, dm, nu, n, length, diffusion=kappa)
    mat = kron_operator(b, dm, nu, d, n, length)
    l2 = sp.csr_matrix(fd.second_derivative(n, length))
    eye = sp.identity(n, format="csr")
    for k in range(d):
        term = None
        for j in range(d):
            m = l2 if j == k else eye
            term = m if term is None else sp.kron(term, m, format="csr")
        mat = mat + kappa * term
    rng = np.random.default_rng(9)
    f = rng.standard_normal((n,) * d) + 1j * rng.standard_normal((n,) * d)
    assert np.linalg.norm(prob.apply(f).ravel() - mat @ f.ravel()) <= 1e-12 * np.linalg.norm(mat @ f.ravel())
    # heat flow alone: exp(t kappa sum_k L2_k) = kron of exp(t kappa L2)
    heat = fullgrid.Problem(np.zeros((d, d, d)), np.zeros((d, d)), 0.0, n, length, diffusion=kappa)
    t = 0.3
    g = f.copy()
    for _ in range(300):
        g = fullgrid.rk4_step(g, t / 300, heat.apply)
    e1 = __import__("scipy.linalg", fromlist=["expm"]).expm(t * kappa * fd.second_derivative(n, length))
    ref = f
    for k in range(d):
        ref = fullgrid.apply_along(e1, ref, k)
    assert fullgrid.rel_l2(g, ref) < 1e-10


def test_implicit_steps_match_sparse_direct_solve():
    """The implicit steps against an LU solve of the independently assembled
    Kronecker matrix: (I - dt M) x = f and (I - dt/2 M) x = (I + dt/2 M) f."""
    d, n, length, nu, dt = 3, 7, 4.0, 0.05, 2e-2
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    prob = fullgrid.Problem(b, dm, nu, n, length)
    mat = kron_operator(b, dm, nu, d, n, length).tocsc()
    eye = sp.identity(n**d, format="csc", dtype=np.complex128)
    mu, sig = inputs.ic_params(d, 1)
    f = fullgrid.gaussian_ic(mu, sig, n, length)
    v = f.ravel()
    euler = spla.splu(eye - dt * mat).solve(v)
    midpoint = spla.splu(eye - 0.5 * dt * mat).solve(v + 0.5 * dt * (mat @ v))
    got_e = fullgrid.implicit_euler_step(f, dt, prob.apply).ravel()
    got_m = fullgrid.implicit_midpoint_step(f, dt, prob.apply).ravel()
    assert np.linalg.norm(got_e - euler) <= 1e-12 * np.linalg.norm(euler)
    assert np.linalg.norm(got_m - midpoint) <= 1e-12 * np.linalg.norm(midpoint)
    # the two differ at second order: a swapped shift sign is caught
    assert np.linalg.norm(got_m - got_e) > 1e-5 * np.linalg.norm(euler)


@pytest.mark.parametrize("scheme,order", [("implicit_euler", 1), ("implicit_midpoint", 2)])
def test_implicit_scheme_global_order(scheme, order):
    d, n, length, nu, tend = 3, 7, 4.0, 0.05, 0.2
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    prob = fullgrid.Problem(b, dm, nu, n, length)
    mat = kron_operator(b, dm, nu, d, n, length)
    mu, sig = inputs.ic_params(d, 3)
    f0 = fullgrid.gaussian_ic(mu, sig, n, length)
    exact = spla.expm_multiply(tend * mat, f0.ravel()).reshape(f0.shape)
    step = getattr(fullgrid, scheme + "_step")
    errs = []
    for steps in (20, 40, 80):
        f = f0.copy()
        for _ in range(steps):
            f = step(f, tend / steps, prob.apply)
        errs.append(fullgrid.rel_l2(f, exact))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(order - 0.25 < r < order + 0.25 for r in rates), (errs, rates)


def test_viscous_only_semidiscrete_exact():
    d, n, length, nu, dt, steps = 3, 16, 4.0, 0.05, 1e-3, 50
    b = np.zeros((d, d, d))
    dm = galerkin.coefficient_D(d)
    prob = fullgrid.Problem(b, dm, nu, n, length)
    mu, sig = inputs.ic_params(d, 1)
    f = fullgrid.gaussian_ic(mu, sig, n, length)
    for _ in range(steps):
        f = fullgrid.rk4_step(f, dt, prob.apply)
    facs = fullgrid.gaussian_ic_factors(mu, sig, n, length)
    cores = [fa.reshape(1, n, 1) for fa in facs]
    ex = closed_forms.viscous_semidiscrete_cores(cores, np.diag(dm), nu, steps * dt, n, length)
    assert fullgrid.rel_l2(f, fullgrid.tt_to_full(ex)) < 1e-12


def test_viscous_only_continuous_second_order_in_h():
    d, length, nu, tend = 2, 6.0, 0.5, 0.5
    b = np.zeros((d, d, d))
    dm = galerkin.coefficient_D(d)
    mu, sig = np.array([0.6, -0.4]), np.array([0.5, 0.7])
    errs = []
    for n in (33, 65, 129):
        prob = fullgrid.Problem(b, dm, nu, n, length)
        f = fullgrid.gaussian_ic(mu, sig, n, length)
        for _ in range(25):
            f = fullgrid.rk4_step(f, tend / 25, prob.apply)
        facs = closed_forms.viscous_continuous_factors(mu, sig, nu, tend, n, length)
        ex = np.multiply.outer(facs[0], facs[1])
        errs.append(fullgrid.rel_l2(f, ex))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[0] < 1e-2 and all(1.7 < r < 2.4 for r in rates), (errs, rates)


def _deterministic_error(n, sign=1.0):
    """Max error over the inner half of the box [-L/2, L/2]^3 (the one-sided
    closures make the boundary layer converge more slowly)."""
    d, length, nu, tend, steps = 3, 4.0, 0.05, 0.3, 80
    b = sign * galerkin.coefficient_B(d)
    dm = galerkin.coefficient_D(d)
    mu = np.array([0.9, -0.7, 0.6])
    prob = fullgrid.Problem(b, dm, nu, n, length)
    f = closed_forms.deterministic_phi(mu, n, length)
    for _ in range(steps):
        f = fullgrid.rk4_step(f, tend / steps, prob.apply)
    u = closed_forms.galerkin_trajectory(mu, galerkin.coefficient_B(d), dm, nu, tend)
    err = np.abs(f - closed_forms.deterministic_phi(u, n, length))
    inner = np.abs(fd.grid(n, length)) <= length / 2
    return float(err[np.ix_(inner, inner, inner)].max())


def test_deterministic_state_pins_advective_term():
    e17, e33 = _deterministic_error(17), _deterministic_error(33)
    assert e33 < 6e-3 and 3.4 < e17 / e33 < 4.6, (e17, e33)
    # a sign error in the advective term is far outside that tolerance
    assert _deterministic_error(33, sign=-1.0) > 20 * e33


def _average_over_gaussian_states(mu, sig, b, dm, nu, t, n, length, q=8):
    """E[exp(i a . u(t))] over initial states u(0) ~ N(mu, diag(sig^2)), by
    tensor Gauss-Hermite quadrature (q nodes per mode) over u(0), each node
    carried to time t by the Galerkin ODE.  The PDE is linear in phi, and
    from a deterministic state its solution is exp(i a . u(t)); averaged
    over the Gaussian it is the solution from the Gaussian characteristic
    function (the Monte-Carlo check of the nonlinear part, with quadrature
    in place of sampling, so without sampling noise)."""
    x, w = np.polynomial.hermite_e.hermegauss(q)
    w = w / w.sum()
    out = np.zeros((n,) * len(mu), dtype=np.complex128)
    for idx in itertools.product(range(q), repeat=len(mu)):
        u = closed_forms.galerkin_trajectory(mu + sig * x[list(idx)], b, dm, nu, t)
        out += np.prod(w[list(idx)]) * closed_forms.deterministic_phi(u, n, length)
    return out


def test_gaussian_state_is_the_average_of_galerkin_trajectories():
    """From a Gaussian initial condition the full-grid RK4 solution converges
    at second order in h to the quadrature average of exp(i a . u(t)) over
    Galerkin trajectories (d = 3: the first mode triad, so B != 0; at d = 2
    B vanishes).  A wrong sign, swapped first two indices, a doubled factor
    or a missing advective term each miss by far more than the grid error."""
    d, length, nu, tend, steps = 3, 4.0, 0.05, 0.3, 60
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    assert np.count_nonzero(b) > 0
    mu, sig = np.array([0.9, -0.7, 0.6]), np.array([0.35, 0.25, 0.3])

    def error(n, bgrid, ref):
        prob = fullgrid.Problem(bgrid, dm, nu, n, length)
        f = fullgrid.gaussian_ic(mu, sig, n, length)
        for _ in range(steps):
            f = fullgrid.rk4_step(f, tend / steps, prob.apply)
        inner = np.abs(fd.grid(n, length)) <= length / 2  # away from the one-sided closures
        return float(np.abs(f - ref)[np.ix_(inner, inner, inner)].max())

    ref17 = _average_over_gaussian_states(mu, sig, b, dm, nu, tend, 17, length)
    ref33 = _average_over_gaussian_states(mu, sig, b, dm, nu, tend, 33, length)
    # the quadrature has converged where the grids are compared: 6 nodes per
    # mode agree with 8 there far below the grid error
    inner17 = np.abs(fd.grid(17, length)) <= length / 2
    q6 = _average_over_gaussian_states(mu, sig, b, dm, nu, tend, 17, length, q=6)
    assert np.abs(q6 - ref17)[np.ix_(inner17, inner17, inner17)].max() < 1e-6
    e17, e33 = error(17, b, ref17), error(33, b, ref33)
    assert e33 < 6e-3 and 3.4 < e17 / e33 < 4.6, (e17, e33)
    for wrong in (-b, b.transpose(1, 0, 2), 2.0 * b, 0.0 * b):
        assert error(33, wrong, ref33) > 20 * e33


def _run(d, n, length, nu, steps, dt, seed):
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    prob = fullgrid.Problem(b, dm, nu, n, length)
    mu, sig = inputs.ic_params(d, seed)
    f = fullgrid.gaussian_ic(mu, sig, n, length)
    for _ in range(steps):
        f = fullgrid.rk4_step(f, dt, prob.apply)
    return f


def test_origin_value_and_hermitian_symmetry():
    f = _run(3, 9, 4.0, 0.05, 20, 2e-3, 5)
    assert abs(f[4, 4, 4] - 1.0) < 1e-14
    assert np.abs(f[::-1, ::-1, ::-1] - np.conj(f)).max() < 1e-13


def test_modulus_bounded():
    f = _run(4, 12, 4.0, 0.05, 20, 1e-3, 0)
    assert np.abs(f).max() <= 1.0 + 1e-6


def test_tt_svd_exact_and_bounded():
    rng = np.random.default_rng(11)
    f = rng.standard_normal((5, 6, 4, 5)) + 1j * rng.standard_normal((5, 6, 4, 5))
    cores, _ = fullgrid.tt_svd(f, 0.0)
    assert fullgrid.rel_l2(fullgrid.tt_to_full(cores), f) < 1e-13
    for eps in (1e-1, 3e-1):
        g = fullgrid.truncate(f, eps)
        assert np.linalg.norm(g - f) <= eps * np.linalg.norm(f) * (1 + 1e-12)
    cores, _ = fullgrid.tt_svd(f, 0.0, cap=3)
    assert max(c.shape[2] for c in cores) <= 3


def test_truncation_rank_rule():
    s = np.array([1.0, 0.5, 0.1, 0.01, 0.001])
    assert fullgrid.truncation_rank(s, 0.0, None) == 5
    assert fullgrid.truncation_rank(s, 0.0011, None) == 4
    assert fullgrid.truncation_rank(s, np.sqrt(0.01**2 + 0.001**2) + 1e-15, None) == 3
    assert fullgrid.truncation_rank(s, 10.0, None) == 1
    assert fullgrid.truncation_rank(s, 0.0, 2) == 2


def test_truncated_step_without_truncation_is_rk4():
    d, n = 3, 6
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    prob = fullgrid.Problem(b, dm, 0.05, n, 4.0)
    mu, sig = inputs.ic_params(d, 2)
    f = fullgrid.gaussian_ic(mu, sig, n, 4.0)
    a = fullgrid.rk4_step(f, 1e-2, prob.apply)
    c = fullgrid.truncated_rk4_step(f, 1e-2, prob.apply, 0.0)
    assert fullgrid.rel_l2(c, a) < 1e-13


def test_tridiagonal_ic_tt_is_the_quadratic_form():
    # the nearest-neighbour product TT against the characteristic function
    # evaluated from the covariance matrix; rho = 0 is the rank-one IC
    d, n, length = 4, 9, 3.0
    mu, sig, rho = inputs.ic_params_tridiag(d, 5)
    full_tt = fullgrid.tt_to_full(closed_forms.tridiag_gaussian_tt(mu, sig, rho, n, length))
    ref = fullgrid.tridiag_gaussian_ic(mu, sig, rho, n, length)
    assert fullgrid.rel_l2(full_tt, ref) < 1e-14
    assert tt_ref.tt_ranks(closed_forms.tridiag_gaussian_tt(mu, sig, rho, n, length)) == [1, n, n, n, 1]
    zero = fullgrid.tridiag_gaussian_ic(mu, sig, np.zeros(d - 1), n, length)
    assert fullgrid.rel_l2(zero, fullgrid.gaussian_ic(mu, sig, n, length)) < 1e-15
    # a characteristic function: phi(0) = 1 (odd n), |phi| <= 1, phi(-a) = conj phi(a)
    c = (n - 1) // 2
    assert abs(ref[(c,) * d] - 1.0) < 1e-15
    assert np.abs(ref).max() <= 1.0 + 1e-15
    assert np.abs(ref[::-1, ::-1, ::-1, ::-1] - np.conj(ref)).max() < 1e-15
    # the correlations matter: a dropped sign or a shifted index changes it
    assert fullgrid.rel_l2(fullgrid.tridiag_gaussian_ic(mu, sig, -rho, n, length), ref) > 1e-3
    assert fullgrid.rel_l2(fullgrid.tridiag_gaussian_ic(mu, sig, rho[::-1], n, length), ref) > 1e-3


def test_viscous_only_tridiagonal_continuous_second_order_in_h():
    # with B = 0 the exact solution from a correlated Gaussian is the same
    # kind of Gaussian with mu, sigma scaled by exp(-nu kappa^2 t) and the
    # correlations unchanged; the grid RK4 solution converges to it at
    # second order in h
    d, length, nu, tend = 2, 6.0, 0.5, 0.5
    b = np.zeros((d, d, d))
    dm = galerkin.coefficient_D(d)
    mu, sig, rho = np.array([0.6, -0.4]), np.array([0.5, 0.7]), np.array([0.28])
    errs = []
    for n in (33, 65, 129):
        prob = fullgrid.Problem(b, dm, nu, n, length)
        f = fullgrid.tridiag_gaussian_ic(mu, sig, rho, n, length)
        for _ in range(25):
            f = fullgrid.rk4_step(f, tend / 25, prob.apply)
        mt, st, rt = closed_forms.viscous_continuous_tridiag(mu, sig, rho, nu, tend)
        errs.append(fullgrid.rel_l2(f, fullgrid.tridiag_gaussian_ic(mt, st, rt, n, length)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[0] < 1e-2 and all(1.7 < r < 2.4 for r in rates), (errs, rates)
