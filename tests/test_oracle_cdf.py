"""Pins of the CDF-equation oracle (Sec. 5, eq. (eqn:cdf-burgers)) against
closed forms derived independently of it."""
import numpy as np
import pytest
from scipy.linalg import expm
from scipy.stats import multivariate_normal

from oracle import cdf, fullgrid

BOX, SIGMA = 1.3, 0.25


def _grid_points(N, n):
    u = cdf.grid(n, BOX)
    mesh = np.meshgrid(*([u] * N), indexing="ij")
    return np.stack([m.ravel() for m in mesh], axis=1)


def test_periodic_differences():
    d1, d2 = cdf.periodic_differences(5)
    x = 2 * np.pi * np.arange(5) / 5
    # exact on the lowest mode up to the second-order factors
    dx = 2 * np.pi / 5
    assert np.allclose(d1 @ np.sin(x), np.sin(dx) / dx * np.cos(x))
    assert np.allclose(d2 @ np.sin(x), (2 * np.cos(dx) - 2) / dx**2 * np.sin(x))
    assert np.allclose(d1, -d1.T) and np.allclose(d2, d2.T)


def test_cumulative_integral_is_the_trapezoid_rule():
    n = 11
    u = cdf.grid(n, BOX)
    j = cdf.cumulative_integral(n, BOX)
    # exact for linear functions, from the lower end
    assert np.allclose(j @ (2 * u + 1), (u**2 + u) - (u[0] ** 2 + u[0]))
    assert np.allclose(j[0], 0.0)


@pytest.mark.parametrize("advection,gamma,alpha", [(1.0, 0.3, 0.7), (1.0, 0.0, 0.0), (0.0, 0.5, 0.0),
                                                   (0.0, 0.0, 1.0)])
def test_operator_converges_to_the_exact_rate(advection, gamma, alpha):
    """dF/dt at t = 0 on the product of Gaussian CDFs: the discrete operator
    against the rate derived from the Liouville equation, second order in h."""
    N = 3
    errs = []
    for n in (33, 65):
        prob = cdf.CdfProblem(N, n, BOX, gamma, alpha, advection)
        f0 = cdf.gaussian_cdf_ic(N, n, BOX, SIGMA)
        rate = prob.apply(f0).ravel()
        assert np.abs(rate.imag).max() == 0.0
        exact = cdf.exact_rate_gaussian(_grid_points(N, n), N, SIGMA, gamma, alpha, advection)
        errs.append(np.abs(rate.real - exact).max() / np.abs(exact).max())
    print("relative max errors", errs)
    assert errs[1] < 0.3 * errs[0]
    assert errs[1] < 2e-2


def test_reaction_counted_once():
    """The printed equation's extra reaction sum would double the reaction
    rate: the oracle's rate matches the Liouville rate, not twice it."""
    N, n = 2, 65
    prob = cdf.CdfProblem(N, n, BOX, 0.0, 1.0, 0.0)
    f0 = cdf.gaussian_cdf_ic(N, n, BOX, SIGMA)
    rate = prob.apply(f0).real.ravel()
    exact = cdf.exact_rate_gaussian(_grid_points(N, n), N, SIGMA, 0.0, 1.0, 0.0)
    assert np.abs(rate - exact).max() < 0.02 * np.abs(exact).max()
    assert np.abs(rate - 2 * exact).max() > 0.5 * np.abs(exact).max()


def test_reaction_only_evolution_matches_characteristics():
    N, alpha, t, dt = 2, 1.0, 0.1, 1e-3
    errs = []
    for n in (41, 81):
        prob = cdf.CdfProblem(N, n, BOX, 0.0, alpha, 0.0)
        f = cdf.gaussian_cdf_ic(N, n, BOX, SIGMA)
        for _ in range(int(round(t / dt))):
            f = fullgrid.rk4_step(f, dt, prob.apply)
        exact = cdf.reaction_only_solution(_grid_points(N, n), SIGMA, alpha, t)
        errs.append(np.abs(f.real.ravel() - exact).max())
    print("max errors", errs)
    assert errs[1] < 0.35 * errs[0]
    assert errs[1] < 5e-3


def test_linear_viscous_evolution_is_the_propagated_gaussian():
    """advection 0, alpha 0: du/dt = gamma D2 u keeps u Gaussian with
    covariance M (sigma^2 I) M^T, M = exp(gamma D2 t)."""
    N, gamma, t, dt = 2, 1.0, 0.3, 2e-3
    _, d2 = cdf.periodic_differences(N)
    m = expm(gamma * d2 * t)
    cov = SIGMA**2 * m @ m.T
    errs = []
    for n in (49, 97):
        prob = cdf.CdfProblem(N, n, BOX, gamma, 0.0, 0.0)
        f = cdf.gaussian_cdf_ic(N, n, BOX, SIGMA)
        for _ in range(int(round(t / dt))):
            f = fullgrid.rk4_step(f, dt, prob.apply)
        pts = _grid_points(N, n)
        sel = np.arange(0, pts.shape[0], 37)
        exact = multivariate_normal.cdf(pts[sel], mean=np.zeros(N), cov=cov, abseps=1e-9, releps=1e-9)
        errs.append(np.abs(f.real.ravel()[sel] - exact).max())
    print("max errors", errs)
    assert errs[1] < 0.35 * errs[0]
    assert errs[1] < 2e-3


def test_separable_pointwise_matches_the_full_grid():
    N, n = 3, 9
    rng = np.random.default_rng(2)
    prob = cdf.CdfProblem(N, n, BOX, 0.2, 0.6, 1.0, diffusion=0.01)
    factors = [rng.standard_normal(n) + 1j * rng.standard_normal(n) for _ in range(N)]
    full = np.einsum("i,j,k->ijk", *factors)
    ref = prob.apply(full)
    idx = np.stack(np.meshgrid(*([np.arange(n)] * N), indexing="ij"), axis=-1).reshape(-1, N)
    pt = cdf.apply_separable_at(idx, factors, prob)
    assert np.abs(pt - ref.ravel()).max() < 1e-12 * np.abs(ref).max()
