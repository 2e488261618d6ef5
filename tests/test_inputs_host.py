"""Host checks of the seeded input generators (no GPU): determinism, the
stated distributions and ranges, and that the correlated initial condition
describes a Gaussian (positive definite covariance)."""
import numpy as np
import pytest

from oracle import fullgrid
from paper_2403_04946_amd import inputs


def test_ic_params_are_seeded_and_follow_their_distributions():
    mu, sigma = inputs.ic_params(20000, 11)
    mu2, sigma2 = inputs.ic_params(20000, 11)
    assert np.array_equal(mu, mu2) and np.array_equal(sigma, sigma2)
    assert not np.array_equal(mu, inputs.ic_params(20000, 12)[0])
    # mu ~ N(0, variance 0.25): sample mean and variance within 5 standard errors
    assert abs(mu.mean()) < 5 * 0.5 / np.sqrt(mu.size)
    assert abs(mu.var() - 0.25) < 5 * 0.25 * np.sqrt(2.0 / mu.size)
    # sigma ~ U(0.3, 1)
    assert sigma.min() >= 0.3 and sigma.max() < 1.0
    assert abs(sigma.mean() - 0.65) < 5 * (0.7 / np.sqrt(12.0)) / np.sqrt(sigma.size)


def test_tridiagonal_parameters_extend_the_product_ones():
    """mu and sigma are drawn first from the same generator, so they equal
    the product initial condition's for the same seed; the d - 1
    correlations follow, uniform on (-0.3, 0.3)."""
    d = 5000
    mu, sigma, rho = inputs.ic_params_tridiag(d, 7)
    mu0, sigma0 = inputs.ic_params(d, 7)
    assert np.array_equal(mu, mu0) and np.array_equal(sigma, sigma0)
    assert rho.shape == (d - 1,)
    assert rho.min() >= -0.3 and rho.max() < 0.3
    assert abs(rho.mean()) < 5 * (0.6 / np.sqrt(12.0)) / np.sqrt(rho.size)
    assert inputs.ic_params_tridiag(1, 7)[2].shape == (0,)


@pytest.mark.parametrize("d", [2, 20, 50, 100])
def test_tridiagonal_covariance_is_positive_definite(d):
    """Sigma = S R S with R the tridiagonal correlation matrix: its smallest
    eigenvalue stays positive for every draw (|rho| < 0.3 keeps R diagonally
    dominant), so the initial condition is the characteristic function of a
    Gaussian."""
    for seed in range(20):
        _, sigma, rho = inputs.ic_params_tridiag(d, seed)
        corr = np.eye(d) + np.diag(rho, 1) + np.diag(rho, -1)
        cov = sigma[:, None] * corr * sigma[None, :]
        assert np.linalg.eigvalsh(corr).min() >= 1.0 - 2 * 0.3 - 1e-12
        assert np.linalg.eigvalsh(cov).min() > 0.0


def test_random_tt_shapes_seed_and_norm():
    cores = inputs.random_tt(4, 5, [1, 2, 6, 3, 1], 3)
    assert [c.shape for c in cores] == [(1, 5, 2), (2, 5, 6), (6, 5, 3), (3, 5, 1)]
    assert all(c.dtype == np.complex128 for c in cores)
    again = inputs.random_tt(4, 5, [1, 2, 6, 3, 1], 3)
    assert all(np.array_equal(a, b) for a, b in zip(cores, again))
    uniform = inputs.random_tt(3, 4, 3, 0)
    assert [c.shape for c in uniform] == [(1, 4, 3), (3, 4, 3), (3, 4, 1)]
    # the default scale gives expected squared Frobenius norm one
    norms = [np.sum(np.abs(fullgrid.tt_to_full(inputs.random_tt(3, 4, 3, s))) ** 2) for s in range(400)]
    assert abs(np.mean(norms) - 1.0) < 0.1


def test_random_points_are_grid_indices():
    pts = inputs.random_points(7, 33, 5000, 2)
    assert pts.shape == (5000, 7) and pts.dtype == np.int32
    assert pts.min() == 0 and pts.max() == 32
    assert np.array_equal(pts, inputs.random_points(7, 33, 5000, 2))


def test_batch_instances_ranges_and_seeds():
    insts = inputs.batch_instances(300, 4)
    assert len(insts) == 300
    again = inputs.batch_instances(300, 4)
    assert all(a["d"] == b["d"] and a["n"] == b["n"] and a["nu"] == b["nu"] and a["cap"] == b["cap"]
               and np.array_equal(a["mu"], b["mu"]) for a, b in zip(insts, again))
    for inst in insts:
        assert 8 <= inst["d"] <= 64 and inst["n"] in (32, 64, 128)
        assert 1e-3 <= inst["nu"] <= 1e-1 and 16 <= inst["cap"] <= 96
        mu, sigma = inputs.ic_params(inst["d"], inst["seed"])
        assert np.array_equal(mu, inst["mu"]) and np.array_equal(sigma, inst["sigma"])
    ds = np.array([i["d"] for i in insts])
    assert ds.min() == 8 and ds.max() == 64  # both ends of the inclusive range are drawn
    assert len({i["n"] for i in insts}) == 3
    assert len({i["seed"] for i in insts}) == 300
