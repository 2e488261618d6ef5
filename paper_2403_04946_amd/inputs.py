"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.

This module holds no arithmetic of the method: it only draws random numbers
and returns plain arrays (initial-condition parameters, random TT cores,
grid index samples).  Both the device path and the CPU oracle receive the
same arrays from here.
"""
import numpy as np


def ic_params(d, seed, mean_var=0.25, sigma_lo=0.3, sigma_hi=1.0):
    """Gaussian initial-condition parameters for d modes.

    mu_k ~ N(0, variance mean_var), sigma_k ~ U(sigma_lo, sigma_hi), drawn
    with numpy's default_rng(seed) in the order mu then sigma.
    """
    rng = np.random.default_rng(seed)
    mu = rng.normal(0.0, np.sqrt(mean_var), size=d)
    sigma = rng.uniform(sigma_lo, sigma_hi, size=d)
    return mu, sigma


def ic_params_tridiag(d, seed, mean_var=0.25, sigma_lo=0.3, sigma_hi=1.0, rho_max=0.3):
    """Parameters of the Gaussian initial condition with tridiagonal
    covariance: mu, sigma as ic_params, then the d-1 neighbour correlations
    rho_k ~ U(-rho_max, rho_max), from one default_rng(seed) in that order."""
    rng = np.random.default_rng(seed)
    mu = rng.normal(0.0, np.sqrt(mean_var), size=d)
    sigma = rng.uniform(sigma_lo, sigma_hi, size=d)
    rho = rng.uniform(-rho_max, rho_max, size=max(d - 1, 0))
    return mu, sigma, rho


def random_tt(d, n, rank, seed, scale=None):
    """Random complex TT cores with i.i.d. standard complex Gaussian entries.

    ``rank`` is an int (all interior ranks) or a list of d+1 ranks.  Cores
    are numpy arrays of shape (r_{k-1}, n, r_k).  ``scale`` multiplies each
    core (default 1/sqrt(2 n r_{k-1}): each core then preserves the expected
    squared norm of what it is contracted with, so the full tensor has
    expected squared Frobenius norm one).
    """
    rng = np.random.default_rng(seed)
    if np.isscalar(rank):
        ranks = [1] + [int(rank)] * (d - 1) + [1]
    else:
        ranks = list(rank)
    cores = []
    for k in range(d):
        r0, r1 = ranks[k], ranks[k + 1]
        re = rng.standard_normal((r0, n, r1))
        im = rng.standard_normal((r0, n, r1))
        s = scale if scale is not None else 1.0 / np.sqrt(2.0 * n * r0)
        cores.append((re + 1j * im) * s)
    return cores


def random_points(d, n, npts, seed):
    """Uniform random grid index tuples, int32 array (npts, d)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, n, size=(npts, d), dtype=np.int64).astype(np.int32)


def batch_instances(count, seed, d_range=(8, 64), n_choices=(32, 64, 128), nu_range=(1e-3, 1e-1),
                    cap_range=(16, 96)):
    """Seeded parameters of uneven independent instances (the batched
    workload): d uniform on d_range (inclusive), n from n_choices, nu
    log-uniform on nu_range, rank cap uniform on cap_range (inclusive), and
    the Gaussian initial-condition parameters of each instance (ic_params
    with the instance's own seed).  Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        d = int(rng.integers(d_range[0], d_range[1] + 1))
        n = int(rng.choice(n_choices))
        nu = float(np.exp(rng.uniform(np.log(nu_range[0]), np.log(nu_range[1]))))
        cap = int(rng.integers(cap_range[0], cap_range[1] + 1))
        mu, sigma = ic_params(d, 1000 * seed + i)
        out.append({"d": d, "n": n, "nu": nu, "cap": cap, "mu": mu, "sigma": sigma, "seed": 1000 * seed + i})
    return out
