"""Exact solutions used as pins (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

1. Viscous-only continuous solution.  With B = 0 the PDE of Sec. 3
   eq. (hyper1) (Burgers coefficients, Sec. 5) is the transport equation
   dphi/dt = nu sum_k D_kk a_k dphi/da_k with D_kk = -kappa_k^2, whose
   characteristics give phi(a,t) = phi0(exp(nu D t) a).  For the Gaussian
   initial condition phi0 = prod exp(i mu_k a_k - sigma_k^2 a_k^2/2) this is
   the Gaussian with mu_k, sigma_k scaled by exp(-nu kappa_k^2 t).

2. Viscous-only semi-discrete solution.  With B = 0 the grid operator is a
   sum of commuting one-axis operators nu D_kk X G, so the exact solution of
   the semi-discrete system is the per-axis matrix exponential applied to
   each TT core (ranks preserved).

3. Correlated Gaussian initial condition.  The characteristic function of
   amplitudes u ~ N(mu, Sigma) with tridiagonal Sigma is a product of
   one-axis and nearest-neighbour factors, an exact TT with bond ranks n;
   under the viscous-only flow it stays such a Gaussian with mu and sigma
   scaled per axis and the correlations unchanged (Sigma(t) = S Sigma S,
   S = exp(nu D t) diagonal).

4. Deterministic initial state.  The Hopf characteristic functional of a
   deterministic solution is exp(i <u, theta>) (Sec. 1 / Sec. 5 definition
   of Phi).  Projected on the Fourier modes: if u(0) = mu exactly, then
   phi(a,t) = exp(i a . u(t)) where u(t) solves the Galerkin ODE
   du_k/dt = -1/2 sum B_kjl u_j u_l + nu sum D_kj u_j.  This pins the sign,
   the factor (i/2) and the index order of the advective term.
"""
import numpy as np
import scipy.integrate
import scipy.linalg

from . import fd
from .galerkin import galerkin_rhs, wavenumbers


def viscous_continuous_factors(mu, sigma, nu, t, n, length):
    """One-dimensional factors of the exact viscous-only solution."""
    a = fd.grid(n, length)
    kap = wavenumbers(len(mu)).astype(np.float64)
    out = []
    for k in range(len(mu)):
        s = np.exp(-nu * kap[k] ** 2 * t)
        out.append(np.exp(1j * mu[k] * s * a - 0.5 * (sigma[k] * s) ** 2 * a**2))
    return out


def tridiag_gaussian_tt(mu, sigma, rho, n, length):
    """Exact TT of the Gaussian characteristic function with tridiagonal
    covariance (Sigma_kk = sigma_k^2, Sigma_k,k+1 = rho_k sigma_k sigma_k+1),
    phi0(a) = exp(i mu.a - a^T Sigma a / 2): the product of the one-axis
    factors exp(i mu_k a_k - sigma_k^2 a_k^2 / 2) and the neighbour factors
    exp(-rho_k sigma_k sigma_k+1 a_k a_k+1).  Core k carries the previous
    coordinate on its left bond and repeats its own on the right one, so
    interior bond ranks are n."""
    a = fd.grid(n, length)
    d = len(mu)
    cores = []
    for k in range(d):
        own = np.exp(1j * mu[k] * a - 0.5 * sigma[k] ** 2 * a**2)
        left = np.ones((1, n)) if k == 0 else np.exp(-rho[k - 1] * sigma[k - 1] * sigma[k] * np.outer(a, a))
        core = left[:, :, None] * own[None, :, None]  # (r0, n, 1)
        if k < d - 1:
            core = core * np.eye(n)[None, :, :]  # repeat the coordinate: (r0, n, n)
        cores.append(core.astype(np.complex128))
    return cores


def viscous_continuous_tridiag(mu, sigma, rho, nu, t):
    """Parameters of the exact viscous-only solution from the tridiagonal
    Gaussian: phi(a, t) = phi0(s a) with s_k = exp(-nu kappa_k^2 t), the same
    kind of Gaussian with mu_k s_k, sigma_k s_k and unchanged rho."""
    kap = wavenumbers(len(mu)).astype(np.float64)
    s = np.exp(-nu * kap**2 * t)
    return np.asarray(mu) * s, np.asarray(sigma) * s, np.asarray(rho)


def viscous_semidiscrete_propagator(dkk, nu, t, n, length):
    """expm(t * nu * D_kk * X G) for one axis."""
    x = fd.position(n, length)
    g = fd.first_derivative(n, length)
    return scipy.linalg.expm(t * nu * dkk * (x @ g))


def viscous_semidiscrete_cores(cores, dm_diag, nu, t, n, length):
    """Apply the per-axis propagators to TT cores (r_{k-1}, n, r_k)."""
    out = []
    for k, core in enumerate(cores):
        p = viscous_semidiscrete_propagator(dm_diag[k], nu, t, n, length)
        out.append(np.einsum("ij,ajb->aib", p, core))
    return out


def galerkin_trajectory(mu, b, dm, nu, t):
    """u(t) of the Galerkin ODE from u(0) = mu, integrated to 1e-13."""
    sol = scipy.integrate.solve_ivp(
        lambda _t, u: galerkin_rhs(u, b, dm, nu),
        (0.0, t),
        np.asarray(mu, dtype=np.float64),
        method="DOP853",
        rtol=1e-13,
        atol=1e-15,
    )
    return sol.y[:, -1]


def deterministic_phi(u, n, length):
    """exp(i a . u) on the full grid."""
    a = fd.grid(n, length)
    d = len(u)
    out = np.ones((1,) * d, dtype=np.complex128)
    for k in range(d):
        shape = [1] * d
        shape[k] = n
        out = out * np.exp(1j * u[k] * a).reshape(shape)
    return out
