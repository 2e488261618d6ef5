"""Fourier basis and Galerkin coefficients of periodic Burgers (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper: Sec. 3, eq. (hyper1) gives the linear PDE obtained by projecting an
FDE onto a finite basis, with coefficients defined by inner products of the
basis functions (eq. (coefficients)).  Sec. 5 states the Burgers equation on
the circle [0, 2*pi] (eq. (eqn:burgers-rxn), here with no reaction term) and
its Hopf FDE (eq. (eqn:BHfde)), whose advective term is (i/2) d/dx of the
second functional derivative and whose viscous term is gamma d^2/dx^2 of the
first.  Projecting onto d orthonormal real Fourier modes gives

    dphi/dt = sum_k a_k [ (i/2) sum_{j,l} B_kjl d2phi/da_j da_l
                          + nu sum_j D_kj dphi/da_j ],

    B_kjl = int_0^{2pi} Gamma_k d/dx(Gamma_j Gamma_l) dx,
    D_kj  = int_0^{2pi} Gamma_k Gamma_j'' dx.

Reading (trigonometric basis, listed by the paper among admissible bases in
Sec. 3): mode k = 1..d has wavenumber kappa_k = ceil(k/2); odd k is
cos(kappa x)/sqrt(pi), even k is sin(kappa x)/sqrt(pi).  The constant mode
is excluded (Burgers conserves the mean).

Pins (tests/test_oracle_galerkin.py): orthonormality; B symmetric in (j, l);
cyclic identity B_kjl + B_jlk + B_lkj = 0 (energy conservation);
hand-derived entries (tests/golden/b_entries_d4.txt); the projection of the
pointwise Burgers nonlinearity -u u_x equals -1/2 sum B_kjl u_j u_l for
random u; D = -diag(kappa^2).
"""
import math

import numpy as np


def wavenumbers(d):
    """kappa_k = ceil(k/2) for k = 1..d (returned 0-based, length d)."""
    return np.array([(k + 2) // 2 for k in range(d)], dtype=np.int64)


def is_cosine(d):
    """True for modes 1, 3, 5, ... (0-based even index)."""
    return np.array([k % 2 == 0 for k in range(d)])


def basis(d, x):
    """Gamma_k(x) and Gamma_k'(x) for k = 1..d; arrays of shape (d, len(x))."""
    x = np.asarray(x, dtype=np.float64)
    kap = wavenumbers(d)
    cos_mask = is_cosine(d)
    g = np.empty((d, x.size))
    gp = np.empty((d, x.size))
    s = 1.0 / math.sqrt(math.pi)
    for k in range(d):
        if cos_mask[k]:
            g[k] = s * np.cos(kap[k] * x)
            gp[k] = -s * kap[k] * np.sin(kap[k] * x)
        else:
            g[k] = s * np.sin(kap[k] * x)
            gp[k] = s * kap[k] * np.cos(kap[k] * x)
    return g, gp


def basis_second_derivative(d, x):
    """Gamma_k''(x) = -kappa_k^2 Gamma_k(x)."""
    g, _ = basis(d, x)
    kap = wavenumbers(d).astype(np.float64)
    return -(kap[:, None] ** 2) * g


def quadrature(d):
    """Uniform periodic rule on [0, 2pi] exact for trig. degree < Q.

    Integrands below are products of three modes, degree <= 3*kappa_max, so
    Q = 4*kappa_max + 4 points integrate them exactly.
    """
    kmax = int(wavenumbers(d).max())
    q = 4 * kmax + 4
    x = 2.0 * math.pi * np.arange(q) / q
    w = np.full(q, 2.0 * math.pi / q)
    return x, w


def coefficient_B(d):
    """B[k, j, l] = int Gamma_k (Gamma_j Gamma_l)' dx (eq. (coefficients))."""
    x, w = quadrature(d)
    g, gp = basis(d, x)
    # (Gamma_j Gamma_l)' = Gamma_j' Gamma_l + Gamma_j Gamma_l'
    dprod = gp[:, None, :] * g[None, :, :] + g[:, None, :] * gp[None, :, :]
    b = np.einsum("kq,jlq,q->kjl", g, dprod, w)
    b[np.abs(b) < 1e-13] = 0.0
    return b


def coefficient_D(d):
    """D[k, j] = int Gamma_k Gamma_j'' dx (eq. (coefficients), viscous part)."""
    x, w = quadrature(d)
    g, _ = basis(d, x)
    gpp = basis_second_derivative(d, x)
    dm = np.einsum("kq,jq,q->kj", g, gpp, w)
    dm[np.abs(dm) < 1e-13] = 0.0
    return dm


def galerkin_rhs(u, b, dm, nu):
    """Galerkin ODE of Burgers: du_k/dt = -1/2 sum B_kjl u_j u_l + nu sum D_kj u_j.

    Used by the deterministic-initial-state pin: for u(0) = mu the
    characteristic function is exactly exp(i a . u(t)).
    """
    return -0.5 * np.einsum("kjl,j,l->k", b, u, u) + nu * dm @ u
