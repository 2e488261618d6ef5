"""Pins for oracle.galerkin (Fourier basis and Galerkin coefficients)."""
import math
import os

import numpy as np
import pytest

from oracle import galerkin

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "b_entries_d4.txt")


@pytest.mark.parametrize("d", [3, 4, 7, 20])
def test_basis_orthonormal(d):
    x, w = galerkin.quadrature(d)
    g, _ = galerkin.basis(d, x)
    gram = (g * w) @ g.T
    assert np.abs(gram - np.eye(d)).max() < 1e-14


def test_hand_derived_entries_d4():
    b = galerkin.coefficient_B(4)
    rows = [ln.split()[:4] for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    assert len(rows) >= 10
    for k, j, l, v in rows:
        got = b[int(k) - 1, int(j) - 1, int(l) - 1] * math.sqrt(math.pi)
        assert abs(got - float(v)) < 1e-13, (k, j, l, got, v)


@pytest.mark.parametrize("d", [4, 9, 20])
def test_symmetry_and_energy_conservation(d):
    b = galerkin.coefficient_B(d)
    assert np.abs(b - b.transpose(0, 2, 1)).max() < 1e-14
    # sum_kjl B_kjl u_k u_j u_l = -int u^2 u_x ... = 0 for every u, i.e. the
    # cyclic sum vanishes (energy conservation of Galerkin Burgers)
    cyc = b + b.transpose(1, 2, 0) + b.transpose(2, 0, 1)
    assert np.abs(cyc).max() < 1e-13


@pytest.mark.parametrize("d", [4, 8, 13])
def test_projection_of_pointwise_nonlinearity(d):
    """-1/2 sum B_kjl u_j u_l must equal int Gamma_k (-u u_x) dx for any u."""
    rng = np.random.default_rng(123 + d)
    b = galerkin.coefficient_B(d)
    kmax = int(galerkin.wavenumbers(d).max())
    q = 3 * kmax + 5
    x = 2 * math.pi * np.arange(q) / q
    w = 2 * math.pi / q
    g, gp = galerkin.basis(d, x)
    for _ in range(3):
        u = rng.standard_normal(d)
        ux, uxx = u @ g, u @ gp
        proj = (g * (-ux * uxx)).sum(axis=1) * w
        rhs = -0.5 * np.einsum("kjl,j,l->k", b, u, u)
        assert np.abs(proj - rhs).max() < 1e-12
    # a transposed index order is caught by the same check
    bt = b.transpose(1, 0, 2)
    u = rng.standard_normal(d)
    proj = (g * (-(u @ g) * (u @ gp))).sum(axis=1) * w
    assert np.abs(proj + 0.5 * np.einsum("kjl,j,l->k", bt, u, u)).max() > 1e-3


@pytest.mark.parametrize("d", [4, 11])
def test_viscous_coefficients(d):
    dm = galerkin.coefficient_D(d)
    kap = galerkin.wavenumbers(d)
    assert np.abs(dm - np.diag(-(kap.astype(float) ** 2))).max() < 1e-12


def test_wavenumbers_and_nonzero_pattern():
    assert list(galerkin.wavenumbers(6)) == [1, 1, 2, 2, 3, 3]
    b = galerkin.coefficient_B(6)
    kap = galerkin.wavenumbers(6)
    # triad rule: B_kjl = 0 unless kappa_k = kappa_j + kappa_l or |kappa_j - kappa_l|
    for k in range(6):
        for j in range(6):
            for l in range(6):
                if b[k, j, l] != 0.0:
                    assert kap[k] in (kap[j] + kap[l], abs(kap[j] - kap[l]))
