"""Pins for oracle.fd (grid and 1-D finite-difference operators)."""
import numpy as np
import pytest

from oracle import fd


@pytest.mark.parametrize("n,length", [(8, 4.0), (32, 4.0), (33, 6.0), (128, 8.0)])
def test_exact_on_polynomials(n, length):
    a = fd.grid(n, length)
    g = fd.first_derivative(n, length)
    l2 = fd.second_derivative(n, length)
    quad = 0.3 - 1.7 * a + 0.45 * a**2
    assert np.abs(g @ quad - (-1.7 + 0.9 * a)).max() < 1e-10 * n
    cub = 0.3 - 1.7 * a + 0.45 * a**2 - 0.2 * a**3
    assert np.abs(l2 @ cub - (0.9 - 1.2 * a)).max() < 1e-9 * n * n


def test_grid_symmetric_and_endpoints():
    a = fd.grid(33, 6.0)
    assert a[0] == -6.0 and a[-1] == 6.0 and abs(a[16]) < 1e-15
    assert np.abs(a + a[::-1]).max() < 1e-14
    assert abs(fd.spacing(33, 6.0) - 12.0 / 32) < 1e-15


def test_reflection_symmetry():
    n, length = 17, 4.0
    r = np.eye(n)[::-1]
    g = fd.first_derivative(n, length)
    l2 = fd.second_derivative(n, length)
    x = fd.position(n, length)
    assert np.abs(r @ g @ r + g).max() < 1e-12
    assert np.abs(r @ l2 @ r - l2).max() < 1e-10
    assert np.abs(r @ x @ r + x).max() < 1e-14


def test_second_order_convergence():
    errs_g, errs_l = [], []
    for n in (33, 65, 129):
        a = fd.grid(n, 4.0)
        f = np.sin(1.3 * a)
        errs_g.append(np.abs(fd.first_derivative(n, 4.0) @ f - 1.3 * np.cos(1.3 * a)).max())
        errs_l.append(np.abs(fd.second_derivative(n, 4.0) @ f + 1.69 * f).max())
    for e in (errs_g, errs_l):
        rates = [np.log2(e[i] / e[i + 1]) for i in range(2)]
        assert all(1.8 < r < 2.3 for r in rates), rates
