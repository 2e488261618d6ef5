"""Tensor-product grid and 1-D finite-difference operators (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper: Sec. 4 expands the solution on a tensor-product basis (eq. (tt)) and
obtains the semi-discrete system (eq. (eqn:ode)); Sec. 5 discretises each
phase variable on an evenly spaced grid with second-order centred finite
differences.  Readings for the characteristic-function PDE (the paper gives
boundary closures only for its CDF equation):

* grid: a_i = -L + 2L i/(n-1), i = 0..n-1 (endpoints included, symmetric),
  h = 2L/(n-1);
* first derivative G: centred (f[i+1]-f[i-1])/(2h); boundary rows are the
  second-order one-sided formulas (-3f0+4f1-f2)/(2h) and its mirror;
* second derivative L2: (f[i+1]-2f[i]+f[i-1])/h^2; boundary rows
  (2f0-5f1+4f2-f3)/h^2 and its mirror;
* X = diag(a).

Pins (tests/test_oracle_fd.py): exactness on quadratics (G) and cubics
(L2 boundary rows) at every row; second-order convergence on a smooth
function; reflection symmetry of the grid and operators.
"""
import numpy as np


def grid(n, length):
    """Symmetric grid on [-L, L] with n points including both endpoints."""
    i = np.arange(n, dtype=np.float64)
    return -length + 2.0 * length * i / (n - 1)


def spacing(n, length):
    return 2.0 * length / (n - 1)


def first_derivative(n, length):
    """Dense n x n matrix of G (n >= 3)."""
    h = spacing(n, length)
    g = np.zeros((n, n))
    for i in range(1, n - 1):
        g[i, i - 1] = -1.0 / (2 * h)
        g[i, i + 1] = 1.0 / (2 * h)
    g[0, 0:3] = np.array([-3.0, 4.0, -1.0]) / (2 * h)
    g[n - 1, n - 3:n] = np.array([1.0, -4.0, 3.0]) / (2 * h)
    return g


def second_derivative(n, length):
    """Dense n x n matrix of L2 (n >= 4)."""
    h = spacing(n, length)
    m = np.zeros((n, n))
    for i in range(1, n - 1):
        m[i, i - 1] = 1.0 / h**2
        m[i, i] = -2.0 / h**2
        m[i, i + 1] = 1.0 / h**2
    m[0, 0:4] = np.array([2.0, -5.0, 4.0, -1.0]) / h**2
    m[n - 1, n - 4:n] = np.array([-1.0, 4.0, -5.0, 2.0]) / h**2
    return m


def position(n, length):
    """X = diag(a)."""
    return np.diag(grid(n, length))
