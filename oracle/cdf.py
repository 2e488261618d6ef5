"""The CDF equation of the stochastic Burgers equation with reaction (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper: Sec. 5.  The Burgers equation with reaction R(u) = alpha sin(pi u)
(eq. (eqn:burgers-rxn)) at N evenly spaced points x_j = 2 pi (j-1)/N of the
circle, with D1 and D2 the periodic second-order first- and second-
difference matrices, moves u = (u_1..u_N) with the velocity

    v_i(u) = sum_j ( -u_i D1_ij u_j + gamma D2_ij u_j ) + R(u_i).

Its joint PDF obeys the Liouville equation (eq. (eqn:pdf-burgers)) and its
joint CDF F the CDF equation (eq. (eqn:cdf-burgers)), taken here in the
form of its first two sums:

    dF/dt = sum_{i,j} ( u_i D1_ij u_j - gamma D2_ij u_j - delta_ij R(u_j) ) dF/du_i
          - sum_{i != j} ( D1_ij u_i - gamma D2_ij ) int_{-inf}^{u_j} dF/du_i du_j.

Reading: the printed equation adds a third sum -alpha sum_j sin(pi u_j)
dF/du_j, which repeats the reaction already in the first sum; integrating
the Liouville equation gives the reaction once, and so does this oracle
(the pin against the closed-form time derivative below would fail with it
twice).

Discretisation (Sec. 5): phase space [-box, box]^N, n evenly spaced points
per axis (ends included); centred second-order first differences in u with
outflow boundaries (dF/du = 0: the derivative is zero on the boundary
rows); the integrals by the trapezoid rule from the lower end of the box;
optional numerical diffusion kappa sum_k d2F/du_k^2 (interior rows of the
centred second difference, zero boundary rows).  ``advection`` scales the
D1 terms (1 is the equation; 0 leaves the linear and reaction parts, which
have closed-form solutions).

Pins (tests/test_oracle_cdf.py): on the product of Gaussian CDFs the
operator converges at second order in h to the exact time derivative of
the CDF, derived independently from the Liouville equation (Gaussian
integrals in closed form); reaction-only evolution against its solution by
characteristics; linear (viscous) evolution against the Gaussian CDF with
the propagated covariance; the pointwise evaluation of the operator on a
separable F against the full grid.
"""
import numpy as np

from . import fullgrid


def grid(n, box):
    return -box + 2.0 * box * np.arange(n, dtype=np.float64) / (n - 1)


def periodic_differences(N):
    """D1, D2 on N points of the circle (spacing 2 pi / N)."""
    dx = 2.0 * np.pi / N
    shift_up = np.roll(np.eye(N), 1, axis=1)    # (S f)_i = f_{i+1}
    shift_down = np.roll(np.eye(N), -1, axis=1)  # (S f)_i = f_{i-1}
    d1 = (shift_up - shift_down) / (2.0 * dx)
    d2 = (shift_up + shift_down - 2.0 * np.eye(N)) / dx**2
    d1[np.abs(d1) < 1e-12] = 0.0
    d2[np.abs(d2) < 1e-12] = 0.0
    return d1, d2


def derivative(n, box):
    """Centred first difference with zero (outflow) boundary rows."""
    h = 2.0 * box / (n - 1)
    g = np.zeros((n, n))
    for i in range(1, n - 1):
        g[i, i - 1] = -1.0 / (2 * h)
        g[i, i + 1] = 1.0 / (2 * h)
    return g


def second_difference(n, box):
    h = 2.0 * box / (n - 1)
    m = np.zeros((n, n))
    for i in range(1, n - 1):
        m[i, i - 1], m[i, i], m[i, i + 1] = 1 / h**2, -2 / h**2, 1 / h**2
    return m


def cumulative_integral(n, box):
    """Trapezoid rule from the lower end: (J g)_m = sum over the m first
    intervals of h (g_l + g_{l+1}) / 2."""
    h = 2.0 * box / (n - 1)
    j = np.zeros((n, n))
    for m in range(1, n):
        for l in range(m):  # interval [l, l+1]
            j[m, l] += 0.5 * h
            j[m, l + 1] += 0.5 * h
    return j


class CdfProblem:
    """Discrete CDF operator on the full n^N grid."""

    def __init__(self, N, n, box, gamma, alpha, advection=1.0, diffusion=0.0):
        self.N, self.n, self.box = int(N), int(n), float(box)
        self.gamma, self.alpha = float(gamma), float(alpha)
        self.advection, self.diffusion = float(advection), float(diffusion)
        self.u = grid(n, box)
        self.g = derivative(n, box)
        self.j = cumulative_integral(n, box)
        self.l2 = second_difference(n, box)
        self.d1, self.d2 = periodic_differences(N)

    def coord(self, k):
        shape = [1] * self.N
        shape[k] = self.n
        return self.u.reshape(shape)

    def apply(self, f):
        N = self.N
        f = np.asarray(f, dtype=np.complex128)
        d1 = self.advection * self.d1
        out = np.zeros_like(f)
        for i in range(N):
            gi = fullgrid.apply_along(self.g, f, i)  # dF/du_i
            ui = self.coord(i)
            # first sum: velocity-like coefficient times dF/du_i
            coef = -self.alpha * np.sin(np.pi * ui)
            for j in range(N):
                uj = self.coord(j)
                coef = coef + ui * d1[i, j] * uj - self.gamma * self.d2[i, j] * uj
            out += coef * gi
            # second sum: the cumulative integrals along u_j of dF/du_i
            for j in range(N):
                if j == i:
                    continue
                c = d1[i, j] * ui - self.gamma * self.d2[i, j]
                if np.all(c == 0):
                    continue
                out -= c * fullgrid.apply_along(self.j, gi, j)
        if self.diffusion != 0.0:
            for i in range(N):
                out += self.diffusion * fullgrid.apply_along(self.l2, f, i)
        return out


def gaussian_cdf_factor(n, box, sigma):
    """0.5 (1 + erf(u / (sigma sqrt 2))) on the grid."""
    from scipy.special import erf

    u = grid(n, box)
    return 0.5 * (1.0 + erf(u / (sigma * np.sqrt(2.0))))


def gaussian_cdf_ic(N, n, box, sigma):
    """F(u, 0) = prod_k g(u_k) on the full grid."""
    g = gaussian_cdf_factor(n, box, sigma)
    f = np.ones([1] * N)
    for k in range(N):
        shape = [1] * N
        shape[k] = n
        f = f * g.reshape(shape)
    return f.astype(np.complex128)


def exact_rate_gaussian(points, N, sigma, gamma, alpha, advection=1.0):
    """dF/dt at t = 0 for F = prod_k Phi(u_k / sigma), from the Liouville
    equation: dF/dt = -sum_i int_{v <= u} d/dv_i (v_i p) dv.  The v_i
    integral leaves v_i p at v_i = u_i; v_i is affine in every other v_j,
    and int_{-inf}^{u} v phi(v) dv = -sigma^2 phi(u) for the N(0, sigma^2)
    density phi.  points: (P, N) array of phase-space points."""
    from scipy.stats import norm

    d1, d2 = periodic_differences(N)
    d1 = advection * d1
    u = np.asarray(points, dtype=np.float64)
    phi = norm.pdf(u, scale=sigma)
    cdf = norm.cdf(u, scale=sigma)
    mean_below = -sigma**2 * phi  # int_{-inf}^{u} v phi(v) dv
    rate = np.zeros(u.shape[0])
    for i in range(N):
        others = np.ones(u.shape[0])
        for k in range(N):
            if k != i:
                others = others * cdf[:, k]
        # c_ii(u_i) + sum_{j != i} c_ij(u_i) E[v_j 1{v_j <= u_j}] / Phi(u_j)
        term = gamma * d2[i, i] * u[:, i] + alpha * np.sin(np.pi * u[:, i]) - u[:, i] * d1[i, i] * u[:, i]
        val = term * others
        for j in range(N):
            if j == i:
                continue
            cij = -u[:, i] * d1[i, j] + gamma * d2[i, j]
            rest = np.ones(u.shape[0])
            for k in range(N):
                if k != i and k != j:
                    rest = rest * cdf[:, k]
            val = val + cij * mean_below[:, j] * rest
        rate -= phi[:, i] * val
    return rate


def reaction_only_solution(points, sigma, alpha, t):
    """F(u, t) for dF/dt = -alpha sum_k sin(pi u_k) dF/du_k from the product
    of Gaussian CDFs: along characteristics tan(pi u / 2) grows like
    exp(alpha pi t), so F(u, t) = prod_k Phi(U0(u_k) / sigma) with U0 the
    foot of the characteristic (branch of the arctangent kept by u)."""
    from scipy.stats import norm

    u = np.asarray(points, dtype=np.float64)
    base = np.arctan(np.tan(0.5 * np.pi * u) * np.exp(-alpha * np.pi * t))
    shift = np.where(u > 1.0, np.pi, np.where(u < -1.0, -np.pi, 0.0))
    u0 = (2.0 / np.pi) * (base + shift)
    u0 = np.where(np.abs(np.abs(u) - 1.0) < 1e-15, u, u0)
    return np.prod(norm.cdf(u0, scale=sigma), axis=1)


def apply_separable_at(points_idx, factors, prob):
    """(L F) at grid index tuples for a separable F = prod_k f_k (factors:
    list of N vectors), without the full grid: every term is a product of
    one-axis operators, so it is a product of 1-D matrix-vector products
    evaluated at the point.  Same terms as ``CdfProblem.apply``."""
    N = prob.N
    idx = np.asarray(points_idx)
    f = [np.asarray(v, dtype=np.complex128) for v in factors]
    d1 = prob.advection * prob.d1
    u = prob.u
    val = [f[k][idx[:, k]] for k in range(N)]
    gval = [(prob.g @ f[k])[idx[:, k]] for k in range(N)]
    jval = [(prob.j @ f[k])[idx[:, k]] for k in range(N)]

    def prod_except(skip):
        p = np.ones(idx.shape[0], dtype=np.complex128)
        for k in range(N):
            if k not in skip:
                p = p * val[k]
        return p

    out = np.zeros(idx.shape[0], dtype=np.complex128)
    for i in range(N):
        ui = u[idx[:, i]]
        coef = -prob.alpha * np.sin(np.pi * ui)
        for j in range(N):
            uj = u[idx[:, j]]
            coef = coef + ui * d1[i, j] * uj - prob.gamma * prob.d2[i, j] * uj
        out += coef * gval[i] * prod_except({i})
        for j in range(N):
            if j == i:
                continue
            c = d1[i, j] * ui - prob.gamma * prob.d2[i, j]
            # J_j acting on G_i F: separable, J along axis j of f_j
            out -= c * gval[i] * jval[j] * prod_except({i, j})
    if prob.diffusion != 0.0:
        for i in range(N):
            out += prob.diffusion * (prob.l2 @ f[i])[idx[:, i]] * prod_except({i})
    return out
