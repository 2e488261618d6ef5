"""Full-grid semi-discrete operator, RK4 and step-truncation (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The semi-discrete system (Sec. 4, eq. (eqn:ode)) for the characteristic
function phi on the n^d grid is df/dt = L f with

    (L f) = sum_k a_k [ (i/2) sum_{j,l} B_kjl D_jl f + nu sum_j D_kj G_j f ]

where D_jl = G_j G_l for j != l and D_jj = L2_j, the subscript naming the
axis an operator acts on, and the multiplication by the coordinate a_k is
applied after differentiation (Sec. 3 eq. (hyper1), Burgers coefficients of
Sec. 5).  Everything is complex float64 on the full grid; memory is
16 * n^d bytes per field, so only small d is feasible (d=4, n=32: 16.8 MB).

Step-truncation (Sec. 4.1, eq. (eqn:discrete-flow-trunc-intro) and the
truncated Euler / midpoint schemes) applies a TT truncation operator to
every tensor the scheme produces.  For classical RK4 the truncations are
placed as in the midpoint scheme, one after every operator application and
one after every stage combination:

    k1 = T[L f]          y2 = T[f + dt/2 k1]
    k2 = T[L y2]         y3 = T[f + dt/2 k2]
    k3 = T[L y3]         y4 = T[f + dt k3]
    k4 = T[L y4]         f+ = T[f + dt/6 (k1 + 2 k2 + 2 k3 + k4)]

The implicit step-truncation schemes of Sec. 4.1 (eq. (EB-linear),
eq. (MP-linear)) are taken by their definition: the truncation of the exact
solution of the linear system, (I - dt L) x = f (Euler) and
(I - dt/2 L) x = (I + dt/2 L) f (midpoint), solved on the full grid by
GMRES on the grid operator to a relative residual of 1e-13.

The two explicit step-truncation schemes of Sec. 4.1 are taken as written
there: truncated Euler (eq. (adaptive-euler-method)) f+ = T[f + dt T[L f]],
and truncated explicit midpoint (eq. (adaptive-midpoint-method_2))
f+ = T[f + dt T[L(f + dt/2 T[L f])]], whose stage input f + dt/2 T[L f] is
not truncated.

T is the TT-SVD of the full array with a relative tolerance and a rank cap
(App. A.1, Alg. 2 applied to an exact representation; sweep order left to
right, per-bond threshold eps*||f||/sqrt(d-1)).  ``truncate`` returns the
full array of the truncated TT so the RK4 loop stays on the full grid.

Pins (tests/test_oracle_fullgrid.py): assembly against an independent sparse
Kronecker-product matrix; RK4 against the matrix exponential of that matrix
(fourth-order convergence in dt); truncated Euler and midpoint without
truncation against the matrix polynomials I + dt M and I + dt M + dt^2/2 M^2,
their global orders one and two against the matrix exponential and their
Richardson local-error slopes two and three; the implicit steps against a
sparse LU solve of that matrix and their orders one and two;
viscous-only run against the per-axis
exponential and the continuous closed form (second order in h); deterministic
initial state against exp(i a.u(t)) of the Galerkin ODE; phi(0,t) = 1 on
odd-n grids; Hermitian symmetry; TT-SVD error bound and exactness.
"""
import numpy as np

from . import fd


def apply_along(mat, f, axis):
    """Apply an n x n matrix to one axis of the full array f."""
    out = np.tensordot(mat, f, axes=([1], [axis]))
    return np.moveaxis(out, 0, axis)


class Problem:
    """Discrete Burgers-Hopf operator on a full n^d grid.

    diffusion > 0 adds the numerical-diffusion stabilisation of Sec. 5.2
    (explicit runs): kappa sum_k d^2 phi / da_k^2 with kappa = diffusion,
    the caller choosing kappa proportional to dt (Lax-Wendroff-like)."""

    def __init__(self, b, dm, nu, n, length, diffusion=0.0):
        self.diffusion = float(diffusion)
        self.b = np.asarray(b, dtype=np.float64)
        self.dm = np.asarray(dm, dtype=np.float64)
        self.d = self.b.shape[0]
        self.nu = float(nu)
        self.n = int(n)
        self.length = float(length)
        self.a = fd.grid(n, length)
        self.g = fd.first_derivative(n, length)
        self.l2 = fd.second_derivative(n, length)

    def coord(self, k):
        """a_k as an array broadcastable against the full grid."""
        shape = [1] * self.d
        shape[k] = self.n
        return self.a.reshape(shape)

    def apply(self, f):
        """(L f) on the full grid."""
        d = self.d
        f = np.asarray(f, dtype=np.complex128)
        gf = [apply_along(self.g, f, j) for j in range(d)]
        # second derivatives D_jl f for j <= l
        second = {}
        for j in range(d):
            second[(j, j)] = apply_along(self.l2, f, j)
            for l in range(j + 1, d):
                second[(j, l)] = apply_along(self.g, gf[j], l)
        out = np.zeros_like(f)
        for k in range(d):
            inner = np.zeros_like(f)
            for j in range(d):
                for l in range(d):
                    c = self.b[k, j, l]
                    if c != 0.0:
                        key = (j, l) if j <= l else (l, j)
                        inner += (0.5j * c) * second[key]
            for j in range(d):
                if self.dm[k, j] != 0.0:
                    inner += (self.nu * self.dm[k, j]) * gf[j]
            out += self.coord(k) * inner
        if self.diffusion != 0.0:
            for j in range(d):
                out += self.diffusion * second[(j, j)]
        return out


def rk4_step(f, dt, op):
    """One classical RK4 step of df/dt = op(f) (no truncation)."""
    k1 = op(f)
    k2 = op(f + 0.5 * dt * k1)
    k3 = op(f + 0.5 * dt * k2)
    k4 = op(f + dt * k3)
    return f + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def bond_cap(cap, bond):
    """The rank cap of bond `bond` (1..d-1): cap is None (no cap), one int
    for every bond, or d+1 per-bond values (entry b for bond b; <= 0 means
    no cap there)."""
    if cap is None:
        return None
    if np.isscalar(cap):
        return int(cap)
    c = int(cap[bond])
    return c if c > 0 else None


def truncation_rank(sigma, delta, cap):
    """Smallest k >= 1 whose discarded tail sqrt(sum_{i>k} s_i^2) <= delta,
    then capped.  Cut by index only."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    # tail[k] = sum_{i >= k} s_i^2 (0-based), tail[len] = 0
    tail = np.concatenate([np.cumsum(s2[::-1])[::-1], [0.0]])
    k = len(s2)
    for kk in range(1, len(s2) + 1):
        if np.sqrt(tail[kk]) <= delta:
            k = kk
            break
    if cap is not None:
        k = min(k, int(cap))
    return max(k, 1)


def tt_svd(f, eps_rel, cap=None):
    """TT-SVD of a full array, left to right (Alg. 2 on an exact TT).
    cap: as in bond_cap.

    Returns (cores, sigmas) with cores[c] of shape (r_{c-1}, n_c, r_c) and
    sigmas[c] the singular values at bond c (before truncation).
    """
    f = np.asarray(f, dtype=np.complex128)
    dims = f.shape
    d = len(dims)
    norm = np.linalg.norm(f.ravel())
    delta = eps_rel * norm / np.sqrt(max(d - 1, 1))
    cores, sigmas = [], []
    rest = f.reshape(1, -1)
    r_prev = 1
    for c in range(d - 1):
        mat = rest.reshape(r_prev * dims[c], -1)
        u, s, vh = np.linalg.svd(mat, full_matrices=False)
        k = truncation_rank(s, delta, bond_cap(cap, c + 1))
        cores.append(u[:, :k].reshape(r_prev, dims[c], k))
        sigmas.append(s)
        rest = s[:k, None] * vh[:k, :]
        r_prev = k
    cores.append(rest.reshape(r_prev, dims[-1], 1))
    return cores, sigmas


def tt_to_full(cores):
    """Contract TT cores (r_{c-1}, n_c, r_c) into the full array."""
    out = cores[0]
    for core in cores[1:]:
        out = np.tensordot(out, core, axes=([-1], [0]))
    return out.reshape(out.shape[1:-1])


def truncate(f, eps_rel, cap=None):
    """Full array of the TT-SVD truncation of f."""
    cores, _ = tt_svd(f, eps_rel, cap)
    return tt_to_full(cores)


def truncated_rk4_step(f, dt, op, eps_rel, cap=None):
    """RK4 step-truncation with a truncation after every operator application
    and every stage combination (placement described in the module header)."""
    t = lambda x: truncate(x, eps_rel, cap)
    k1 = t(op(f))
    y2 = t(f + 0.5 * dt * k1)
    k2 = t(op(y2))
    y3 = t(f + 0.5 * dt * k2)
    k3 = t(op(y3))
    y4 = t(f + dt * k3)
    k4 = t(op(y4))
    return t(f + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4))


def truncated_euler_step(f, dt, op, eps_rel, cap=None):
    """Truncated explicit Euler, Sec. 4.1 eq. (adaptive-euler-method):
    f+ = T_r[f + dt T_s[L f]]."""
    t = lambda x: truncate(x, eps_rel, cap)
    return t(f + dt * t(op(f)))


def truncated_midpoint_step(f, dt, op, eps_rel, cap=None):
    """Truncated explicit midpoint, Sec. 4.1 eq. (adaptive-midpoint-method_2):
    f+ = T_a[f + dt T_b[L(f + dt/2 T_g[L f])]]; the stage input
    f + dt/2 T_g[L f] itself is not truncated."""
    t = lambda x: truncate(x, eps_rel, cap)
    g = t(op(f))
    h = t(op(f + 0.5 * dt * g))
    return t(f + dt * h)


def solve_shifted(f, c, op, rtol=1e-13):
    """x with x - c op(x) = f on the full grid (GMRES on the grid operator;
    the identity shift makes the system well conditioned for c ||L|| < 1)."""
    import scipy.sparse.linalg as spla

    shape = f.shape
    size = f.size
    a = spla.LinearOperator((size, size), matvec=lambda v: v - c * op(v.reshape(shape)).ravel(),
                            dtype=np.complex128)
    x, info = spla.gmres(a, f.ravel(), rtol=rtol, atol=0.0, restart=200, maxiter=50)
    if info != 0:
        raise RuntimeError(f"oracle GMRES did not converge (info {info})")
    return x.reshape(shape)


def implicit_euler_step(f, dt, op, eps_rel=0.0, cap=None):
    """Implicit step-truncation Euler, Sec. 4.1 eq. (EB-linear):
    f+ = T[(I - dt L)^-1 f]."""
    return truncate(solve_shifted(f, dt, op), eps_rel, cap)


def implicit_midpoint_step(f, dt, op, eps_rel=0.0, cap=None):
    """Implicit step-truncation midpoint, Sec. 4.1 eq. (MP-linear):
    f+ = T[(I - dt/2 L)^-1 (I + dt/2 L) f]."""
    return truncate(solve_shifted(f + 0.5 * dt * op(f), 0.5 * dt, op), eps_rel, cap)


def richardson_local_error(step, f, dt, order):
    """Local error of one step of size dt of a method of the given order,
    estimated against the Richardson extrapolation of one order higher
    built from two steps of dt/2 and the step of dt (the estimate the
    paper's order study uses, Sec. 5.2):
        R = (2^p y_half - y_full) / (2^p - 1),  error = ||y_full - R||."""
    y_full = step(f, dt)
    y_half = step(step(f, 0.5 * dt), 0.5 * dt)
    w = 2.0**order
    r = (w * y_half - y_full) / (w - 1.0)
    return float(np.linalg.norm((y_full - r).ravel()))


def gaussian_ic(mu, sigma, n, length):
    """phi0(a) = prod_k exp(i mu_k a_k - sigma_k^2 a_k^2 / 2), full grid.

    This is the characteristic function of independent Gaussian modal
    amplitudes u_k ~ N(mu_k, sigma_k^2); it is rank one in TT format.
    """
    a = fd.grid(n, length)
    d = len(mu)
    out = np.ones((1,) * d, dtype=np.complex128)
    for k in range(d):
        shape = [1] * d
        shape[k] = n
        fac = np.exp(1j * mu[k] * a - 0.5 * sigma[k] ** 2 * a**2).reshape(shape)
        out = out * fac
    return out


def tridiag_gaussian_ic(mu, sigma, rho, n, length):
    """exp(i mu.a - a^T Sigma a / 2) on the full grid, Sigma tridiagonal
    with Sigma_kk = sigma_k^2 and Sigma_k,k+1 = rho_k sigma_k sigma_k+1: the
    characteristic function of amplitudes u ~ N(mu, Sigma), evaluated from
    the quadratic form."""
    d = len(mu)
    sig = np.diag(np.asarray(sigma, dtype=np.float64) ** 2)
    for k in range(d - 1):
        sig[k, k + 1] = sig[k + 1, k] = rho[k] * sigma[k] * sigma[k + 1]
    a = fd.grid(n, length)
    pts = np.stack(np.meshgrid(*([a] * d), indexing="ij"), axis=-1)  # (n,)*d + (d,)
    quad = np.einsum("...j,jk,...k->...", pts, sig, pts)
    return np.exp(1j * pts @ np.asarray(mu, dtype=np.float64) - 0.5 * quad)


def gaussian_ic_factors(mu, sigma, n, length):
    """The d one-dimensional factors of the rank-one Gaussian IC."""
    a = fd.grid(n, length)
    return [np.exp(1j * mu[k] * a - 0.5 * sigma[k] ** 2 * a**2) for k in range(len(mu))]


def rel_l2(x, y):
    """||x - y||_F / ||y||_F over full arrays."""
    return float(np.linalg.norm((x - y).ravel()) / np.linalg.norm(np.asarray(y).ravel()))
