"""TT arithmetic written from App. A.1 of the paper (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* A TT tensor is a list of cores C_k of shape (r_{k-1}, n_k, r_k),
  r_0 = r_d = 1, whose entries are the iterated matrix product
  f[i_1..i_d] = C_1[0,i_1,:] C_2[:,i_2,:] ... C_d[:,i_d,0]  (App. A.1).
* Sum by concatenation: first cores side by side, middle cores block
  diagonal, last cores stacked; scalar multiplication scales one core
  (App. A.1).
* Orthogonalisation and truncation: App. A.1, Alg. 1 (QR sweep) and Alg. 2
  (truncated-SVD sweep).  The paper notes the left and right variants are
  the same algorithm mirrored; this oracle uses the mirror image that the
  device path uses: right-to-left orthogonalisation by LQ (computed as the
  QR of the conjugate transpose), then a left-to-right sweep of truncated
  SVDs with per-bond threshold eps*||f||/sqrt(d-1) (the relative form of
  Alg. 2's eps/sqrt(d-1)).  The SVD is taken directly of the flattened core
  (the plain definition; no QR preprocessing).
* ``operator_at_points`` evaluates (L x)(i) at given grid points for a TT x,
  at any dimension, in O(d^2 r^2) per point, by summing the operator's terms
  (Sec. 3 eq. (hyper1) with the Burgers coefficients of Sec. 5) over
  modified matrix chains.  It needs no operator representation in TT form.

Pins (tests/test_oracle_tt.py): eval and to_full against full-grid
reconstruction; sum exactness; orthogonality of the outputs; rounding with
eps=0 reproduces the input; the rounding error bound; agreement of rounding
with the full-grid TT-SVD; ``operator_at_points`` against the full-grid
operator at d = 4.
"""
import numpy as np

from . import fd
from .fullgrid import bond_cap, truncation_rank, tt_to_full  # noqa: F401  (re-export)


def tt_eval(cores, idx):
    """Entries at integer index tuples idx of shape (npts, d)."""
    idx = np.asarray(idx)
    v = cores[0][0, idx[:, 0], :]  # (npts, r1)
    for k in range(1, len(cores)):
        sl = np.transpose(cores[k][:, idx[:, k], :], (1, 0, 2))  # (npts, r, r')
        v = np.einsum("pa,pab->pb", v, sl)
    return v[:, 0]


def tt_ranks(cores):
    return [1] + [c.shape[2] for c in cores]


def tt_add(x, y, alpha=1.0, beta=1.0):
    """alpha*x + beta*y by concatenation (App. A.1)."""
    d = len(x)
    out = []
    for k in range(d):
        cx, cy = x[k], y[k]
        if d == 1:
            out.append(alpha * cx + beta * cy)
        elif k == 0:
            out.append(np.concatenate([alpha * cx, beta * cy], axis=2))
        elif k == d - 1:
            out.append(np.concatenate([cx, cy], axis=0))
        else:
            r0 = cx.shape[0] + cy.shape[0]
            r1 = cx.shape[2] + cy.shape[2]
            c = np.zeros((r0, cx.shape[1], r1), dtype=np.complex128)
            c[: cx.shape[0], :, : cx.shape[2]] = cx
            c[cx.shape[0]:, :, cx.shape[2]:] = cy
            out.append(c)
    return out


def right_orthogonalize(cores):
    """Right-to-left LQ sweep; cores 2..d become right-orthonormal:
    H(C_k) H(C_k)^H = I (App. A.1, mirror of Alg. 1)."""
    cores = [np.array(c, dtype=np.complex128) for c in cores]
    for k in range(len(cores) - 1, 0, -1):
        r0, n, r1 = cores[k].shape
        h = cores[k].reshape(r0, n * r1)
        q, rr = np.linalg.qr(h.conj().T)  # h^H = q rr  ->  h = rr^H q^H
        kk = q.shape[1]
        cores[k] = q.conj().T.reshape(kk, n, r1)
        cores[k - 1] = np.einsum("aib,bc->aic", cores[k - 1], rr.conj().T)
    return cores


def tt_norm(cores):
    """Frobenius norm via orthogonalisation."""
    c = right_orthogonalize(cores)
    return float(np.linalg.norm(c[0].ravel()))


def tt_round(cores, eps_rel, cap=None):
    """TT rounding: right-to-left orthogonalisation, then a left-to-right
    truncated-SVD sweep (mirror of Alg. 2).  cap: None, one cap for every
    bond, or d+1 per-bond caps (fullgrid.bond_cap).  Returns (cores, info)
    where info holds the per-bond singular values and kept ranks."""
    c = right_orthogonalize(cores)
    d = len(c)
    norm = float(np.linalg.norm(c[0].ravel()))
    delta = eps_rel * norm / np.sqrt(max(d - 1, 1))
    sig, kept = [], []
    for k in range(d - 1):
        r0, n, r1 = c[k].shape
        v = c[k].reshape(r0 * n, r1)
        u, s, wh = np.linalg.svd(v, full_matrices=False)
        kk = truncation_rank(s, delta, bond_cap(cap, k + 1))
        c[k] = u[:, :kk].reshape(r0, n, kk)
        carry = s[:kk, None] * wh[:kk, :]  # (kk, r1)
        c[k + 1] = np.einsum("ab,bic->aic", carry, c[k + 1])
        sig.append(s)
        kept.append(kk)
    return c, {"sigma": sig, "ranks": kept, "norm": norm, "delta": delta}


def tt_diff_norm(x, y):
    """||x - y|| as the norm of the concatenated difference (no cancellation
    from expanding ||x||^2 + ||y||^2 - 2 Re<x,y>)."""
    return tt_norm(tt_add(x, y, 1.0, -1.0))


def apply_axis(mat, core):
    """mat (n x n) applied along the mode index of a core (r0, n, r1)."""
    return np.einsum("ij,ajb->aib", mat, core)


def operator_at_points(cores, idx, b, dm, nu, n, length):
    """(L x)(i) for a TT x at grid index tuples idx (npts, d).

    (L x)(i) = (i/2) sum_{j,l} A_jl(i) (D_jl x)(i) + sum_j c_j(i) (G_j x)(i)
    with A_jl(i) = sum_k B_kjl a_{i_k} and c_j(i) = nu sum_k a_{i_k} D_kj;
    D_jl = G_j G_l (j != l), L2_j (j = l).  Each (D x)(i) is a matrix chain
    with one or two cores replaced by their differentiated versions.
    """
    idx = np.asarray(idx)
    npts, d = idx.shape
    a = fd.grid(n, length)
    g = fd.first_derivative(n, length)
    l2 = fd.second_derivative(n, length)
    ai = a[idx]  # (npts, d)
    amat = np.einsum("kjl,pk->pjl", b, ai)
    cvec = nu * np.einsum("pk,kj->pj", ai, dm)

    def slices(core, ik):
        return np.transpose(core[:, ik, :], (1, 0, 2))

    s_sl, t_sl, u_sl = [], [], []
    for k in range(d):
        ik = idx[:, k]
        s_sl.append(slices(cores[k], ik))
        t_sl.append(slices(apply_axis(g, cores[k]), ik))
        u_sl.append(slices(apply_axis(l2, cores[k]), ik))
    # prefix[k]: product of slices 0..k-1, (npts, r_k); suffix[k]: slices k..d-1
    prefix = [np.ones((npts, 1), dtype=np.complex128)]
    for k in range(d):
        prefix.append(np.einsum("pa,pab->pb", prefix[-1], s_sl[k]))
    suffix = [None] * (d + 1)
    suffix[d] = np.ones((npts, 1), dtype=np.complex128)
    for k in range(d - 1, -1, -1):
        suffix[k] = np.einsum("pab,pb->pa", s_sl[k], suffix[k + 1])

    def close(vec, sl, k):
        return np.einsum("pa,pab,pb->p", vec, sl, suffix[k + 1])

    total = np.zeros(npts, dtype=np.complex128)
    # diagonal second derivatives and first-derivative (viscous) terms
    for j in range(d):
        total += 0.5j * amat[:, j, j] * close(prefix[j], u_sl[j], j)
        total += cvec[:, j] * close(prefix[j], t_sl[j], j)
    # mixed second derivatives, j < l, counted twice by symmetry of A
    acc = [np.zeros_like(prefix[l]) for l in range(d)]
    for j in range(d):
        v = np.einsum("pa,pab->pb", prefix[j], t_sl[j])
        for l in range(j + 1, d):
            acc[l] += (2.0 * amat[:, j, l])[:, None] * v
            v = np.einsum("pa,pab->pb", v, s_sl[l])
    for l in range(1, d):
        total += 0.5j * close(acc[l], t_sl[l], l)
    return total
