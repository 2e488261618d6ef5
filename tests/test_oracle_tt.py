"""Pins for oracle.tt_ref (TT arithmetic and pointwise operator evaluation)."""
import numpy as np
import pytest

from oracle import fullgrid, galerkin, tt_ref
from paper_2403_04946_amd import inputs


def full(c):
    return fullgrid.tt_to_full(c)


def test_eval_matches_full():
    x = inputs.random_tt(4, 5, [1, 3, 4, 2, 1], 0)
    f = full(x)
    idx = inputs.random_points(4, 5, 50, 1)
    got = tt_ref.tt_eval(x, idx)
    ref = f[tuple(idx.T)]
    assert np.abs(got - ref).max() < 1e-14


def test_sum_is_exact():
    x = inputs.random_tt(4, 5, 3, 0)
    y = inputs.random_tt(4, 5, 2, 1)
    z = tt_ref.tt_add(x, y, 0.3 - 0.2j, -1.7)
    assert fullgrid.rel_l2(full(z), (0.3 - 0.2j) * full(x) - 1.7 * full(y)) < 1e-14
    assert tt_ref.tt_ranks(z) == [1, 5, 5, 5, 1]


def test_right_orthogonalize():
    x = inputs.random_tt(5, 4, 6, 2)
    c = tt_ref.right_orthogonalize(x)
    for k in range(1, 5):
        h = c[k].reshape(c[k].shape[0], -1)
        assert np.abs(h @ h.conj().T - np.eye(h.shape[0])).max() < 1e-13
    assert fullgrid.rel_l2(full(c), full(x)) < 1e-13
    assert abs(tt_ref.tt_norm(x) - np.linalg.norm(full(x))) < 1e-12 * np.linalg.norm(full(x))


def test_round_exact_orthogonal_and_bounded():
    x = inputs.random_tt(5, 4, 6, 3)
    y, info = tt_ref.tt_round(x, 0.0)
    assert fullgrid.rel_l2(full(y), full(x)) < 1e-13
    for k in range(4):
        v = y[k].reshape(-1, y[k].shape[2])
        assert np.abs(v.conj().T @ v - np.eye(v.shape[1])).max() < 1e-13
    # ranks never exceed the unfolding dimensions
    assert tt_ref.tt_ranks(y)[1] <= 4 and tt_ref.tt_ranks(y)[4] <= 4
    # a spectrum that decays, so the tolerances below actually cut ranks
    w = tt_ref.tt_add(inputs.random_tt(5, 4, 2, 4), inputs.random_tt(5, 4, 6, 5), 1.0, 0.05)
    nw = np.linalg.norm(full(w))
    for eps in (0.01, 0.05, 0.2):
        z, info = tt_ref.tt_round(w, eps)
        assert sum(info["ranks"]) < sum(tt_ref.tt_ranks(w)[1:-1])
        err = np.linalg.norm(full(z) - full(w))
        tails = [np.sqrt((s[k:] ** 2).sum()) for s, k in zip(info["sigma"], info["ranks"])]
        assert err <= np.sqrt(np.sum(np.square(tails))) * (1 + 1e-10) + 1e-13 * nw
        assert err <= eps * nw * (1 + 1e-10)


def test_round_equals_full_grid_tt_svd():
    # sum of a rank-2 and a rank-3 TT, rounded with a cap: both the TT
    # rounding and the full-grid TT-SVD give the same projection
    x = tt_ref.tt_add(inputs.random_tt(4, 6, 2, 4), inputs.random_tt(4, 6, 3, 5), 1.0, 0.01)
    for eps, cap in ((1e-12, None), (1e-3, 3), (0.0, 2)):
        y, _ = tt_ref.tt_round(x, eps, cap)
        ref = fullgrid.truncate(full(x), eps, cap)
        assert fullgrid.rel_l2(full(y), ref) < 1e-11


@pytest.mark.parametrize("bond,cap", [(1, 2), (2, 5), (3, 3), (4, 1)])
def test_round_with_one_capped_bond_is_the_best_approximation_of_that_unfolding(bond, cap):
    # with no tolerance and a cap on one bond only, the sweep reaches that
    # bond with an exact orthonormal left factor, so the result is the best
    # rank-`cap` approximation of the bond's unfolding (Eckart-Young):
    # checked against a numpy SVD of the full unfolding, for the TT rounding
    # and for the full-grid TT-SVD
    d, n = 5, 4
    x = inputs.random_tt(d, n, [1, 4, 9, 7, 3, 1], 12)
    f = full(x)
    u, s, vh = np.linalg.svd(f.reshape(n ** bond, -1), full_matrices=False)
    best = ((u[:, :cap] * s[:cap]) @ vh[:cap]).reshape(f.shape)
    caps = [0] * (d + 1)
    caps[bond] = cap
    y, info = tt_ref.tt_round(x, 0.0, caps)
    assert info["ranks"][bond - 1] == cap
    assert fullgrid.rel_l2(full(y), best) < 1e-12
    assert fullgrid.rel_l2(fullgrid.truncate(f, 0.0, caps), best) < 1e-12
    # a list of equal caps is the single cap; non-positive entries are none
    z, _ = tt_ref.tt_round(x, 0.0, [7, 2, 2, 2, 2, 9])
    w, _ = tt_ref.tt_round(x, 0.0, 2)
    assert fullgrid.rel_l2(full(z), full(w)) < 1e-13
    v, _ = tt_ref.tt_round(x, 0.0, [0, -1, 0, 0, 0, 0])
    assert fullgrid.rel_l2(full(v), f) < 1e-13


def test_diff_norm_small_differences():
    x = inputs.random_tt(4, 5, 3, 6)
    y = [c.copy() for c in x]
    y[2] = y[2] * (1 + 1e-11)
    ref = np.linalg.norm(full(x) - full(y))
    got = tt_ref.tt_diff_norm(x, y)
    assert abs(got - ref) <= 1e-3 * ref


@pytest.mark.parametrize("nu", [0.0, 0.05])
def test_operator_at_points_matches_full_grid(nu):
    d, n, length = 4, 8, 4.0
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    x = inputs.random_tt(d, n, [1, 3, 2, 4, 1], 8)
    prob = fullgrid.Problem(b, dm, nu, n, length)
    ref = prob.apply(full(x))
    idx = inputs.random_points(d, n, 200, 9)
    got = tt_ref.operator_at_points(x, idx, b, dm, nu, n, length)
    assert np.abs(got - ref[tuple(idx.T)]).max() < 1e-12 * np.abs(ref).max()


def test_operator_at_points_large_d_runs():
    d, n = 50, 128
    b, dm = galerkin.coefficient_B(d), galerkin.coefficient_D(d)
    x = inputs.random_tt(d, n, 4, 10)
    idx = inputs.random_points(d, n, 3, 11)
    v = tt_ref.operator_at_points(x, idx, b, dm, 0.01, n, 8.0)
    assert np.all(np.isfinite(v))
