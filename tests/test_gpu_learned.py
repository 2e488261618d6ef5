"""Learned form: the randomised tt_round whose per-bond sketch widths the
rank predictor sets, its a posteriori error, and (below) the predictor's
MLP kernels against the oracle's FP64 MLP."""
import numpy as np
import pytest

from gpu_util import full, make_ctx, rel, upload
from oracle import fullgrid, tt_ref
from paper_2403_04946_amd import inputs, tt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    yield c
    c.sync()
    c.close()


def _sum_tt(d, n):
    return tt_ref.tt_add(inputs.random_tt(d, n, 3, 5), inputs.random_tt(d, n, 4, 6), 1.0, 0.5)


def test_randomized_round_exact_when_widths_cover_the_ranks(ctx):
    d, n = 4, 8
    x = _sum_tt(d, n)  # ranks 7
    tx = upload(ctx, x, caps=8)
    ty = tt.Tensor(ctx, d, n, 12)
    err = tt.tt_round_randomized(ctx, tx, [1, 10, 10, 10, 1], 7, ty)
    assert rel(full(ty), fullgrid.tt_to_full(x)) < 1e-11
    assert err < 1e-7  # the inner-product formula resolves about 1e-8
    # right-orthonormal cores after the first
    for c in ty.get_cores()[1:]:
        h = c.reshape(c.shape[0], -1, order="F")
        assert np.abs(h @ h.conj().T - np.eye(h.shape[0])).max() < 1e-12
    tx.close()
    ty.close()


def test_randomized_round_reports_its_error(ctx):
    d, n = 4, 8
    x = _sum_tt(d, n)
    tx = upload(ctx, x, caps=8)
    ty = tt.Tensor(ctx, d, n, 8)
    err = tt.tt_round_randomized(ctx, tx, [1, 3, 4, 3, 1], 11, ty)
    assert max(ty.ranks()) <= 4
    full_x = fullgrid.tt_to_full(x)
    true = rel(full(ty), full_x)
    print(f"randomised rounding to widths 3,4,3: reported {err:.6e}, true {true:.6e}")
    assert 1e-3 < true < 1.0
    assert abs(err - true) < 1e-6
    # never better than the optimal (deterministic) truncation to the same ranks
    ref, _ = tt_ref.tt_round(x, 0.0, 4)
    assert true >= rel(fullgrid.tt_to_full(ref), full_x) * (1 - 1e-9)
    tx.close()
    ty.close()
