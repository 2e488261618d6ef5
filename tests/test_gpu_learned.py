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


N_IN, WIDTH = 12, 128


def _mlp_data(rng, bsz):
    x = rng.standard_normal((bsz, N_IN)).astype(np.float32)
    t = (np.sin(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2] - 0.3 * np.abs(x[:, 3])).astype(np.float32)
    return x, t


def test_mlp_forward_and_gradients_match_the_oracle(ctx):
    """Device forward pass, loss and gradients (FP16 parameters, FP32
    accumulation) against the oracle's FP64 network evaluated at the same
    FP16-rounded parameters."""
    import torch

    from oracle import mlp as omlp

    rng = np.random.default_rng(4)
    net = tt.MLP(ctx, N_IN, WIDTH, 2048)
    p0 = omlp.init(N_IN, WIDTH, 3) + 0.05 * rng.standard_normal(omlp.count(N_IN, WIDTH))
    net.set_params(p0)
    used = net.get_params(as_used=True).astype(np.float64)
    assert np.abs(used - p0).max() <= 2e-3 * np.abs(p0).max()  # FP16 rounding only
    x, t = _mlp_data(rng, 1500)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    y = net.forward(xd).cpu().numpy()
    yref, _ = omlp.forward(used, x.astype(np.float64), N_IN, WIDTH)
    assert np.abs(y - yref).max() <= 1e-5 * (np.abs(yref).max() + 1)
    loss, g = net.gradients(xd, td)
    gref = omlp.gradients(used, x.astype(np.float64), t.astype(np.float64), N_IN, WIDTH)
    lref = omlp.loss(used, x.astype(np.float64), t.astype(np.float64), N_IN, WIDTH)
    print(f"loss {loss:.6f} (oracle {lref:.6f}); gradient rel error "
          f"{np.linalg.norm(g - gref) / np.linalg.norm(gref):.2e}")
    assert abs(loss - lref) <= 1e-5 * max(lref, 1e-3)
    assert np.linalg.norm(g - gref) <= 1e-4 * np.linalg.norm(gref)
    net.close()


def test_mlp_training_is_deterministic_and_learns(ctx):
    import torch

    from oracle import mlp as omlp

    rng = np.random.default_rng(5)
    x, t = _mlp_data(rng, 2000)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    runs = []
    for _ in range(2):
        net = tt.MLP(ctx, N_IN, WIDTH, 2048)
        net.set_params(omlp.init(N_IN, WIDTH, 7))
        l0, _ = net.gradients(xd, td)
        l1 = net.train(xd, td, 400, 3e-3)
        runs.append((l0, l1, net.get_params()))
        net.close()
    (l0, l1, p1), (_, l1b, p2) = runs
    print(f"training loss {l0:.4f} -> {l1:.4f}")
    assert l1 < 0.1 * l0
    assert l1 == l1b and np.array_equal(p1, p2)
