"""The GEMM launch-shape autotuner: tuned GEMMs stay within the accuracy of
the untuned ones, are deterministic for a given table, and the table can be
read, written and cleared through the C ABI."""
import numpy as np
import pytest

from gpu_util import make_ctx
from paper_2403_04946_amd import autotune, inputs, tt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    tt.gemm_table_clear()
    yield c
    tt.gemm_table_clear()  # later tests run with the rule, not this table
    c.sync()
    c.close()


def _gemm(ctx, prec, M, N, K, seed):
    import torch

    rng = np.random.default_rng(seed)
    a = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    b = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    A = torch.from_numpy(np.asfortranarray(a).ravel(order="F")).cuda()
    B = torch.from_numpy(np.asfortranarray(b).ravel(order="F")).cuda()
    C = torch.zeros(M * N, dtype=torch.complex128, device="cuda")
    tt.tt_zgemm(ctx, 0, 0, M, N, K, 1.0, A, M, M * K, B, K, K * N, 0.0, C, M, M * N, 1, precision=prec)
    return C.cpu().numpy().reshape((M, N), order="F"), a @ b, np.abs(a) @ np.abs(b)


@pytest.mark.parametrize("prec,M,N,K,coef", [(tt.TT_PREC_FP64, 300, 32, 3000, 1e-13), (tt.TT_PREC_FP64, 4100, 20, 37, 1e-13),
                                             (tt.TT_PREC_FP16X3, 200, 48, 2000, 2.0 ** -18),
                                             (tt.TT_PREC_FP32, 96, 96, 5000, 2.0 ** -17)])
def test_tuned_gemm_is_accurate_and_deterministic(ctx, prec, M, N, K, coef):
    choice, us = tt.gemm_autotune(ctx, prec, 0, 0, M, N, K, 1)
    print(f"precision {prec} {M}x{N}x{K}: tile {choice[:2]}, split {choice[2]}, {us:.1f} us")
    assert us > 0 and 1 <= choice[2] <= 128
    assert [prec, 0, 0, M, N, K, 1, *choice] in tt.gemm_table()
    g1, ref, absprod = _gemm(ctx, prec, M, N, K, 1)
    g2, _, _ = _gemm(ctx, prec, M, N, K, 1)
    assert np.array_equal(g1, g2)
    bound = coef * absprod * (np.sqrt(K) if prec == tt.TT_PREC_FP64 else 1.0) + 1e-300
    assert np.all(np.abs(g1 - ref) <= bound)


def test_table_set_get_clear(ctx):
    tt.gemm_table_clear()
    assert tt.gemm_table() == []
    entry = [0, 0, 2, 64, 64, 128, 1, 32, 64, 4]
    tt.gemm_table_set([entry])
    assert tt.gemm_table() == [entry]
    with pytest.raises(tt.TTError):
        tt.gemm_table_set([[0, 0, 0, 8, 8, 8, 1, 48, 48, 1]])  # no such tile
    with pytest.raises(tt.TTError):
        tt.gemm_table_set([[2, 0, 0, 8, 8, 8, 1, 1, 1, 0]])  # split 0
    tt.gemm_table_clear()
    assert tt.gemm_table() == []


def test_profile_and_tune_a_step(ctx, tmp_path):
    """The workflow on a small step: profile the GEMM shapes, tune the
    heaviest, save and reload the table; the tuned step stays within
    rounding of the untuned one."""
    d, n, cap = 8, 32, 16
    op = tt.Operator(ctx, d, n, 4.0, 0.05)
    f0 = tt.Tensor(ctx, d, n, cap)
    f0.set_cores(inputs.random_tt(d, n, cap, 3))
    f = tt.Tensor(ctx, d, n, cap)

    def step():
        f.copy_from(f0)
        tt.tt_step(ctx, op, f, 1e-3, cap, 1e-10, tt.TT_APPLY_SKETCH, 24, 5, precision=tt.TT_PREC_FP16X3)

    tt.gemm_table_clear()
    step()
    plain = tt.Tensor(ctx, d, n, cap)
    plain.copy_from(f)
    shapes = autotune.profile_shapes(ctx, step)
    assert shapes and all(len(k) == 7 for k in shapes)
    res = autotune.tune(ctx, shapes, top=6)
    assert len(res) >= 1
    path = str(tmp_path / "table.json")
    autotune.save(path)
    saved = tt.gemm_table()
    tt.gemm_table_clear()
    autotune.load(path)
    assert tt.gemm_table() == saved
    step()
    # ||tuned - plain|| / ||plain|| from TT inner products (resolves ~1e-8)
    xx, yy, xy = (tt.tt_dot(ctx, a, b).real for a, b in ((f, f), (plain, plain), (f, plain)))
    diff = np.sqrt(max(xx + yy - 2 * xy, 0.0) / yy)
    print("tuned vs untuned step:", diff)
    assert diff <= 1e-6
    tt.gemm_table_clear()
    for t_ in (f0, f, plain):
        t_.close()
    op.close()
