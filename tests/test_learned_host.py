"""Host logic of the learned form: the predictor's features, the width rule
and the training pairs taken from a trajectory (no GPU)."""
import math

import numpy as np

from paper_2403_04946_amd import learned


def _report(d, rank, sv_scale):
    ranks = [1] + [rank] * (d - 1) + [1]
    sv = [[0.0] * 3 + [sv_scale * 10.0 ** (-j) for j in range(5)] for _ in range(d - 1)]
    return ranks, sv


def test_bond_features_layout():
    d, rmax = 5, 32
    ranks, sv = _report(d, 8, 2.0)
    x = learned.bond_features(ranks, sv, 4.0, 0.05, 0.25, rmax)
    assert x.shape == (d - 1, learned.N_FEATURES) and x.dtype == np.float32
    assert np.allclose(x[:, 0], 8 / rmax)
    # zeros in front of the tail are floored at 1e-20: log10 / 10 = -2
    assert np.allclose(x[:, 1:4], -2.0)
    # kept values relative to the norm: 2/4 * 10^-j
    assert np.allclose(x[0, 4:9], [math.log10(0.5 * 10.0 ** (-j)) / 10 for j in range(5)], atol=1e-6)
    assert np.allclose(x[:, 9], math.log10(0.05))
    assert np.allclose(x[:, 10], 0.25)
    assert np.allclose(x[:, 11], [k / d for k in range(1, d)])
    assert np.allclose(x[:, 12], math.log10(4.0) / d)


def test_widths_rule():
    assert learned.widths_from_ranks([3, 5, 4], 4, 16) == [1, 11, 13, 12, 1]
    assert learned.widths_from_ranks([3, 16, 4], 4, 16) is None  # a bond at the cap
    assert learned.widths_from_ranks([0, 1], 3, 16) == [1, 9, 9, 1]
    assert learned.widths_from_ranks([509], 2, 600) == [1, 512, 1]


def test_apply_widths_rule():
    assert learned.apply_widths([1, 10, 20, 1], 64, 80) == [1, 18, 28, 1]
    assert learned.apply_widths([1, 10, 78, 1], 96, 80) == [1, 18, 80, 1]  # capped at the plain width
    assert learned.apply_widths([1, 64, 20, 1], 64, 80) is None  # a derivative at the cap


def test_samples_from_records_pairs_features_with_next_ranks():
    recs = []
    for s in range(3):
        ranks, sv = _report(4, 2 + s, 1.0)
        recs.append({"ranks": ranks, "features": learned.bond_features(ranks, sv, 1.0, 0.1, 0.1 * s, 16)})
    x, y = learned.samples_from_records(recs)
    assert x.shape == (6, learned.N_FEATURES)
    assert np.array_equal(y, np.array([3, 3, 3, 4, 4, 4], dtype=np.float32))
    assert np.array_equal(x[:3], recs[0]["features"]) and np.array_equal(x[3:], recs[1]["features"])
    x0, y0 = learned.samples_from_records(recs[:1])
    assert x0.shape == (0, learned.N_FEATURES) and y0.shape == (0,)


def test_he_init_matches_the_parameter_count():
    p = learned.he_init(13, 128, 0)
    assert p.dtype == np.float32
    assert p.size == 128 * 13 + 128 + 128 * 128 + 128 + 128 + 1
    assert np.all(p[128 * 13:128 * 13 + 128] == 0)


def test_autotune_shape_keys_are_parsed():
    from paper_2403_04946_amd import autotune, tt

    stats = {
        "zgemm:NC:300x32x3000x1": {"ms": 1.5},
        "zgemm_fp16x3:CN:64x80x10240x2": {"ms": 2.0},
        "zgemm_fp32:TN:8x8x8x1": {"ms": 0.1},
        "zgemm": {"ms": 9.0},  # a kernel class, not a shape
        "jacobi:320x320": {"ms": 3.0},
    }
    got = autotune.gemm_shapes(stats)
    assert got == {(tt.TT_PREC_FP64, 0, 2, 300, 32, 3000, 1): 1.5,
                   (tt.TT_PREC_FP16X3, 2, 0, 64, 80, 10240, 2): 2.0,
                   (tt.TT_PREC_FP32, 1, 0, 8, 8, 8, 1): 0.1}
    more = autotune.gemm_shapes({"zgemm:NC:300x32x3000x1": {"ms": 0.5}}, got)
    assert more[(tt.TT_PREC_FP64, 0, 2, 300, 32, 3000, 1)] == 2.0


def test_gemm_table_roundtrip_without_a_device(tmp_path):
    from paper_2403_04946_amd import autotune, tt

    tt.gemm_table_clear()
    tt.gemm_table_set([[0, 0, 2, 64, 64, 128, 1, 32, 64, 4], [2, 2, 0, 16, 16, 64, 1, 1, 1, 2]])
    path = str(tmp_path / "t.json")
    autotune.save(path)
    saved = tt.gemm_table()
    tt.gemm_table_clear()
    assert tt.gemm_table() == []
    autotune.load(path)
    assert tt.gemm_table() == saved and len(saved) == 2
    import pytest

    with pytest.raises(tt.TTError):
        tt.gemm_table_set([[2, 0, 0, 8, 8, 8, 1, 64, 64, 1]])  # split 16-bit tiles are 1 or 2 blocks
    tt.gemm_table_clear()
