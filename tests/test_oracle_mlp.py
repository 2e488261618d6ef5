"""Pins for oracle.mlp: analytic gradients against central finite
differences, and the network's output against a hand-built case."""
import numpy as np

from oracle import mlp


def test_gradients_match_finite_differences():
    n_in, width, bsz = 5, 7, 9
    rng = np.random.default_rng(0)
    p = mlp.init(n_in, width, 1) + 0.01 * rng.standard_normal(mlp.count(n_in, width))
    x = rng.standard_normal((bsz, n_in))
    t = rng.standard_normal(bsz)
    g = mlp.gradients(p, x, t, n_in, width)
    h = 1e-6
    num = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        num[i] = (mlp.loss(p + e, x, t, n_in, width) - mlp.loss(p - e, x, t, n_in, width)) / (2 * h)
    assert np.abs(g - num).max() <= 1e-6 * max(1.0, np.abs(num).max())
    # a plausible slip (dropping the 1/B, a sign) would fail by orders of magnitude
    assert np.abs(g).max() > 1e-3


def test_forward_hand_built():
    # width 2, one input: h1 = relu([x, -x]), h2 = relu(h1), y = h2[0] + h2[1] + 1 = |x| + 1
    n_in, width = 1, 2
    w1 = np.array([[1.0], [-1.0]])
    w2 = np.eye(2)
    w3 = np.array([[1.0, 1.0]])
    p = np.concatenate([w1.ravel(), [0, 0], w2.ravel(), [0, 0], w3.ravel(), [1.0]])
    x = np.array([[-2.0], [0.5], [3.0]])
    y, _ = mlp.forward(p, x, n_in, width)
    assert np.allclose(y, [3.0, 1.5, 4.0])
