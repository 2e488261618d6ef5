"""Plain FP64 multilayer perceptron (oracle for the rank predictor).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The learned form's rank predictor is a fully connected network with two
hidden layers of `width` ReLU units and one linear output:

    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3,

trained on the mean squared error L = (1 / 2B) sum_b (y_b - t_b)^2 over a
batch of B samples.  Parameters are one flat vector in the order W1 (width
x n_in, row-major), b1, W2 (width x width), b2, W3 (1 x width), b3.  The
gradients are the textbook backpropagation of L, written out; pinned by
central finite differences (tests/test_oracle_mlp.py).
"""
import numpy as np


def sizes(n_in, width):
    return [(width, n_in), (width,), (width, width), (width,), (1, width), (1,)]


def unpack(params, n_in, width):
    out, o = [], 0
    for shp in sizes(n_in, width):
        k = int(np.prod(shp))
        out.append(np.asarray(params[o:o + k], dtype=np.float64).reshape(shp))
        o += k
    return out


def count(n_in, width):
    return sum(int(np.prod(s)) for s in sizes(n_in, width))


def forward(params, x, n_in, width):
    """x: (B, n_in) -> y (B,), and the hidden activations."""
    w1, b1, w2, b2, w3, b3 = unpack(params, n_in, width)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.maximum(x @ w1.T + b1, 0.0)
    h2 = np.maximum(h1 @ w2.T + b2, 0.0)
    y = (h2 @ w3.T + b3)[:, 0]
    return y, (x, h1, h2)


def loss(params, x, t, n_in, width):
    y, _ = forward(params, x, n_in, width)
    return 0.5 * float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def gradients(params, x, t, n_in, width):
    """Gradient of the loss with respect to the flat parameter vector."""
    w1, b1, w2, b2, w3, b3 = unpack(params, n_in, width)
    y, (x, h1, h2) = forward(params, x, n_in, width)
    bsz = x.shape[0]
    d3 = ((y - np.asarray(t, dtype=np.float64)) / bsz)[:, None]  # dL/dy
    gw3 = d3.T @ h2
    gb3 = d3.sum(axis=0)
    d2 = (d3 @ w3) * (h2 > 0)
    gw2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ w2) * (h1 > 0)
    gw1 = d1.T @ x
    gb1 = d1.sum(axis=0)
    return np.concatenate([g.ravel() for g in (gw1, gb1, gw2, gb2, gw3, gb3)])


def init(n_in, width, seed):
    """He-scaled Gaussian weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for shp in sizes(n_in, width):
        if len(shp) == 2:
            parts.append(rng.standard_normal(shp).ravel() * np.sqrt(2.0 / shp[1]))
        else:
            parts.append(np.zeros(shp))
    return np.concatenate(parts)
