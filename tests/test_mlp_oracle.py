"""The FP64 reference of the ranking MLP: gradient against central finite
differences of the loss (an independent check of the backpropagation
formulas).  CPU only."""
from __future__ import annotations

import numpy as np

import oracle


def _params(rng):
    sizes = [3 * 64, 64, 64 * 64, 64, 64, 1]
    scales = [0.6, 0.1, 0.15, 0.1, 0.2, 0.1]
    return np.concatenate([rng.standard_normal(s) * c for s, c in zip(sizes, scales)])


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    params = _params(rng)
    X = rng.random((40, 3))
    y = (rng.random(40) < 0.3).astype(float)
    g = oracle.mlp_grad(params, X, y)
    h = 1e-6
    idx = np.concatenate([rng.choice(len(params), 120, replace=False), [len(params) - 1]])
    for k in idx:
        e = np.zeros_like(params)
        e[k] = h
        fd = (oracle.mlp_loss(params + e, X, y) - oracle.mlp_loss(params - e, X, y)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 + 1e-5 * abs(fd), (k, fd, g[k])


def test_mlp_forward_shapes_and_relu():
    rng = np.random.default_rng(1)
    params = _params(rng)
    X = rng.random((5, 3))
    z = oracle.mlp_forward(params, X)
    assert z.shape == (5,)
    W1, b1, W2, b2, W3, b3 = oracle.mlp_unpack(params)
    ref = np.array([np.maximum(np.maximum(x @ W1 + b1, 0) @ W2 + b2, 0) @ W3 + b3 for x in X])
    np.testing.assert_allclose(z, ref, rtol=1e-13)


def test_mlp_forward_hand_computed_network():
    """A sparse network whose output is worked out by hand pins the flat
    parameter layout (W1[in][out], b1, W2[in][out], b2, W3, b3), the
    direction of each weight matrix and the ReLU.

    Path 1: feature 0 -> unit 2 (W1[0][2] = 2, b1[2] = -0.5) -> unit 5
    (W2[2][5] = 3, b2[5] = 0.25) -> output (W3[5] = -1.5).  Path 2: feature
    1 -> unit 7 (W1[1][7] = -1) -> unit 9 (W2[7][9] = 4) -> W3[9] = 2, which
    the first ReLU closes for a positive feature 1.  b3 = 0.1.
    x = (0.7, 0.3, 0.9): h1[2] = relu(1.4 - 0.5) = 0.9, h1[7] = relu(-0.3) = 0;
    h2[5] = relu(2.7 + 0.25) = 2.95, h2[9] = 0; output -1.5 * 2.95 + 0.1 = -4.325.
    x = (0.1, -0.5, 0.0): h1[2] = relu(-0.3) = 0, h1[7] = 0.5; h2[5] = relu(0.25)
    = 0.25, h2[9] = 2; output -0.375 + 4 + 0.1 = 3.725."""
    p = np.zeros(3 * 64 + 64 + 64 * 64 + 64 + 64 + 1)
    oW1, ob1, oW2, ob2, oW3, ob3 = 0, 192, 256, 4352, 4416, 4480
    p[oW1 + 0 * 64 + 2] = 2.0
    p[ob1 + 2] = -0.5
    p[oW2 + 2 * 64 + 5] = 3.0
    p[ob2 + 5] = 0.25
    p[oW3 + 5] = -1.5
    p[oW1 + 1 * 64 + 7] = -1.0
    p[oW2 + 7 * 64 + 9] = 4.0
    p[oW3 + 9] = 2.0
    p[ob3] = 0.1
    z = oracle.mlp_forward(p, np.array([[0.7, 0.3, 0.9], [0.1, -0.5, 0.0]]))
    np.testing.assert_allclose(z, [-4.325, 3.725], rtol=0, atol=1e-12)
