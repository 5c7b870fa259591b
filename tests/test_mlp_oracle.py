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
