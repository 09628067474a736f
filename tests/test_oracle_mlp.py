"""Pins of the rank-predictor network's oracle (oracle/mlp.py): the
network is not part of the paper, so its backpropagation is pinned by
central differences of the loss (FP64) and by special cases with closed
forms."""
import numpy as np

from oracle import mlp


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(mlp.NPARAM)
    off = 0
    for name, shape in mlp.SHAPES:
        n = int(np.prod(shape))
        if name.startswith("W"):
            p[off:off + n] = rng.uniform(-1, 1, n) * np.sqrt(6.0 / shape[0]) * scale
        else:
            p[off:off + n] = rng.uniform(-0.1, 0.1, n)
        off += n
    return p


def test_backprop_matches_central_differences():
    rng = np.random.default_rng(1)
    p = _params(2)
    x = rng.uniform(-2, 0, (5, mlp.IN))
    t = rng.normal(0, 0.5, 5)
    _, g = mlp.gradient(p, x, t)
    # every output-layer parameter and a random sample of the others
    idx = np.concatenate([np.arange(mlp.NPARAM - mlp.H - 1, mlp.NPARAM),
                          rng.choice(mlp.NPARAM - mlp.H - 1, 400, replace=False)])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss(pp, x, t) - mlp.loss(pm, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_constant_network_closed_form():
    """All weights and hidden biases zero: y = b4 for every input, so the
    loss is mean (b4 - t)^2, its b4-derivative 2 (b4 - mean t), and every
    other derivative vanishes (the hidden activations are relu(0) = 0)."""
    rng = np.random.default_rng(3)
    p = np.zeros(mlp.NPARAM)
    p[-1] = 0.7
    x = rng.normal(size=(9, mlp.IN))
    t = rng.normal(size=9)
    loss, g = mlp.gradient(p, x, t)
    assert abs(loss - np.mean((0.7 - t) ** 2)) < 1e-14
    assert abs(g[-1] - 2 * (0.7 - t.mean())) < 1e-14
    assert np.all(g[:-1] == 0.0)


def test_linear_regime_closed_form():
    """Zero hidden weights, zero first and second biases and a positive
    third bias: the third layer's activation is a3 = b3 for every input, so
    y = b3 . W4 + b4 and dL/dW4 = b3 * mean 2 (y - t), dL/db3 = W4 * mean
    2 (y - t)."""
    rng = np.random.default_rng(4)
    p = np.zeros(mlp.NPARAM)
    off = {}
    o = 0
    for name, shape in mlp.SHAPES:
        off[name] = o
        o += int(np.prod(shape))
    b3 = rng.uniform(0.5, 1.5, mlp.H)
    W4 = rng.normal(size=mlp.H)
    p[off["b3"]:off["b3"] + mlp.H] = b3
    p[off["W4"]:off["W4"] + mlp.H] = W4
    p[-1] = -0.2
    x = rng.normal(size=(6, mlp.IN))
    t = rng.normal(size=6)
    y0 = b3 @ W4 - 0.2
    loss, g = mlp.gradient(p, x, t)
    assert abs(loss - np.mean((y0 - t) ** 2)) < 1e-12
    gW4 = g[off["W4"]:off["W4"] + mlp.H]
    assert np.allclose(gW4, b3 * np.mean(2 * (y0 - t)), rtol=1e-12, atol=1e-14)
    # the first two layers output relu(0) = 0, so W1 and W3 get no gradient
    assert np.allclose(g[off["b3"]:off["b3"] + mlp.H], W4 * np.mean(2 * (y0 - t)), rtol=1e-12)
    assert np.all(g[off["W1"]:off["b1"]] == 0.0) and np.all(g[off["W3"]:off["b3"]] == 0.0)
