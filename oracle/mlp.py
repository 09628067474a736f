"""Oracle of the rank-predictor network (test infrastructure only: the
library never imports it).  Plain numpy in FP64.

The network is the multilayer perceptron of the learned rank predictor:
33 inputs, three hidden layers of 128 with ReLU, one linear output, the
mean squared error against targets.  The parameter vector has the layout
the library uses: W1 (33 x 128, row i = input i), b1 (128), W2 (128 x 128),
b2, W3 (128 x 128), b3, W4 (128 x 1), b4 (1).  Backpropagation is written
layer by layer from the chain rule; its result is pinned in the tests by
central differences and by closed forms of special cases.
"""
import numpy as np

IN, H = 33, 128
SHAPES = [("W1", (IN, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
          ("W3", (H, H)), ("b3", (H,)), ("W4", (H, 1)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    """Views of the parameter vector as the named arrays."""
    out, off = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(p[off:off + n], dtype=np.float64).reshape(shape)
        off += n
    return out


def forward(p, x):
    """Output (batch) and the pre-activations of the hidden layers."""
    w = unpack(p)
    z1 = x @ w["W1"] + w["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ w["W2"] + w["b2"]
    a2 = np.maximum(z2, 0.0)
    z3 = a2 @ w["W3"] + w["b3"]
    a3 = np.maximum(z3, 0.0)
    y = (a3 @ w["W4"] + w["b4"])[:, 0]
    return y, (z1, a1, z2, a2, z3, a3)


def loss(p, x, t):
    y, _ = forward(p, x)
    return float(np.mean((y - t) ** 2))


def gradient(p, x, t):
    """Loss and its gradient with respect to the parameter vector."""
    w = unpack(p)
    y, (z1, a1, z2, a2, z3, a3) = forward(p, x)
    B = x.shape[0]
    dy = 2.0 * (y - t) / B                      # dL/dy
    g = {}
    g["W4"] = a3.T @ dy[:, None]
    g["b4"] = np.array([dy.sum()])
    d3 = (dy[:, None] @ w["W4"].T) * (z3 > 0)   # dL/dz3
    g["W3"] = a2.T @ d3
    g["b3"] = d3.sum(axis=0)
    d2 = (d3 @ w["W3"].T) * (z2 > 0)
    g["W2"] = a1.T @ d2
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ w["W2"].T) * (z1 > 0)
    g["W1"] = x.T @ d1
    g["b1"] = d1.sum(axis=0)
    flat = np.concatenate([g[name].ravel() for name, _ in SHAPES])
    return float(np.mean((y - t) ** 2)), flat
