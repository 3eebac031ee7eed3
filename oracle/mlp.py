"""fp64 reference for the learned key-CDF model.  TEST INFRASTRUCTURE ONLY.

The paper partitions the parallel merge at "segmentation points" (Sec. 2.1,
and the overhead discussion of Sec. 3.2).  The learned part predicts those
points with a small multilayer perceptron F(x) ~ CDF(key); an exact bounded
search then corrects each prediction, so sort results never depend on it.
This module is the plain definition of that perceptron, its loss, its
gradients and the Adam update (Kingma and Ba, 2015, Algorithm 1), in float64
NumPy, with no blocking or fusion.

Parameter vector layout (1153 values, float):
    W1[32]        first layer weights (32 x 1)
    b1[32]
    W2[32*32]     second layer, row-major [out][in]
    b2[32]
    W3[32]        output layer (1 x 32)
    b3[1]
Activations are ReLU with derivative 0 at 0 (the derivative of max(z, 0) is
taken as 1 only for z > 0).  The loss is the mean squared error over the
batch.
"""
import numpy as np

H = 32
N_PARAMS = H + H + H * H + H + H + 1  # 1153

_SLICES = {}
_o = 0
for _name, _size in (("W1", H), ("b1", H), ("W2", H * H), ("b2", H), ("W3", H), ("b3", 1)):
    _SLICES[_name] = slice(_o, _o + _size)
    _o += _size
assert _o == N_PARAMS


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (N_PARAMS,)
    return (p[_SLICES["W1"]], p[_SLICES["b1"]], p[_SLICES["W2"]].reshape(H, H),
            p[_SLICES["b2"]], p[_SLICES["W3"]], p[_SLICES["b3"]][0])


def forward(p, x):
    """Model output for each input x[b]; returns (y, cache)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = np.outer(x, W1) + b1          # [B, H]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2                # [B, H]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3                   # [B]
    return y, (x, z1, h1, z2, h2)


def loss(p, x, t):
    y, _ = forward(p, x)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def backward(p, x, t):
    """Loss and its gradient with respect to every parameter (chain rule)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    y, (x, z1, h1, z2, h2) = forward(p, x)
    t = np.asarray(t, dtype=np.float64)
    B = x.shape[0]
    L = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / B             # dL/dy, [B]
    gW3 = h2.T @ dy
    gb3 = np.sum(dy)
    dh2 = np.outer(dy, W3)             # [B, H]
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1                   # [H_out, H_in]
    gb2 = np.sum(dz2, axis=0)
    dh1 = dz2 @ W2                     # [B, H]
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ x
    gb1 = np.sum(dz1, axis=0)
    g = np.concatenate([gW1, gb1, gW2.reshape(-1), gb2, gW3, [gb3]])
    return L, g


def adam_step(p, m, v, g, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; `step` counts from 1.  Returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v
