"""MLP surrogate oracle -- TEST INFRASTRUCTURE (numpy, float64).

The forward and backward passes of the surrogate network written directly
from their definitions, with the same bfloat16 rounding points as the GPU
kernels (weights and GEMM inputs rounded to nearest even; everything else
float64 here, float32 there).  With rounding=False the same code is plain
float64, which central finite differences pin in the tests.

Network: d_in -> width -> ... -> width -> d_out; `hidden` SiLU layers
(SiLU(z) = z sigmoid(z)); linear output.  Parameter vector: for each layer W
(out x in, row-major) then b.
"""
import numpy as np


def bf16(x):
    """Round to bfloat16 (nearest even) through float32, as float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def layers(d_in, width, d_out, hidden):
    dims = [d_in] + [width] * hidden + [d_out]
    out, off = [], 0
    for i in range(len(dims) - 1):
        n_in, n_out = dims[i], dims[i + 1]
        out.append((n_in, n_out, off, off + n_in * n_out))
        off += n_in * n_out + n_out
    return out, off


def unpack(params, shape):
    lys, total = layers(*shape)
    params = np.asarray(params, np.float64)
    assert params.size == total
    return [(params[w:w + i * o].reshape(o, i), params[b:b + o]) for (i, o, w, b) in lys]


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(shape, params, x, rounding=True):
    """Returns y and the cache the backward pass needs."""
    R = bf16 if rounding else (lambda a: np.asarray(a, np.float64))
    Ws = unpack(params, shape)
    xb = R(x)
    cache = []
    for li, (W, b) in enumerate(Ws):
        z = xb @ R(W).T + b
        cache.append((xb, z))
        if li < len(Ws) - 1:
            xb = R(z * _sig(z))
        else:
            y = z
    return y, cache


def backward(shape, params, cache, dy, rounding=True):
    """Gradient of the parameter vector and of the input, given dL/dy."""
    R = bf16 if rounding else (lambda a: np.asarray(a, np.float64))
    Ws = unpack(params, shape)
    lys, total = layers(*shape)
    grad = np.zeros(total)
    dh = None
    for li in range(len(Ws) - 1, -1, -1):
        W, b = Ws[li]
        xb, z = cache[li]
        if li == len(Ws) - 1:
            dz = np.asarray(dy, np.float64)
        else:
            s = _sig(z)
            dz = dh * s * (1.0 + z * (1.0 - s))
        dzb = R(dz)
        i, o, woff, boff = lys[li]
        grad[woff:woff + i * o] = (dzb.T @ xb).ravel()
        grad[boff:boff + o] = dz.sum(axis=0)
        dh = dzb @ R(W)
    return grad, dh


def mse_grad(y, t, mask=None, col_weight=None):
    """loss = sum w_j mask (y - t)^2 / B and its gradient."""
    y = np.asarray(y, np.float64)
    B = y.shape[0]
    w = np.ones_like(y)
    if mask is not None:
        w = w * mask
    if col_weight is not None:
        w = w * np.asarray(col_weight)[None, :]
    d = y - t
    return 2.0 * w * d / B, float((w * d * d).sum() / B)


def adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; returns new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
