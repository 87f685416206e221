"""Pins of the MLP oracle: in plain float64 its analytic gradients equal
central finite differences; the bfloat16 rounding is round-to-nearest-even;
one Adam step from zero moments moves every parameter by lr against the
sign of its gradient."""
import numpy as np
import pytest

from oracle import mlp

SHAPE = (5, 16, 7, 3)


def _params(seed, shape=SHAPE):
    rng = np.random.default_rng(seed)
    _, total = mlp.layers(*shape)
    return rng.normal(0, 0.4, size=total)


def test_bf16_rounding():
    # exact bf16 values stay; halfway cases go to even; 1 + 2^-8 rounds to 1
    assert mlp.bf16(np.array([1.0]))[0] == 1.0
    assert mlp.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0
    assert mlp.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6
    assert mlp.bf16(np.array([1.0 + 2 ** -7]))[0] == 1.0 + 2 ** -7
    x = np.random.default_rng(0).normal(size=1000)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2 ** -8 + 1e-300)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = _params(2)
    x = rng.normal(size=(6, SHAPE[0]))
    t = rng.normal(size=(6, SHAPE[2]))
    mask = (rng.uniform(size=t.shape) > 0.2).astype(float)
    w = rng.uniform(0.5, 2.0, size=SHAPE[2])

    def loss(pp, xx):
        y, _ = mlp.forward(SHAPE, pp, xx, rounding=False)
        return mlp.mse_grad(y, t, mask, w)[1]

    y, cache = mlp.forward(SHAPE, p, x, rounding=False)
    dy, _ = mlp.mse_grad(y, t, mask, w)
    g, dx = mlp.backward(SHAPE, p, cache, dy, rounding=False)
    h = 1e-6
    idx = rng.choice(p.size, size=60, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (loss(p + e, x) - loss(p - e, x)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)), (i, fd, g[i])
    for (r, c) in [(0, 0), (3, 4), (5, 2)]:
        e = np.zeros_like(x)
        e[r, c] = h
        fd = (loss(p, x + e) - loss(p, x - e)) / (2 * h)
        assert abs(fd - dx[r, c]) <= 1e-6 * max(1e-3, abs(fd))


def test_rounded_forward_close_to_exact():
    rng = np.random.default_rng(3)
    p = _params(4)
    x = rng.normal(size=(32, SHAPE[0]))
    y1, _ = mlp.forward(SHAPE, p, x, rounding=True)
    y0, _ = mlp.forward(SHAPE, p, x, rounding=False)
    assert np.max(np.abs(y1 - y0)) < 0.05 * np.max(np.abs(y0))


def test_adam_first_step_is_signed_lr():
    g = np.array([0.3, -2.0, 1e-3, -5e-2])
    p = np.zeros(4)
    p1, m, v = mlp.adam(p, g, np.zeros(4), np.zeros(4), step=1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(p1, -0.01 * np.sign(g), rtol=1e-9)
