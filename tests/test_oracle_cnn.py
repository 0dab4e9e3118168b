"""Pins for the FP64 reference of the control-variate network: parameter count, circular
convolution against an explicit loop, the backward pass against central finite differences,
and a decreasing loss under Adam on a learnable target."""
import numpy as np
import pytest

from oracle import cnn


def test_parameter_count():
    assert cnn.n_params() == 5953


def test_conv_matches_explicit_loops():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 5, 5))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = cnn.conv(x, W, b)
    ref = np.zeros_like(out)
    n = 5
    for bb in range(2):
        for o in range(4):
            for y in range(n):
                for xx in range(n):
                    s = b[o]
                    for c in range(3):
                        for dy in range(3):
                            for dx in range(3):
                                s += W[o, c, dy, dx] * x[bb, c, (y + dy - 1) % n, (xx + dx - 1) % n]
                    ref[bb, o, y, xx] = s
    assert np.max(np.abs(out - ref)) < 1e-12


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = cnn.init_params(3)
    for k in p:
        if k.startswith(("b", "c")):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((3, 6, 6))
    y = rng.standard_normal(3)
    loss, g = cnn.loss_and_grad(p, x, y)
    flat = cnn.flatten(p)
    gflat = cnn.flatten(g)
    idx = rng.choice(len(flat), size=120, replace=False)
    h = 1e-6
    for i in idx:
        v = flat.copy(); v[i] += h
        lp = float(np.mean((cnn.forward(cnn.unflatten(v), x) - y) ** 2))
        v[i] -= 2 * h
        lm = float(np.mean((cnn.forward(cnn.unflatten(v), x) - y) ** 2))
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gflat[i])


def test_adam_reduces_loss_on_learnable_target():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((64, 8, 8))
    y = (x ** 2).mean(axis=(1, 2))          # a smooth function of the field
    p = cnn.init_params(0)
    st = {}
    l0, _ = cnn.loss_and_grad(p, x, y)
    for _ in range(200):
        _, g = cnn.loss_and_grad(p, x, y)
        cnn.adam_step(p, g, st, lr=3e-3)
    l1, _ = cnn.loss_and_grad(p, x, y)
    assert l1 < 0.2 * l0
