"""Pins of the warm-start network oracle (CPU): the convolution against
SciPy's 2D correlation, the backward operators by adjointness, the whole
gradient by finite differences, Adam by its closed forms."""
import numpy as np
import pytest
import scipy.signal as sps

from oracle import warmstart as ws


def rand_params(channels, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return {k: rng.standard_normal((3, 3, ci, co)) * scale / np.sqrt(9 * ci)
            for k, (ci, co) in ws.shapes(channels).items()}


def test_conv_is_scipy_correlation_with_zero_padding():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 9, 7, 3))
    W = rng.standard_normal((3, 3, 3, 4))
    out = ws.conv(x, W)
    for b in range(2):
        for o in range(4):
            ref = sum(sps.correlate2d(x[b, :, :, i], W[:, :, i, o], mode="same", boundary="fill")
                      for i in range(3))
            assert np.allclose(out[b, :, :, o], ref, atol=1e-12)


def test_backward_operators_are_adjoints():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 8, 6, 3))
    W = rng.standard_normal((3, 3, 3, 5))
    d = rng.standard_normal((2, 8, 6, 5))
    lhs = np.sum(ws.conv(x, W) * d)
    assert np.isclose(lhs, np.sum(x * ws.conv_grad_input(d, W)), rtol=1e-12)
    assert np.isclose(lhs, np.sum(W * ws.conv_grad_weight(x, d)), rtol=1e-12)
    p = rng.standard_normal((2, 4, 3, 3))
    assert np.isclose(np.sum(ws.pool(x) * p), np.sum(x * ws.pool_grad(p)), rtol=1e-12)
    u = rng.standard_normal((2, 16, 12, 3))
    assert np.isclose(np.sum(ws.up(x) * u), np.sum(x * ws.up_grad(u)), rtol=1e-12)
    assert np.allclose(ws.pool(ws.up(x)), x)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_finite_differences(seed):
    channels = (4, 6, 8, 8, 8)
    params = rand_params(channels, seed, scale=1.0)
    rng = np.random.default_rng(10 + seed)
    x = rng.standard_normal((2, 16, 16, 2))
    target = rng.standard_normal((2, 16, 16, 2))
    y, t = ws.forward(params, x)
    g = ws.backward(params, t, target)
    for k in ws.NAMES:                  # every weight tensor, one direction each
        dirn = {n: np.zeros_like(p) for n, p in params.items()}
        dirn[k] = rng.standard_normal(params[k].shape)
        eps = 1e-6
        lp = ws.loss(ws.forward({n: params[n] + eps * dirn[n] for n in params}, x)[0], target)
        lm = ws.loss(ws.forward({n: params[n] - eps * dirn[n] for n in params}, x)[0], target)
        fd = (lp - lm) / (2 * eps)
        an = float(np.sum(g[k] * dirn[k]))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (k, fd, an)


def test_adam_closed_forms():
    rng = np.random.default_rng(3)
    p = {"a": rng.standard_normal((3, 3, 2, 2))}
    g = {"a": rng.standard_normal((3, 3, 2, 2))}
    m = {"a": np.zeros((3, 3, 2, 2))}
    v = {"a": np.zeros((3, 3, 2, 2))}
    # with a constant gradient the bias-corrected moments are g and g^2 at
    # every step, so every step moves by -lr g / (|g| + eps)
    q = p
    for step in range(1, 6):
        q2, m, v = ws.adam_step(q, g, m, v, step, lr=1e-2)
        assert np.allclose(q2["a"] - q["a"], -1e-2 * g["a"] / (np.abs(g["a"]) + 1e-8), rtol=1e-9)
        q = q2
