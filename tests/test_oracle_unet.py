"""Pins of the density-network oracle: convolution against a brute-force
loop, every backward pass against central finite differences, the upsampling
adjoint identity, and Adam's closed-form first step."""
import math

import numpy as np
import pytest

from oracle import unet as U


def _brute_conv(x, w, b, stride):
    k = w.shape[2]
    pad = k // 2
    C, D, H, W = x.shape
    Do = (D + stride - 1) // stride
    out = np.zeros((w.shape[0], Do, Do, Do))
    for o in range(w.shape[0]):
        for z in range(Do):
            for y in range(Do):
                for xx in range(Do):
                    s = b[o]
                    for i in range(C):
                        for dz in range(k):
                            for dy in range(k):
                                for dx in range(k):
                                    zz, yy, x3 = stride * z + dz - pad, stride * y + dy - pad, stride * xx + dx - pad
                                    if 0 <= zz < D and 0 <= yy < H and 0 <= x3 < W:
                                        s += w[o, i, dz, dy, dx] * x[i, zz, yy, x3]
                    out[o, z, y, xx] = s
    return out


@pytest.mark.parametrize("k,stride", [(3, 1), (3, 2), (1, 1)])
def test_conv_matches_brute_force(k, stride):
    rng = np.random.default_rng(k + stride)
    x = rng.standard_normal((3, 6, 6, 6))
    w = rng.standard_normal((2, 3, k, k, k))
    b = rng.standard_normal(2)
    assert np.allclose(U.conv3d(x, w, b, stride), _brute_conv(x, w, b, stride), atol=1e-12)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_backward_finite_differences(stride):
    rng = np.random.default_rng(10 + stride)
    x = rng.standard_normal((2, 4, 4, 4))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    gy = rng.standard_normal(U.conv3d(x, w, b, stride).shape)
    dx, dw, db = U.conv3d_backward(x, w, gy, stride)
    f = lambda xx, ww, bb: float((U.conv3d(xx, ww, bb, stride) * gy).sum())
    eps = 1e-6
    for arr, grad, args in ((x, dx, 0), (w, dw, 1), (b, db, 2)):
        for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(5)]:
            a1 = [x.copy(), w.copy(), b.copy()]
            a2 = [x.copy(), w.copy(), b.copy()]
            a1[args][idx] += eps
            a2[args][idx] -= eps
            num = (f(*a1) - f(*a2)) / (2 * eps)
            assert abs(num - grad[idx]) < 1e-6 * max(1.0, abs(num))


def test_upsample_adjoint():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 3, 3))
    y = rng.standard_normal((2, 6, 6, 6))
    assert abs((U.upsample(x) * y).sum() - (x * U.upsample_backward(y)).sum()) < 1e-12


def test_silu_grad():
    z = np.linspace(-6, 6, 41)
    num = (U.silu(z + 1e-6) - U.silu(z - 1e-6)) / 2e-6
    assert np.allclose(U.silu_grad(z), num, atol=1e-8)


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(4)
    p = U.init_params(C=4, seed=5)
    p["out.w"] = rng.standard_normal(p["out.w"].shape) * 0.5
    x = rng.standard_normal((1, 8, 8, 8))
    t = rng.standard_normal((1, 8, 8, 8))
    y, tape = U.forward(p, x, keep=True)
    loss, dy = U.mse(y, t)
    g = U.backward(p, tape, dy)
    eps = 1e-6
    for name in ("c1a.w", "c2b.w", "d3.w", "c4b.b", "u3.w", "c5a.w", "c7a.w", "out.w", "out.b", "d1.b"):
        for _ in range(2):
            idx = tuple(rng.integers(0, s) for s in p[name].shape)
            old = p[name][idx]
            p[name][idx] = old + eps
            lp = U.mse(U.forward(p, x), t)[0]
            p[name][idx] = old - eps
            lm = U.mse(U.forward(p, x), t)[0]
            p[name][idx] = old
            num = (lp - lm) / (2 * eps)
            assert abs(num - g[name][idx]) < 1e-6 * max(1e-3, abs(num)), (name, num, g[name][idx])


def test_mse_is_the_mean_square_and_its_gradient():
    # a uniform offset c: loss c^2 and gradient 2c/n everywhere; one element off by d: d^2 / n
    t = np.random.default_rng(2).standard_normal((1, 4, 4, 4))
    n = t.size
    loss, dy = U.mse(t + 0.3, t)
    assert abs(loss - 0.09) < 1e-15 and np.allclose(dy, 0.6 / n, rtol=1e-14)
    y = t.copy()
    y[0, 1, 2, 3] += 0.5
    loss, dy = U.mse(y, t)
    assert abs(loss - 0.25 / n) < 1e-15
    assert abs(dy[0, 1, 2, 3] - 1.0 / n) < 1e-15 and np.count_nonzero(dy) == 1


def test_adam_first_step_is_signed_lr():
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.5, -4.0, 1e-3])}
    m = {"a": np.zeros(3)}
    v = {"a": np.zeros(3)}
    U.adam_step(p, g, m, v, 1, lr=0.01)
    assert np.allclose(p["a"], np.array([1.0, -2.0, 3.0]) - 0.01 * np.sign(g["a"]), atol=1e-7)


def test_untrained_network_predicts_zero():
    p = U.init_params(C=4, seed=1)
    y = U.forward(p, np.random.default_rng(0).standard_normal((1, 8, 8, 8)))
    assert np.all(y == 0.0)


def test_gaussian_highpass_closed_forms():
    # a unit impulse away from the faces: the blur is the separable product
    # of the normalised weights, so the high-pass is 1 - g0^3 at the impulse
    # and -g_i g_j g_k elsewhere; a constant field far from the faces is
    # removed exactly
    sigma = 1.3
    r = math.ceil(3 * sigma)
    k = np.arange(-r, r + 1)
    g = np.exp(-k * k / (2 * sigma * sigma))
    g /= g.sum()
    D = 2 * r + 5
    c = D // 2
    b = np.zeros((D, D, D))
    b[c, c, c] = 1.0
    hp = U.gaussian_highpass(b, sigma)
    assert abs(hp[c, c, c] - (1.0 - g[r] ** 3)) < 1e-14
    assert abs(hp[c + 1, c - 2, c + 3] + g[r + 1] * g[r - 2] * g[r + 3]) < 1e-15
    assert abs(hp.sum()) < 1e-13
    ones = U.gaussian_highpass(np.ones((D, D, D)), sigma)
    assert np.abs(ones[r:D - r, r:D - r, r:D - r]).max() < 1e-14
