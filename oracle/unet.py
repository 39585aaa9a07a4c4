"""Oracle: the 3-D convolutional network that corrects the initial SCF density.

The paper has no learned component; this network is the method's extension
that maps the superposition of atomic densities to a corrected start density
(trained on converged densities the method itself produces).  The oracle is
plain NumPy in FP64 with hand-derived backward passes, pinned by central
finite differences in the tests.

Architecture (C channels, input/output on an S^3 patch, S divisible by 8):
    e1 = f(c1b(f(c1a(x))))                     S^3     (c1a: 1 -> C)
    e2 = f(c2b(f(c2a(f(d1(e1))))))              (S/2)^3 (d: stride-2 3^3 conv)
    e3 = f(c3b(f(c3a(f(d2(e2))))))              (S/4)^3
    b  = f(c4b(f(c4a(f(d3(e3))))))              (S/8)^3
    g3 = f(c5b(f(c5a([f(u3(up(b))),  e3]))))    (S/4)^3 (up: nearest x2, [.,.]: channel concat)
    g2 = f(c6b(f(c6a([f(u2(up(g3))), e2]))))
    g1 = f(c7b(f(c7a([f(u1(up(g2))), e1]))))
    y  = out(g1)                                 1^3 conv C -> 1, no activation
f = SiLU(z) = z sigma(z).  3^3 convolutions use zero padding 1 ("same").
Layout: arrays are [C, D, H, W]; weights [C_out, C_in, 3, 3, 3] (or 1^3), bias [C_out].
"""
from __future__ import annotations

import math

import numpy as np

LAYERS = [  # name, c_in multiple of C (None = 1 channel), c_out, kernel, stride
    ("c1a", "in", "C", 3, 1), ("c1b", "C", "C", 3, 1),
    ("d1", "C", "C", 3, 2), ("c2a", "C", "C", 3, 1), ("c2b", "C", "C", 3, 1),
    ("d2", "C", "C", 3, 2), ("c3a", "C", "C", 3, 1), ("c3b", "C", "C", 3, 1),
    ("d3", "C", "C", 3, 2), ("c4a", "C", "C", 3, 1), ("c4b", "C", "C", 3, 1),
    ("u3", "C", "C", 3, 1), ("c5a", "2C", "C", 3, 1), ("c5b", "C", "C", 3, 1),
    ("u2", "C", "C", 3, 1), ("c6a", "2C", "C", 3, 1), ("c6b", "C", "C", 3, 1),
    ("u1", "C", "C", 3, 1), ("c7a", "2C", "C", 3, 1), ("c7b", "C", "C", 3, 1),
    ("out", "C", "1", 1, 1),
]


def _ch(tag: str, C: int) -> int:
    return {"in": 1, "1": 1, "C": C, "2C": 2 * C}[tag]


def init_params(C: int = 32, seed: int = 0) -> dict:
    """He-style normal initialisation (the output layer starts at zero so the
    untrained network predicts no correction)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co, k, _ in LAYERS:
        cin, cout = _ch(ci, C), _ch(co, C)
        fan_in = cin * k ** 3
        w = rng.standard_normal((cout, cin, k, k, k)) * np.sqrt(2.0 / fan_in)
        if name == "out":
            w = np.zeros_like(w)
        p[name + ".w"] = w
        p[name + ".b"] = np.zeros(cout)
    return p


# ---------------------------------------------------------------------------
# primitives
# ---------------------------------------------------------------------------
def conv3d(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int = 1) -> np.ndarray:
    """out[o, p] = b[o] + sum_{i, t} w[o, i, t] x[i, stride p + t - pad] (zero padding)."""
    k = w.shape[2]
    pad = k // 2
    xp = np.pad(x, ((0, 0), (pad, pad), (pad, pad), (pad, pad)))
    D, H, W = x.shape[1:]
    out = np.zeros((w.shape[0], D, H, W))
    for dz in range(k):
        for dy in range(k):
            for dx in range(k):
                sl = xp[:, dz:dz + D, dy:dy + H, dx:dx + W]
                out += np.einsum("oi,idhw->odhw", w[:, :, dz, dy, dx], sl)
    out += b[:, None, None, None]
    if stride == 2:
        out = out[:, ::2, ::2, ::2]
    return out


def conv3d_backward(x: np.ndarray, w: np.ndarray, dy: np.ndarray, stride: int = 1):
    """Gradients (dx, dw, db) of conv3d given dL/d(out)."""
    k = w.shape[2]
    pad = k // 2
    D, H, W = x.shape[1:]
    if stride == 2:
        full = np.zeros((dy.shape[0], D, H, W))
        full[:, ::2, ::2, ::2] = dy
        dy = full
    db = dy.sum(axis=(1, 2, 3))
    xp = np.pad(x, ((0, 0), (pad, pad), (pad, pad), (pad, pad)))
    dw = np.zeros_like(w)
    dxp = np.zeros_like(xp)
    for dz in range(k):
        for dy_ in range(k):
            for dx in range(k):
                sl = xp[:, dz:dz + D, dy_:dy_ + H, dx:dx + W]
                dw[:, :, dz, dy_, dx] = np.einsum("odhw,idhw->oi", dy, sl)
                dxp[:, dz:dz + D, dy_:dy_ + H, dx:dx + W] += np.einsum("oi,odhw->idhw", w[:, :, dz, dy_, dx], dy)
    dx = dxp[:, pad:pad + D, pad:pad + H, pad:pad + W]
    return dx, dw, db


def silu(z: np.ndarray) -> np.ndarray:
    return z / (1.0 + np.exp(-z))


def silu_grad(z: np.ndarray) -> np.ndarray:
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def upsample(x: np.ndarray) -> np.ndarray:
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def upsample_backward(dy: np.ndarray) -> np.ndarray:
    C, D, H, W = dy.shape
    return dy.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).sum(axis=(2, 4, 6))


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def forward(p: dict, x: np.ndarray, keep: bool = False):
    """x [1, S, S, S] -> y [1, S, S, S]; with keep=True also the tape."""
    tape = []

    def conv_act(name, inp, stride=1, act=True):
        z = conv3d(inp, p[name + ".w"], p[name + ".b"], stride)
        tape.append((name, inp, z, stride, act))
        return silu(z) if act else z

    e1 = conv_act("c1b", conv_act("c1a", x))
    e2 = conv_act("c2b", conv_act("c2a", conv_act("d1", e1, 2)))
    e3 = conv_act("c3b", conv_act("c3a", conv_act("d2", e2, 2)))
    bt = conv_act("c4b", conv_act("c4a", conv_act("d3", e3, 2)))
    g3 = conv_act("c5b", conv_act("c5a", np.concatenate([conv_act("u3", upsample(bt)), e3])))
    g2 = conv_act("c6b", conv_act("c6a", np.concatenate([conv_act("u2", upsample(g3)), e2])))
    g1 = conv_act("c7b", conv_act("c7a", np.concatenate([conv_act("u1", upsample(g2)), e1])))
    y = conv_act("out", g1, act=False)
    return (y, tape) if keep else y


def backward(p: dict, tape: list, dy: np.ndarray) -> dict:
    """Parameter gradients for dL/dy, walking the tape in reverse with the
    skip connections accumulated explicitly."""
    C = p["c1b.w"].shape[0]
    g = {k: np.zeros_like(v) for k, v in p.items()}
    byname = {t[0]: t for t in tape}

    def back(name, dout):
        _, inp, z, stride, act = byname[name]
        dz = dout * silu_grad(z) if act else dout
        dx, dw, db = conv3d_backward(inp, p[name + ".w"], dz, stride)
        g[name + ".w"] += dw
        g[name + ".b"] += db
        return dx

    d = back("out", dy)
    d = back("c7a", back("c7b", d))
    du1, de1 = d[:C], d[C:]
    d = upsample_backward(back("u1", du1))
    d = back("c6a", back("c6b", d))
    du2, de2 = d[:C], d[C:]
    d = upsample_backward(back("u2", du2))
    d = back("c5a", back("c5b", d))
    du3, de3 = d[:C], d[C:]
    d = upsample_backward(back("u3", du3))
    d = back("d3", back("c4a", back("c4b", d)))
    d = back("d2", back("c3a", back("c3b", d + de3)))
    d = back("d1", back("c2a", back("c2b", d + de2)))
    back("c1a", back("c1b", d + de1))
    return g


def mse(y: np.ndarray, t: np.ndarray) -> tuple[float, np.ndarray]:
    diff = y - t
    return float((diff * diff).mean()), 2.0 * diff / diff.size


def adam_step(p: dict, g: dict, m: dict, v: dict, step: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8) -> None:
    """Adam (Kingma & Ba) with bias correction, in place."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def gaussian_highpass(box: np.ndarray, sigma: float) -> np.ndarray:
    """box - G_sigma * box for a cubic array: the separable Gaussian
    exp(-k^2 / (2 sigma^2)) truncated at |k| <= ceil(3 sigma), normalised to
    unit sum, applied along each axis in turn with zero values outside."""
    r = int(math.ceil(3.0 * sigma))
    k = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-k * k / (2.0 * sigma * sigma))
    g /= g.sum()
    out = np.asarray(box, dtype=np.float64)
    for axis in range(3):
        out = np.apply_along_axis(lambda v: np.convolve(v, g, mode="same"), axis, out)
    return np.asarray(box, dtype=np.float64) - out
