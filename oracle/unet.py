"""ORACLE -- test infrastructure only.  Plain numpy reference of the learned
hole filler: a 4-level convolutional encoder-decoder that replaces the
disocclusion fill of Section 7 (the paper itself rejects data-driven patching
as too heavy for mobile GPUs and compares against a GAN baseline; the
network here is this project's own, not the paper's).

Architecture (3x3 convolutions, stride 1, zero padding 1, no bias):
  encoder level l = 0..3, channels C_l = 32 * 2^l:
      conv + ReLU, conv + ReLU  (e_l); 2x2 average pool between levels;
  decoder l = 2, 1, 0:
      nearest x2 upsample, conv (C_{l+1} -> C_l) + ReLU (a_l),
      concat [a_l, e_l], conv (2 C_l -> C_l) + ReLU, conv (C_l -> C_l) + ReLU;
  head: conv (32 -> 3), no activation: a residual added to the plain fill.
Input (5 channels): plain-filled RGB / 255, hole mask (1 on holes), and
log-depth mapped from [log 0.3, log 50] to [0, 1] and clamped.

Numerics: products and sums in float64; every stored activation, gradient
and weight copy used by a convolution is rounded to bfloat16 (round to
nearest, ties to even) at the same points as the GPU path.  The head output
(residual) is kept in full precision.  ``rounding=False`` turns all the
rounding off (used for the finite-difference gradient pin).

Weights: w[t, co, ci] with tap t = 3*ky + kx applied to the input pixel at
(y + ky - 1, x + kx - 1) (cross-correlation, as in most frameworks).
"""
from __future__ import annotations

import numpy as np

LOG_ZMIN, LOG_ZMAX = np.log(0.3), np.log(50.0)

# (name, cin, cout) in forward order; "cat" inputs are [decoder half, skip half].
LAYERS = [
    ("e0a", 5, 32), ("e0b", 32, 32),
    ("e1a", 32, 64), ("e1b", 64, 64),
    ("e2a", 64, 128), ("e2b", 128, 128),
    ("e3a", 128, 256), ("e3b", 256, 256),
    ("d2a", 256, 128), ("d2b", 256, 128), ("d2c", 128, 128),
    ("d1a", 128, 64), ("d1b", 128, 64), ("d1c", 64, 64),
    ("d0a", 64, 32), ("d0b", 64, 32), ("d0c", 32, 32),
    ("head", 32, 3),
]


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


class Rounder:
    def __init__(self, on: bool):
        self.on = on

    def __call__(self, x):
        return bf16(x) if self.on else np.asarray(x, dtype=np.float64)


# ------------------------------------------------------------- primitives --

def conv3x3(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """x [N, H, W, Cin], w [9, Cout, Cin] -> [N, H, W, Cout], zero padding."""
    N, H, W, C = x.shape
    xp = np.zeros((N, H + 2, W + 2, C), dtype=np.float64)
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((N, H, W, w.shape[1]), dtype=np.float64)
    for t in range(9):
        ky, kx = divmod(t, 3)
        out += xp[:, ky:ky + H, kx:kx + W, :] @ w[t].T
    return out


def conv3x3_grad_input(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Gradient w.r.t. the input of conv3x3 given the output gradient g."""
    N, H, W, _ = g.shape
    dxp = np.zeros((N, H + 2, W + 2, w.shape[2]), dtype=np.float64)
    for t in range(9):
        ky, kx = divmod(t, 3)
        dxp[:, ky:ky + H, kx:kx + W, :] += g @ w[t]
    return dxp[:, 1:-1, 1:-1]


def conv3x3_grad_weight(x: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Gradient w.r.t. w [9, Cout, Cin] given the input x and output gradient g."""
    N, H, W, C = x.shape
    xp = np.zeros((N, H + 2, W + 2, C), dtype=np.float64)
    xp[:, 1:-1, 1:-1] = x
    gw = np.zeros((9, g.shape[3], C), dtype=np.float64)
    gf = g.reshape(-1, g.shape[3])
    for t in range(9):
        ky, kx = divmod(t, 3)
        gw[t] = gf.T @ xp[:, ky:ky + H, kx:kx + W, :].reshape(-1, C)
    return gw


def avgpool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_grad(g):
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_grad(g):
    N, H, W, C = g.shape
    return g.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


# ------------------------------------------------------------ input/output --

def make_input(rgba: np.ndarray, depth: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """[N, H, W, 5] network input from the plain fill (RGBA u8, depth, mask u8)."""
    rgb = rgba[..., :3].astype(np.float64) / 255.0
    hole = (mask != 0).astype(np.float64)[..., None]
    with np.errstate(divide="ignore", invalid="ignore"):
        ld = (np.log(depth.astype(np.float64)) - LOG_ZMIN) / (LOG_ZMAX - LOG_ZMIN)
    ld = np.where(np.isnan(ld), 1.0, ld)
    ld = np.clip(ld, 0.0, 1.0)[..., None]
    return np.concatenate([rgb, hole, ld], axis=-1)


def composite(res: np.ndarray, rgba: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Hole pixels: u8 = clamp(rint(255 * (plain/255 + residual))), alpha and
    non-hole pixels unchanged.  The quantisation turns floating point into an
    integer, so it is decided in the precision the device uses for it: FP32
    (plain/255 and the product correctly rounded, the sum of an FP32
    residual, round half to even)."""
    f = np.float32
    pred = rgba[..., :3].astype(f) / f(255.0) + np.asarray(res).astype(f)
    q = np.clip(np.rint(f(255.0) * pred), 0, 255).astype(np.uint8)
    out = rgba.copy()
    hole = mask != 0
    out[..., :3][hole] = q[hole]
    return out


def masked_l1(res, rgba, mask, target):
    """Mean |plain/255 + res - target/255| over hole pixels and RGB; and d/dres."""
    pred = rgba[..., :3].astype(np.float64) / 255.0 + res
    diff = pred - target[..., :3].astype(np.float64) / 255.0
    hole = (mask != 0)[..., None]
    n = int((mask != 0).sum())
    if n == 0:
        return 0.0, np.zeros_like(res)
    loss = float(np.abs(diff * hole).sum() / (3.0 * n))
    grad = np.sign(diff) * hole / (3.0 * n)
    return loss, grad


# --------------------------------------------------------- network -------

def forward(params, x, rounding: bool = True):
    """params: list of w [9, cout, cin] in LAYERS order; x [N, H, W, 5].
    Returns (residual [N, H, W, 3], cache of every stored activation)."""
    r = Rounder(rounding)
    W = [r(w) for w in params]
    relu = lambda v: np.maximum(v, 0.0)  # noqa: E731
    a = {}
    a["x"] = r(x)
    a["e0a"] = r(relu(conv3x3(a["x"], W[0])))
    a["e0b"] = r(relu(conv3x3(a["e0a"], W[1])))
    a["p1"] = r(avgpool2(a["e0b"]))
    a["e1a"] = r(relu(conv3x3(a["p1"], W[2])))
    a["e1b"] = r(relu(conv3x3(a["e1a"], W[3])))
    a["p2"] = r(avgpool2(a["e1b"]))
    a["e2a"] = r(relu(conv3x3(a["p2"], W[4])))
    a["e2b"] = r(relu(conv3x3(a["e2a"], W[5])))
    a["p3"] = r(avgpool2(a["e2b"]))
    a["e3a"] = r(relu(conv3x3(a["p3"], W[6])))
    a["e3b"] = r(relu(conv3x3(a["e3a"], W[7])))
    a["u2"] = upsample2(a["e3b"])
    a["d2a"] = r(relu(conv3x3(a["u2"], W[8])))
    a["c2"] = np.concatenate([a["d2a"], a["e2b"]], axis=-1)
    a["d2b"] = r(relu(conv3x3(a["c2"], W[9])))
    a["d2c"] = r(relu(conv3x3(a["d2b"], W[10])))
    a["u1"] = upsample2(a["d2c"])
    a["d1a"] = r(relu(conv3x3(a["u1"], W[11])))
    a["c1"] = np.concatenate([a["d1a"], a["e1b"]], axis=-1)
    a["d1b"] = r(relu(conv3x3(a["c1"], W[12])))
    a["d1c"] = r(relu(conv3x3(a["d1b"], W[13])))
    a["u0"] = upsample2(a["d1c"])
    a["d0a"] = r(relu(conv3x3(a["u0"], W[14])))
    a["c0"] = np.concatenate([a["d0a"], a["e0b"]], axis=-1)
    a["d0b"] = r(relu(conv3x3(a["c0"], W[15])))
    a["d0c"] = r(relu(conv3x3(a["d0b"], W[16])))
    res = conv3x3(a["d0c"], W[17])
    return res, a


def backward(params, a, g_res, rounding: bool = True):
    """Weight gradients (list, LAYERS order, float64) and the stored activation
    gradients, given the cache of ``forward`` and d(loss)/d(residual)."""
    r = Rounder(rounding)
    W = [r(w) for w in params]
    pos = lambda v: (v > 0).astype(np.float64)  # noqa: E731
    gw = [None] * len(LAYERS)
    g = {}
    g["res"] = r(g_res)
    gw[17] = conv3x3_grad_weight(a["d0c"], g["res"])
    g["d0c"] = r(conv3x3_grad_input(g["res"], W[17]) * pos(a["d0c"]))
    gw[16] = conv3x3_grad_weight(a["d0b"], g["d0c"])
    g["d0b"] = r(conv3x3_grad_input(g["d0c"], W[16]) * pos(a["d0b"]))
    gw[15] = conv3x3_grad_weight(a["c0"], g["d0b"])
    g["c0"] = r(conv3x3_grad_input(g["d0b"], W[15]) * pos(a["c0"]))
    g_d0a, g_e0b_skip = g["c0"][..., :32], g["c0"][..., 32:]
    gw[14] = conv3x3_grad_weight(a["u0"], g_d0a)
    g["u0"] = r(conv3x3_grad_input(g_d0a, W[14]) * pos(a["u0"]))
    g["d1c"] = r(upsample2_grad(g["u0"]))
    gw[13] = conv3x3_grad_weight(a["d1b"], g["d1c"])
    g["d1b"] = r(conv3x3_grad_input(g["d1c"], W[13]) * pos(a["d1b"]))
    gw[12] = conv3x3_grad_weight(a["c1"], g["d1b"])
    g["c1"] = r(conv3x3_grad_input(g["d1b"], W[12]) * pos(a["c1"]))
    g_d1a, g_e1b_skip = g["c1"][..., :64], g["c1"][..., 64:]
    gw[11] = conv3x3_grad_weight(a["u1"], g_d1a)
    g["u1"] = r(conv3x3_grad_input(g_d1a, W[11]) * pos(a["u1"]))
    g["d2c"] = r(upsample2_grad(g["u1"]))
    gw[10] = conv3x3_grad_weight(a["d2b"], g["d2c"])
    g["d2b"] = r(conv3x3_grad_input(g["d2c"], W[10]) * pos(a["d2b"]))
    gw[9] = conv3x3_grad_weight(a["c2"], g["d2b"])
    g["c2"] = r(conv3x3_grad_input(g["d2b"], W[9]) * pos(a["c2"]))
    g_d2a, g_e2b_skip = g["c2"][..., :128], g["c2"][..., 128:]
    gw[8] = conv3x3_grad_weight(a["u2"], g_d2a)
    g["u2"] = r(conv3x3_grad_input(g_d2a, W[8]) * pos(a["u2"]))
    g["e3b"] = r(upsample2_grad(g["u2"]))
    gw[7] = conv3x3_grad_weight(a["e3a"], g["e3b"])
    g["e3a"] = r(conv3x3_grad_input(g["e3b"], W[7]) * pos(a["e3a"]))
    gw[6] = conv3x3_grad_weight(a["p3"], g["e3a"])
    g["p3"] = r(conv3x3_grad_input(g["e3a"], W[6]))
    g["e2b"] = r((avgpool2_grad(g["p3"]) + g_e2b_skip) * pos(a["e2b"]))
    gw[5] = conv3x3_grad_weight(a["e2a"], g["e2b"])
    g["e2a"] = r(conv3x3_grad_input(g["e2b"], W[5]) * pos(a["e2a"]))
    gw[4] = conv3x3_grad_weight(a["p2"], g["e2a"])
    g["p2"] = r(conv3x3_grad_input(g["e2a"], W[4]))
    g["e1b"] = r((avgpool2_grad(g["p2"]) + g_e1b_skip) * pos(a["e1b"]))
    gw[3] = conv3x3_grad_weight(a["e1a"], g["e1b"])
    g["e1a"] = r(conv3x3_grad_input(g["e1b"], W[3]) * pos(a["e1a"]))
    gw[2] = conv3x3_grad_weight(a["p1"], g["e1a"])
    g["p1"] = r(conv3x3_grad_input(g["e1a"], W[2]))
    g["e0b"] = r((avgpool2_grad(g["p1"]) + g_e0b_skip) * pos(a["e0b"]))
    gw[1] = conv3x3_grad_weight(a["e0a"], g["e0b"])
    g["e0a"] = r(conv3x3_grad_input(g["e0b"], W[1]) * pos(a["e0a"]))
    gw[0] = conv3x3_grad_weight(a["x"], g["e0a"])
    return gw, g


def loss_of(params, rgba, depth, mask, target, rounding: bool = True):
    res, _ = forward(params, make_input(rgba, depth, mask), rounding)
    return masked_l1(res, rgba, mask, target)[0]


# ---------------------------------------------------------------- AdamW --

def adamw_step(w, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wd=0.01):
    """One AdamW update (decoupled weight decay, bias-corrected moments), in
    the order: decay, moments, bias correction, update.  step counts from 1."""
    w = w * (1.0 - lr * wd)
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    w = w - lr * mh / (np.sqrt(vh) + eps)
    return w, m, v
