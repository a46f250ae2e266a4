"""The learned hole filler: a 4-level convolutional encoder-decoder that
predicts a residual over the plain nearest-background fill on hole pixels.

This module only sequences the library's kernels (include/yoro_nn.h) and
owns their buffers (torch device tensors, allocated once per input shape so
a whole forward or training step can be captured in a HIP graph).  All
arithmetic runs in the HIP kernels.

Layers (3x3 convolutions, no bias; channel counts as (cin, cout)):
  e0a (5, 32), e0b (32, 32), pool, e1a (32, 64), e1b (64, 64), pool,
  e2a (64, 128), e2b (128, 128), pool, e3a (128, 256), e3b (256, 256),
  up, d2a (256, 128), cat[d2a, e2b], d2b (256, 128), d2c (128, 128),
  up, d1a (128, 64),  cat[d1a, e1b], d1b (128, 64),  d1c (64, 64),
  up, d0a (64, 32),   cat[d0a, e0b], d0b (64, 32),   d0c (32, 32),
  head (32, 3): the residual, no activation.
ReLU after every convolution except the head.  The 5-channel input is padded
to 32 channels and the 3-channel head to 32 outputs with zero weights, so
every convolution is a multiple of 32 wide for the matrix cores.
"""
from __future__ import annotations

import copy
import ctypes

import numpy as np
import torch

from . import yoro

ARCH = [
    ("e0a", 5, 32), ("e0b", 32, 32),
    ("e1a", 32, 64), ("e1b", 64, 64),
    ("e2a", 64, 128), ("e2b", 128, 128),
    ("e3a", 128, 256), ("e3b", 256, 256),
    ("d2a", 256, 128), ("d2b", 256, 128), ("d2c", 128, 128),
    ("d1a", 128, 64), ("d1b", 128, 64), ("d1c", 64, 64),
    ("d0a", 64, 32), ("d0b", 64, 32), ("d0c", 32, 32),
    ("head", 32, 3),
]
EPI_NONE, EPI_RELU, EPI_RELU_GRAD = 0, 1, 2


def _pad32(c: int) -> int:
    return (c + 31) // 32 * 32


_nn = None


def nnlib():
    """libyoro.so with the yoro_nn_* signatures set."""
    global _nn
    if _nn is None:
        L = yoro.load()
        vp, i32, i64, f32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
        sig = {
            "yoro_nn_conv3x3": [vp, i32, i32, i32, i32, i32, vp, i32, vp, i32, i32, i32, i32, vp, i32, vp],
            "yoro_nn_conv3x3_wgrad": [vp, i32, vp, i32, i32, i32, i32, i32, i32, vp, vp, sz, vp],
            "yoro_nn_pack_weights": [vp, i32, i32, vp, vp, vp],
            "yoro_nn_avgpool2": [vp, i32, i32, i32, i32, i32, vp, i32, vp],
            "yoro_nn_avgpool2_grad": [vp, i32, vp, i32, vp, i32, i32, i32, i32, i32, vp, i32, vp],
            "yoro_nn_upsample2": [vp, i32, i32, i32, i32, i32, vp, i32, vp],
            "yoro_nn_upsample2_grad": [vp, i32, i32, i32, i32, i32, vp, i32, vp],
            "yoro_nn_input": [vp, vp, vp, i64, vp, vp],
            "yoro_nn_l1_grad": [vp, vp, vp, vp, i64, vp, vp, vp, vp],
            "yoro_nn_composite": [vp, vp, vp, i64, vp, vp],
            "yoro_nn_adamw": [vp, vp, vp, vp, i64, f32, f32, f32, f32, f32, i32, vp],
            "yoro_nn_tile_holes": [vp, i32, i32, i32, vp, vp],
            "yoro_nn_gather_crops": [vp, vp, vp, i32, i32, vp, i32, i32, vp, vp, vp, vp],
            "yoro_nn_composite_tiles": [vp, vp, i32, i32, i32, vp, vp, i32, i32, vp, vp],
            "yoro_model_layout": [vp, vp, vp],
            "yoro_model_pack": [vp, vp, vp],
            "yoro_model_pack_train": [vp, vp, vp, vp],
            "yoro_model_residual": [vp, vp, vp, vp, i32, i32, i32, vp, vp, sz, vp],
            "yoro_model_fill": [vp, vp, vp, vp, i32, i32, i32, vp, vp, sz, vp],
            "yoro_model_fill_tiles": [vp, vp, vp, vp, i32, i32, vp, i32, i32, i32, i32, vp, vp, sz, vp],
            "yoro_model_fill_bands": [vp, vp, vp, vp, i32, i32, i32, i32, vp, vp, vp, sz, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = i32
        L.yoro_nn_conv3x3_wgrad_workspace.argtypes = [i32, i32, i32, i32, i32]
        L.yoro_nn_conv3x3_wgrad_workspace.restype = sz
        L.yoro_model_weights_bytes.argtypes = []
        L.yoro_model_weights_bytes.restype = sz
        L.yoro_model_workspace_layout.argtypes = [i32, i32, i32, vp]
        L.yoro_model_workspace_layout.restype = i32
        L.yoro_model_workspace_bytes.argtypes = [i32, i32, i32]
        L.yoro_model_workspace_bytes.restype = sz
        L.yoro_model_bands_workspace_bytes.argtypes = [i32, i32, i32, i32]
        L.yoro_model_bands_workspace_bytes.restype = sz
        L.yoro_model_tiles_workspace_bytes.argtypes = [i32, i32, i32, i32]
        L.yoro_model_tiles_workspace_bytes.restype = sz
        _nn = L
    return _nn


def boundary_reach() -> int:
    """How far (level-0 pixels) the zero padding at a crop's edge reaches into
    the network's output: outputs farther than this from every edge of a crop
    that is not a frame edge equal those of the whole frame, provided the crop
    sits on the 8-pixel grid of the three 2x2 pools.  Each 3x3 convolution
    adds one pixel, a pool halves (rounding up), an upsample doubles, and a
    concatenation takes the larger reach of its two inputs."""
    r, skips = 0, []
    for level in range(4):
        r += 2                      # two convolutions
        if level < 3:
            skips.append(r)
            r = -(-r // 2)          # 2x2 average pool
    for level in (2, 1, 0):
        r = 2 * r + 1               # upsample, then the first decoder convolution
        r = max(r, skips[level])    # concatenation with the encoder's output
        r += 2                      # two more convolutions
    return r + 1                    # head


TILE, HALO = 128, 64                # crop = 256 x 256, the training window size


def tile_plan(counts, h: int, w: int, tile: int = TILE, halo: int = HALO):
    """Crops for the tile x tile blocks of an h x w frame whose hole count is
    nonzero: int32 [k, 4] rows (crop x, crop y, block x, block y).  Each crop
    (tile + 2 halo square) is placed on the frame, shifted inward at the
    frame's edges, so every crop edge is a frame edge or at least `halo`
    pixels from its block."""
    crop = tile + 2 * halo
    if crop > h or crop > w:
        raise ValueError(f"frame {w}x{h} smaller than a {crop}-pixel crop")
    if tile % 8 or halo % 8 or h % 8 or w % 8:
        raise ValueError("tile, halo and the frame size must be multiples of 8")
    ntx = (w + tile - 1) // tile
    idx = np.flatnonzero(np.asarray(counts).reshape(-1))
    ty, tx = (idx // ntx) * tile, (idx % ntx) * tile
    ox = np.clip(tx - halo, 0, w - crop)
    oy = np.clip(ty - halo, 0, h - crop)
    return np.stack([ox, oy, tx, ty], 1).astype(np.int32).reshape(-1, 4)


def _p(t, offset: int = 0):
    """Device address of tensor t plus an element offset."""
    return ctypes.c_void_p(t.data_ptr() + offset * t.element_size())


def _ok(status):
    if status != 0:
        raise yoro.YoroError(status, yoro.load().yoro_last_error().decode())


class Buffers:
    """Activations and gradients for n images of h x w (h, w multiples of 8)."""

    def __init__(self, n, h, w, device, train: bool):
        if h % 8 or w % 8:
            raise ValueError("height and width must be multiples of 8 (three 2x2 pools)")
        self.n, self.h, self.w = n, h, w
        P = [n * (h >> l) * (w >> l) for l in range(4)]
        self.P = P
        bf = dict(dtype=torch.bfloat16, device=device)
        E = lambda p, c: torch.empty((p, c), **bf)  # noqa: E731
        self.x0 = E(P[0], 32)
        self.e0a, self.c0, self.d0b, self.d0c, self.u0 = E(P[0], 32), E(P[0], 64), E(P[0], 32), E(P[0], 32), E(P[0], 64)
        self.p1, self.e1a, self.c1, self.d1b, self.d1c, self.u1 = (E(P[1], 32), E(P[1], 64), E(P[1], 128), E(P[1], 64),
                                                                  E(P[1], 64), E(P[1], 128))
        self.p2, self.e2a, self.c2, self.d2b, self.d2c, self.u2 = (E(P[2], 64), E(P[2], 128), E(P[2], 256),
                                                                  E(P[2], 128), E(P[2], 128), E(P[2], 256))
        self.p3, self.e3a, self.e3b = E(P[3], 128), E(P[3], 256), E(P[3], 256)
        self.res = torch.empty((P[0], 3), dtype=torch.float32, device=device)
        self.train = train
        if train:
            self.g_res = E(P[0], 32)
            self.g_d0c, self.g_d0b, self.g_c0, self.g_u0 = E(P[0], 32), E(P[0], 32), E(P[0], 64), E(P[0], 64)
            self.g_d1c, self.g_d1b, self.g_c1, self.g_u1 = E(P[1], 64), E(P[1], 64), E(P[1], 128), E(P[1], 128)
            self.g_d2c, self.g_d2b, self.g_c2, self.g_u2 = E(P[2], 128), E(P[2], 128), E(P[2], 256), E(P[2], 256)
            self.g_e3b, self.g_e3a, self.g_p3 = E(P[3], 256), E(P[3], 256), E(P[3], 128)
            self.g_e2b, self.g_e2a, self.g_p2 = E(P[2], 128), E(P[2], 128), E(P[2], 64)
            self.g_e1b, self.g_e1a, self.g_p1 = E(P[1], 64), E(P[1], 64), E(P[1], 32)
            self.g_e0b, self.g_e0a = E(P[0], 32), E(P[0], 32)
            self.loss = torch.zeros(1, dtype=torch.float32, device=device)
            self.l1_ws = torch.empty(16 + 512, dtype=torch.float32, device=device)
            L = nnlib()
            ws = 0
            for lev, (cin, cout) in [(0, (32, 32)), (0, (64, 32)), (1, (32, 64)), (1, (64, 64)), (1, (128, 64)),
                                     (2, (64, 128)), (2, (128, 128)), (2, (256, 128)), (3, (128, 256)),
                                     (3, (256, 256))]:
                ws = max(ws, L.yoro_nn_conv3x3_wgrad_workspace(n, h >> lev, w >> lev, cin, cout))
            self.wgrad_ws = torch.empty(ws // 4 + 4, dtype=torch.float32, device=device)

    def first(self, n):
        """The same buffers, used for the first n images only."""
        if n == self.n:
            return self
        if not 0 < n <= self.n:
            raise ValueError(f"{n} images do not fit buffers for {self.n}")
        c = copy.copy(self)
        c.n = n
        c.P = [n * (self.h >> lev) * (self.w >> lev) for lev in range(4)]
        return c


class UNet:
    """Parameters (FP32 masters, bf16 copies, AdamW state) and the kernel sequence."""

    def __init__(self, device="cuda", params=None, seed: int = 0):
        self.device = torch.device(device)
        self.shapes = [(9, _pad32(cout) if name == "head" else cout, _pad32(cin)) for name, cin, cout in ARCH]
        sizes = [int(np.prod(s)) for s in self.shapes]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        n = int(self.offsets[-1])
        lay = (ctypes.c_int64 * (len(ARCH) + 1))()
        nnlib().yoro_model_layout(None, None, lay)
        if list(lay) != [int(o) for o in self.offsets]:
            raise RuntimeError("parameter layout differs from the library's model layout")
        f32 = dict(dtype=torch.float32, device=self.device)
        self.master = torch.zeros(n, **f32)
        self.grad = torch.zeros(n, **f32)
        self.m = torch.zeros(n, **f32)
        self.v = torch.zeros(n, **f32)
        self.wf = torch.zeros(n, dtype=torch.bfloat16, device=self.device)
        self.wb = torch.zeros(n, dtype=torch.bfloat16, device=self.device)
        self.step = 0
        self.set_params(params if params is not None else init_params(seed))
        self._bufs = {}

    # -------------------------------------------------------- parameters --
    def _view(self, flat, i):
        return flat[int(self.offsets[i]):int(self.offsets[i + 1])].view(self.shapes[i])

    def set_params(self, params):
        """params: list of FP32 arrays [9, cout, cin] in ARCH order (unpadded)."""
        if len(params) != len(ARCH):
            raise ValueError("wrong number of parameter tensors")
        self.master.zero_()
        for i, (p, (name, cin, cout)) in enumerate(zip(params, ARCH)):
            p = np.asarray(p, dtype=np.float32)
            if p.shape != (9, cout, cin):
                raise ValueError(f"{name}: shape {p.shape}, want {(9, cout, cin)}")
            self._view(self.master, i)[:, :cout, :cin] = torch.from_numpy(p).to(self.device)
        self.pack()

    def get_params(self):
        return [self._view(self.master, i)[:, :cout, :cin].cpu().numpy().copy()
                for i, (_, cin, cout) in enumerate(ARCH)]

    def get_grads(self):
        return [self._view(self.grad, i)[:, :cout, :cin].cpu().numpy().copy()
                for i, (_, cin, cout) in enumerate(ARCH)]

    def pack(self, stream=None):
        """Both bf16 copies of every layer from the FP32 masters (the masters'
        layout is the model layout of yoro_model.h), in one launch."""
        _ok(nnlib().yoro_model_pack_train(_p(self.master), _p(self.wf), _p(self.wb), yoro._stream(stream)))

    def buffers(self, n, h, w, train=False) -> Buffers:
        key = (n, h, w, train)
        if key not in self._bufs:
            self._bufs[key] = Buffers(n, h, w, self.device, train)
        return self._bufs[key]

    # ------------------------------------------------------------ layers --
    def _conv(self, i, x, ldx, lev, b, cin, y, ldy, epi, y_fp32=False, cout_store=None, backward=False, msrc=None,
              ldm=0, s=None):
        """Layer i forward (or its input gradient when backward=True)."""
        _, cout_p, cin_p = self.shapes[i]
        o = int(self.offsets[i])
        if backward:  # input gradient: conv of dy (cout_p channels) with the flipped copy -> cin_p channels
            cin_k, cout_k, wgt = cout_p, cin_p, _p(self.wb, o)
        else:
            cin_k, cout_k, wgt = cin_p, cout_p, _p(self.wf, o)
        store = cout_k if cout_store is None else cout_store
        _ok(nnlib().yoro_nn_conv3x3(x, ldx, b.n, b.h >> lev, b.w >> lev, cin_k, wgt, cout_k, y, ldy,
                                    1 if y_fp32 else 0, store, epi, msrc, ldm, s))

    def _wgrad(self, i, x, ldx, dy, lddy, lev, b, s):
        _, cout_p, cin_p = self.shapes[i]
        o = int(self.offsets[i])
        _ok(nnlib().yoro_nn_conv3x3_wgrad(x, ldx, dy, lddy, b.n, b.h >> lev, b.w >> lev, cin_p, cout_p,
                                          _p(self.grad, o), _p(b.wgrad_ws), b.wgrad_ws.numel() * 4, s))

    # ----------------------------------------------------------- forward --
    def forward(self, rgba, depth, mask, b: Buffers, stream=None):
        """rgba [n, h, w, 4] u8, depth [n, h, w] f32, mask [n, h, w] u8 (the plain
        fill); leaves the residual in b.res ([n*h*w, 3] FP32)."""
        L, s = nnlib(), yoro._stream(stream)
        P0 = b.P[0]
        _ok(L.yoro_nn_input(_p(rgba), _p(depth), _p(mask), P0, _p(b.x0), s))
        R = EPI_RELU
        self._conv(0, _p(b.x0), 32, 0, b, 32, _p(b.e0a), 32, R, s=s)
        self._conv(1, _p(b.e0a), 32, 0, b, 32, _p(b.c0, 32), 64, R, s=s)              # e0b -> c0[:, 32:]
        _ok(L.yoro_nn_avgpool2(_p(b.c0, 32), 64, b.n, b.h, b.w, 32, _p(b.p1), 32, s))
        self._conv(2, _p(b.p1), 32, 1, b, 32, _p(b.e1a), 64, R, s=s)
        self._conv(3, _p(b.e1a), 64, 1, b, 64, _p(b.c1, 64), 128, R, s=s)             # e1b -> c1[:, 64:]
        _ok(L.yoro_nn_avgpool2(_p(b.c1, 64), 128, b.n, b.h >> 1, b.w >> 1, 64, _p(b.p2), 64, s))
        self._conv(4, _p(b.p2), 64, 2, b, 64, _p(b.e2a), 128, R, s=s)
        self._conv(5, _p(b.e2a), 128, 2, b, 128, _p(b.c2, 128), 256, R, s=s)          # e2b -> c2[:, 128:]
        _ok(L.yoro_nn_avgpool2(_p(b.c2, 128), 256, b.n, b.h >> 2, b.w >> 2, 128, _p(b.p3), 128, s))
        self._conv(6, _p(b.p3), 128, 3, b, 128, _p(b.e3a), 256, R, s=s)
        self._conv(7, _p(b.e3a), 256, 3, b, 256, _p(b.e3b), 256, R, s=s)
        _ok(L.yoro_nn_upsample2(_p(b.e3b), 256, b.n, b.h >> 3, b.w >> 3, 256, _p(b.u2), 256, s))
        self._conv(8, _p(b.u2), 256, 2, b, 256, _p(b.c2), 256, R, s=s)                # d2a -> c2[:, :128]
        self._conv(9, _p(b.c2), 256, 2, b, 256, _p(b.d2b), 128, R, s=s)
        self._conv(10, _p(b.d2b), 128, 2, b, 128, _p(b.d2c), 128, R, s=s)
        _ok(L.yoro_nn_upsample2(_p(b.d2c), 128, b.n, b.h >> 2, b.w >> 2, 128, _p(b.u1), 128, s))
        self._conv(11, _p(b.u1), 128, 1, b, 128, _p(b.c1), 128, R, s=s)               # d1a -> c1[:, :64]
        self._conv(12, _p(b.c1), 128, 1, b, 128, _p(b.d1b), 64, R, s=s)
        self._conv(13, _p(b.d1b), 64, 1, b, 64, _p(b.d1c), 64, R, s=s)
        _ok(L.yoro_nn_upsample2(_p(b.d1c), 64, b.n, b.h >> 1, b.w >> 1, 64, _p(b.u0), 64, s))
        self._conv(14, _p(b.u0), 64, 0, b, 64, _p(b.c0), 64, R, s=s)                  # d0a -> c0[:, :32]
        self._conv(15, _p(b.c0), 64, 0, b, 64, _p(b.d0b), 32, R, s=s)
        self._conv(16, _p(b.d0b), 32, 0, b, 32, _p(b.d0c), 32, R, s=s)
        self._conv(17, _p(b.d0c), 32, 0, b, 32, _p(b.res), 3, EPI_NONE, y_fp32=True, cout_store=3, s=s)

    # ---------------------------------------------------------- backward --
    def backward(self, rgba, mask, target, b: Buffers, stream=None):
        """Loss (into b.loss) and every weight gradient (into self.grad)."""
        L, s = nnlib(), yoro._stream(stream)
        G = EPI_RELU_GRAD
        _ok(L.yoro_nn_l1_grad(_p(b.res), _p(rgba), _p(mask), _p(target), b.P[0], _p(b.g_res), _p(b.loss),
                              _p(b.l1_ws), s))
        self._wgrad(17, _p(b.d0c), 32, _p(b.g_res), 32, 0, b, s)
        self._conv(17, _p(b.g_res), 32, 0, b, 32, _p(b.g_d0c), 32, G, backward=True, msrc=_p(b.d0c), ldm=32, s=s)
        self._wgrad(16, _p(b.d0b), 32, _p(b.g_d0c), 32, 0, b, s)
        self._conv(16, _p(b.g_d0c), 32, 0, b, 32, _p(b.g_d0b), 32, G, backward=True, msrc=_p(b.d0b), ldm=32, s=s)
        self._wgrad(15, _p(b.c0), 64, _p(b.g_d0b), 32, 0, b, s)
        self._conv(15, _p(b.g_d0b), 32, 0, b, 32, _p(b.g_c0), 64, G, backward=True, msrc=_p(b.c0), ldm=64, s=s)
        self._wgrad(14, _p(b.u0), 64, _p(b.g_c0), 64, 0, b, s)
        self._conv(14, _p(b.g_c0), 64, 0, b, 32, _p(b.g_u0), 64, G, backward=True, msrc=_p(b.u0), ldm=64, s=s)
        _ok(L.yoro_nn_upsample2_grad(_p(b.g_u0), 64, b.n, b.h >> 1, b.w >> 1, 64, _p(b.g_d1c), 64, s))
        self._wgrad(13, _p(b.d1b), 64, _p(b.g_d1c), 64, 1, b, s)
        self._conv(13, _p(b.g_d1c), 64, 1, b, 64, _p(b.g_d1b), 64, G, backward=True, msrc=_p(b.d1b), ldm=64, s=s)
        self._wgrad(12, _p(b.c1), 128, _p(b.g_d1b), 64, 1, b, s)
        self._conv(12, _p(b.g_d1b), 64, 1, b, 64, _p(b.g_c1), 128, G, backward=True, msrc=_p(b.c1), ldm=128, s=s)
        self._wgrad(11, _p(b.u1), 128, _p(b.g_c1), 128, 1, b, s)
        self._conv(11, _p(b.g_c1), 128, 1, b, 64, _p(b.g_u1), 128, G, backward=True, msrc=_p(b.u1), ldm=128, s=s)
        _ok(L.yoro_nn_upsample2_grad(_p(b.g_u1), 128, b.n, b.h >> 2, b.w >> 2, 128, _p(b.g_d2c), 128, s))
        self._wgrad(10, _p(b.d2b), 128, _p(b.g_d2c), 128, 2, b, s)
        self._conv(10, _p(b.g_d2c), 128, 2, b, 128, _p(b.g_d2b), 128, G, backward=True, msrc=_p(b.d2b), ldm=128, s=s)
        self._wgrad(9, _p(b.c2), 256, _p(b.g_d2b), 128, 2, b, s)
        self._conv(9, _p(b.g_d2b), 128, 2, b, 128, _p(b.g_c2), 256, G, backward=True, msrc=_p(b.c2), ldm=256, s=s)
        self._wgrad(8, _p(b.u2), 256, _p(b.g_c2), 256, 2, b, s)
        self._conv(8, _p(b.g_c2), 256, 2, b, 128, _p(b.g_u2), 256, G, backward=True, msrc=_p(b.u2), ldm=256, s=s)
        _ok(L.yoro_nn_upsample2_grad(_p(b.g_u2), 256, b.n, b.h >> 3, b.w >> 3, 256, _p(b.g_e3b), 256, s))
        self._wgrad(7, _p(b.e3a), 256, _p(b.g_e3b), 256, 3, b, s)
        self._conv(7, _p(b.g_e3b), 256, 3, b, 256, _p(b.g_e3a), 256, G, backward=True, msrc=_p(b.e3a), ldm=256, s=s)
        self._wgrad(6, _p(b.p3), 128, _p(b.g_e3a), 256, 3, b, s)
        self._conv(6, _p(b.g_e3a), 256, 3, b, 256, _p(b.g_p3), 128, EPI_NONE, backward=True, s=s)
        _ok(L.yoro_nn_avgpool2_grad(_p(b.g_p3), 128, _p(b.g_c2, 128), 256, _p(b.c2, 128), 256, b.n, b.h >> 2,
                                    b.w >> 2, 128, _p(b.g_e2b), 128, s))
        self._wgrad(5, _p(b.e2a), 128, _p(b.g_e2b), 128, 2, b, s)
        self._conv(5, _p(b.g_e2b), 128, 2, b, 128, _p(b.g_e2a), 128, G, backward=True, msrc=_p(b.e2a), ldm=128, s=s)
        self._wgrad(4, _p(b.p2), 64, _p(b.g_e2a), 128, 2, b, s)
        self._conv(4, _p(b.g_e2a), 128, 2, b, 128, _p(b.g_p2), 64, EPI_NONE, backward=True, s=s)
        _ok(L.yoro_nn_avgpool2_grad(_p(b.g_p2), 64, _p(b.g_c1, 64), 128, _p(b.c1, 64), 128, b.n, b.h >> 1, b.w >> 1,
                                    64, _p(b.g_e1b), 64, s))
        self._wgrad(3, _p(b.e1a), 64, _p(b.g_e1b), 64, 1, b, s)
        self._conv(3, _p(b.g_e1b), 64, 1, b, 64, _p(b.g_e1a), 64, G, backward=True, msrc=_p(b.e1a), ldm=64, s=s)
        self._wgrad(2, _p(b.p1), 32, _p(b.g_e1a), 64, 1, b, s)
        self._conv(2, _p(b.g_e1a), 64, 1, b, 64, _p(b.g_p1), 32, EPI_NONE, backward=True, s=s)
        _ok(L.yoro_nn_avgpool2_grad(_p(b.g_p1), 32, _p(b.g_c0, 32), 64, _p(b.c0, 32), 64, b.n, b.h, b.w, 32,
                                    _p(b.g_e0b), 32, s))
        self._wgrad(1, _p(b.e0a), 32, _p(b.g_e0b), 32, 0, b, s)
        self._conv(1, _p(b.g_e0b), 32, 0, b, 32, _p(b.g_e0a), 32, G, backward=True, msrc=_p(b.e0a), ldm=32, s=s)
        self._wgrad(0, _p(b.x0), 32, _p(b.g_e0a), 32, 0, b, s)

    def adamw(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wd=0.01, stream=None):
        self.step += 1
        s = yoro._stream(stream)
        _ok(nnlib().yoro_nn_adamw(_p(self.master), _p(self.m), _p(self.v), _p(self.grad), self.master.numel(),
                                  lr, b1, b2, eps, wd, self.step, s))
        self.pack(stream)

    def train_step(self, rgba, depth, mask, target, lr=1e-3, stream=None):
        n, h, w = depth.shape
        b = self.buffers(n, h, w, train=True)
        self.forward(rgba, depth, mask, b, stream)
        self.backward(rgba, mask, target, b, stream)
        self.adamw(lr=lr, stream=stream)
        return b.loss

    def composite(self, rgba, mask, b: Buffers, out, stream=None):
        _ok(nnlib().yoro_nn_composite(_p(b.res), _p(rgba), _p(mask), b.P[0], _p(out), yoro._stream(stream)))
        return out

    def fill(self, rgba, depth, mask, out=None, stream=None):
        """Learned fill of n plain-filled frames: hole pixels replaced."""
        n, h, w = depth.shape
        b = self.buffers(n, h, w, train=False)
        self.forward(rgba, depth, mask, b, stream)
        if out is None:
            out = torch.empty_like(rgba)
        return self.composite(rgba, mask, b, out, stream)

    def tile_holes(self, mask, tile: int = TILE, stream=None):
        """Device u32 hole count per tile x tile block of one frame's mask."""
        h, w = mask.shape
        counts = torch.empty(((w + tile - 1) // tile) * ((h + tile - 1) // tile), dtype=torch.int32,
                             device=mask.device)
        _ok(nnlib().yoro_nn_tile_holes(_p(mask), w, h, tile, _p(counts), yoro._stream(stream)))
        return counts

    def fill_tiles(self, rgba, depth, mask, out=None, tile: int = TILE, halo: int = HALO, chunk: int = 32,
                   stream=None):
        """Learned fill of one plain-filled frame (rgba [h, w, 4], depth and
        mask [h, w]) that runs the network only on tile x tile blocks with a
        hole, each inside a crop reaching `halo` pixels around it
        (yoro_model_fill_tiles).  With halo >= boundary_reach() the result
        equals fill() on the whole frame.  Reads the block hole counts back to
        the host to plan the crops.  Returns (out, crops run)."""
        h, w = depth.shape
        if out is None:
            out = torch.empty_like(rgba)
        if out.data_ptr() != rgba.data_ptr():
            out.copy_(rgba)
        plan = tile_plan(self.tile_holes(mask, tile, stream).cpu().numpy(), h, w, tile, halo)
        k = plan.shape[0]
        if k == 0:
            return out, 0
        L = nnlib()
        plan_d = torch.from_numpy(plan).to(self.device)
        nbytes = L.yoro_model_tiles_workspace_bytes(k, chunk, tile, halo)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        _ok(L.yoro_model_fill_tiles(_p(self.wf), _p(rgba), _p(depth), _p(mask), w, h, _p(plan_d), k, tile, halo, chunk,
                                    _p(out), _p(ws), nbytes, yoro._stream(stream)))
        return out, k

    def fill_bands(self, rgba, depth, mask, out=None, band: int = 256, halo: int = HALO, band_has_holes=None,
                   stream=None):
        """Learned fill of one frame in full-width bands (yoro_model_fill_bands);
        equal to fill_native bit for bit with halo >= boundary_reach()."""
        h, w = depth.shape
        L = nnlib()
        if out is None:
            out = rgba.clone()
        nbytes = L.yoro_model_bands_workspace_bytes(w, h, band, halo)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        flags = None
        if band_has_holes is not None:
            flags = np.ascontiguousarray(band_has_holes, dtype=np.uint8)
        _ok(L.yoro_model_fill_bands(_p(self.wf), _p(rgba), _p(depth), _p(mask), w, h, band, halo,
                                    None if flags is None else flags.ctypes.data, _p(out), _p(ws), nbytes,
                                    yoro._stream(stream)))
        return out

    def fill_native(self, rgba, depth, mask, out=None, stream=None):
        """fill() through the library's own forward sequence (yoro_model_fill)."""
        n, h, w = depth.shape
        L = nnlib()
        if out is None:
            out = torch.empty_like(rgba)
        nbytes = L.yoro_model_workspace_bytes(n, h, w)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        _ok(L.yoro_model_fill(_p(self.wf), _p(rgba), _p(depth), _p(mask), n, h, w, _p(out), _p(ws), nbytes,
                              yoro._stream(stream)))
        return out

    # ----------------------------------------------------- checkpointing --
    def state_dict(self):
        return {"master": self.master.cpu(), "m": self.m.cpu(), "v": self.v.cpu(), "step": self.step}

    def load_state_dict(self, st):
        self.master.copy_(st["master"].to(self.device))
        self.m.copy_(st["m"].to(self.device))
        self.v.copy_(st["v"].to(self.device))
        self.step = int(st["step"])
        self.pack()


def init_params(seed: int = 0):
    """He-normal weights (std sqrt(2 / (9 cin))) for the ReLU layers; the head
    starts at 1 % of that, so the untrained network is close to the plain fill."""
    rng = np.random.default_rng(seed)
    out = []
    for name, cin, cout in ARCH:
        std = np.sqrt(2.0 / (9 * cin)) * (0.01 if name == "head" else 1.0)
        out.append(rng.normal(0.0, std, size=(9, cout, cin)).astype(np.float32))
    return out
