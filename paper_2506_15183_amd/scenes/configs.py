"""Workload recipes: seeded scenes shaped like VR frames.

The paper's Unity scenes and image dataset are not available; these seeded,
analytically ray-cast scenes stand in for them.  Each recipe fixes the frame
size, the object count and depth distribution, the stereo baseline B
(metres) and the focal length f (pixels), the two parameters of the
disparity (Section 6, reprojection equation, reduced to parallel stereo).

* ``config1_frame``: one 256 x 256 frame, 8 objects, centre depth U[0.5, 20] m,
  B = 0.064 m, f = 200 px, source = left eye, target = right eye.
* ``config2_frame``: one 1832 x 1920 frame (a Quest 2 eye, Section 12), 200
  objects, centre depth log-uniform on [0.3, 50] m, object-space checker of
  cell U{4..32} px at the object's depth, B = 0.063 m, f = 900 px.
* ``config3_frames``: 64 frames, 16 each of 1024x1024, 1440x1600, 1832x1920
  and 2160x2160 (width x height), each with its own scene of U{50..300}
  objects (depth log-uniform on [0.3, 50] m, checker as above),
  B ~ U[0.055, 0.072] m, f ~ U[600, 1100] px.
* ``training_window``: a 256 x 256 window of a virtual 1832 x 1920 frame with
  a 50..300-object scene (B, f drawn as in config 3); the source eye is
  rendered with an extra margin on the side the sources come from, so the
  window has no artificial border band of holes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import raycast

TARGET_RIGHT, TARGET_LEFT = 0, 1


def frame_seed(config_id: int, frame_id: int) -> int:
    return raycast.hash64(0x59_4F_52_4F_0000_0000 | config_id, frame_id)


@dataclass
class FrameSpec:
    width: int
    height: int
    baseline_m: float
    focal_px: float
    target_eye: int
    n_objects: int
    zmin: float
    zmax: float
    log_uniform: bool
    checker: tuple
    seed: int

    def scene(self) -> raycast.Scene:
        return raycast.make_scene(self.seed, self.width, self.height, self.focal_px, self.n_objects,
                                  self.zmin, self.zmax, self.log_uniform, self.checker)

    def source_eye_x(self) -> float:
        return 0.0 if self.target_eye == TARGET_RIGHT else self.baseline_m

    def target_eye_x(self) -> float:
        return self.baseline_m if self.target_eye == TARGET_RIGHT else 0.0

    def render_source(self, nthreads: int = 0, out_rgba=None, out_depth=None):
        return raycast.render(self.scene(), self.source_eye_x(), nthreads=nthreads,
                              out_rgba=out_rgba, out_depth=out_depth)

    def render_target(self, nthreads: int = 0):
        return raycast.render(self.scene(), self.target_eye_x(), nthreads=nthreads)

    @property
    def pixels(self) -> int:
        return self.width * self.height


def config1_frame(frame_id: int = 0) -> FrameSpec:
    return FrameSpec(256, 256, 0.064, 200.0, TARGET_RIGHT, 8, 0.5, 20.0, False, (0, 0),
                     frame_seed(1, frame_id))


def config2_frame(frame_id: int = 0) -> FrameSpec:
    return FrameSpec(1832, 1920, 0.063, 900.0, TARGET_RIGHT, 200, 0.3, 50.0, True, (4, 32),
                     frame_seed(2, frame_id))


CONFIG3_SIZES = ((1024, 1024), (1440, 1600), (1832, 1920), (2160, 2160))


def config3_frames(n_per_size: int = 16) -> list[FrameSpec]:
    """The 64-frame mixed-resolution batch (frames interleaved by size)."""
    specs = []
    k = 0
    for rep in range(n_per_size):
        for (w, h) in CONFIG3_SIZES:
            u = raycast.uniforms(frame_seed(3, 1_000_000 + k), 3)
            B = 0.055 + (0.072 - 0.055) * float(u[0])
            f = 600.0 + (1100.0 - 600.0) * float(u[1])
            n = 50 + int(u[2] * 251)
            specs.append(FrameSpec(w, h, B, f, TARGET_RIGHT, n, 0.3, 50.0, True, (4, 32),
                                   frame_seed(3, k)))
            k += 1
    return specs


@dataclass
class TrainingWindow:
    """A window of a virtual frame plus the source-side margin it needs."""

    spec: FrameSpec  # the virtual frame (scene, B, f)
    x_off: int
    y_off: int
    size: int
    margin: int  # extra source columns on the side sources come from

    def render(self, nthreads: int = 0):
        """(src rgba, src depth) of width size+margin, (true target rgba, depth) of width size."""
        sc = self.spec.scene()
        s = self.size
        if self.spec.target_eye == TARGET_RIGHT:
            src_x0 = self.x_off  # sources lie to the right of their targets
        else:
            src_x0 = self.x_off - self.margin
        src = raycast.render(sc, self.spec.source_eye_x(), W=s + self.margin, H=s, x_off=src_x0,
                             y_off=self.y_off, nthreads=nthreads)
        tgt = raycast.render(sc, self.spec.target_eye_x(), W=s, H=s, x_off=self.x_off,
                             y_off=self.y_off, nthreads=nthreads)
        return src, tgt


def training_window(index: int, split: str = "train", size: int = 256) -> TrainingWindow:
    """Window ``index`` of the training ('train'), validation ('val') or test split."""
    cid = {"train": 4, "val": 40, "test": 41}[split]
    u = raycast.uniforms(frame_seed(cid, 2_000_000 + index), 6)
    W, H = 1832, 1920
    B = 0.055 + (0.072 - 0.055) * float(u[0])
    f = 600.0 + (1100.0 - 600.0) * float(u[1])
    n = 50 + int(u[2] * 251)
    spec = FrameSpec(W, H, B, f, TARGET_RIGHT, n, 0.3, 50.0, True, (4, 32), frame_seed(cid, index))
    x_off = int(u[3] * (W - size + 1))
    y_off = int(u[4] * (H - size + 1))
    # Objects are kept at least 0.25 m from the eye plane, so no disparity exceeds B*f/0.25.
    margin = int(math.ceil(B * f / 0.25)) + 2
    return TrainingWindow(spec, x_off, y_off, size, margin)


def render_frames(specs, nthreads: int = 0):
    """Render the source eye of every spec: list of (rgba, depth)."""
    return [s.render_source(nthreads=nthreads) for s in specs]


def as_float32(x) -> np.float32:
    return np.float32(x)


# ------------------------------------------------------------- serving --
SERVE_SIZES = ((1440, 1600), (1832, 1920), (2160, 2160))
SERVE_RATES_HZ = (72.0, 90.0, 120.0)


@dataclass
class HeadsetSpec:
    index: int
    rate_hz: float
    width: int
    height: int
    target_eye: int  # the eye to produce; the headset renders the other (its dominant eye)
    baseline_m: float
    focal_px: float
    phase_s: float   # first frame time, U[0, 1 / rate)


def config5_headsets(n: int = 32, seed: int = 0) -> list[HeadsetSpec]:
    """n headsets with rates and resolutions balanced over their three values
    (seeded assignment), a seeded dominant eye, B ~ U[0.055, 0.072] m and
    f ~ U[600, 1100] px."""
    rng = np.random.default_rng(raycast.hash64(0x5345_5256, seed) & 0xFFFF_FFFF)
    rates = rng.permutation(np.arange(n) % len(SERVE_RATES_HZ))
    sizes = rng.permutation(np.arange(n) % len(SERVE_SIZES))
    out = []
    for i in range(n):
        u = raycast.uniforms(frame_seed(5, 3_000_000 + seed * 4096 + i), 4)
        r = SERVE_RATES_HZ[int(rates[i])]
        w, h = SERVE_SIZES[int(sizes[i])]
        out.append(HeadsetSpec(i, r, w, h, TARGET_RIGHT if u[0] < 0.5 else TARGET_LEFT,
                               0.055 + (0.072 - 0.055) * float(u[1]), 600.0 + (1100.0 - 600.0) * float(u[2]),
                               float(u[3]) / r))
    return out


def config5_pool_frame(width: int, height: int, target_eye: int, slot: int, sparse: bool = False) -> FrameSpec:
    """Pool frame `slot` for headsets of one resolution and eye: a scene of
    U{100..300} objects, depth log-uniform on [0.3, 50] m, checker as config 2,
    rendered with B = 0.063 m and f = 900 px.  sparse: U{20..60} objects at
    depth log-uniform on [2, 50] m (about 2-3 % of pixels are holes, under the
    learned policy's threshold)."""
    key = (SERVE_SIZES.index((width, height)) * 2 + target_eye) * 1024 + slot + (1 << 20 if sparse else 0)
    u = raycast.uniforms(frame_seed(5, 4_000_000 + key), 1)
    if sparse:
        return FrameSpec(width, height, 0.063, 900.0, target_eye, 20 + int(u[0] * 41), 2.0, 50.0, True, (4, 32),
                         frame_seed(5, key))
    n = 100 + int(u[0] * 201)
    return FrameSpec(width, height, 0.063, 900.0, target_eye, n, 0.3, 50.0, True, (4, 32), frame_seed(5, key))


def config4_test_frames(n: int = 16) -> list[FrameSpec]:
    """Held-out full 1832 x 1920 frames for the learned fill (seeds disjoint
    from the training and validation windows); scenes and B, f as config 3."""
    out = []
    for i in range(n):
        u = raycast.uniforms(frame_seed(42, 5_000_000 + i), 3)
        out.append(FrameSpec(1832, 1920, 0.055 + (0.072 - 0.055) * float(u[0]), 600.0 + (1100.0 - 600.0) * float(u[1]),
                             TARGET_RIGHT, 50 + int(u[2] * 251), 0.3, 50.0, True, (4, 32), frame_seed(42, i)))
    return out
