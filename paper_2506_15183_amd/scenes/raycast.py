"""ctypes wrapper over the C ray-caster in ``raycast.c``.

The shared library ``libyoro_scene.so`` is built next to this file by the
package build step (gcc, OpenMP, FP64 geometry).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libyoro_scene.so")

SPHERE, BOX = 0, 1
BACKGROUND_DEPTH = 1.0e6


class _Obj(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("id", ctypes.c_uint32),
        ("c", ctypes.c_double * 3),
        ("h", ctypes.c_double * 3),
        ("texel", ctypes.c_double),
        ("cell", ctypes.c_double),
        ("rgb", ctypes.c_int32 * 3),
        ("noise", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"scene generator library missing: {LIB_PATH}; run __graft_entry__.build() first"
            )
        L = ctypes.CDLL(LIB_PATH)
        L.ys_generate.restype = ctypes.c_int
        L.ys_generate.argtypes = [
            ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
            ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
            ctypes.c_int32, ctypes.POINTER(_Obj),
        ]
        L.ys_render.restype = None
        L.ys_render.argtypes = [
            ctypes.POINTER(_Obj), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
            ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_uint64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_int32,
        ]
        L.ys_hash64.restype = ctypes.c_uint64
        L.ys_hash64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.ys_uniform_fill.restype = None
        L.ys_uniform_fill.argtypes = [ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int64]
        _lib = L
    return _lib


def hash64(a: int, b: int) -> int:
    return int(lib().ys_hash64(a & 0xFFFFFFFFFFFFFFFF, b & 0xFFFFFFFFFFFFFFFF))


def uniforms(seed: int, n: int) -> np.ndarray:
    """n doubles in [0, 1) from xoshiro256** seeded through SplitMix64."""
    out = np.empty(n, dtype=np.float64)
    lib().ys_uniform_fill(seed & 0xFFFFFFFFFFFFFFFF, out.ctypes.data, n)
    return out


@dataclass
class Scene:
    """A seeded set of boxes and spheres in left-eye camera coordinates."""

    objects: ctypes.Array
    n: int
    seed: int
    Wv: int  # virtual frame width (pixels)
    Hv: int  # virtual frame height (pixels)
    f: float  # focal length (pixels)


def make_scene(seed: int, Wv: int, Hv: int, f: float, n_objects: int, zmin: float, zmax: float,
               log_uniform: bool, checker=(0, 0), noise: int = 16) -> Scene:
    objs = (_Obj * max(n_objects, 1))()
    lib().ys_generate(seed & 0xFFFFFFFFFFFFFFFF, Wv, Hv, f, n_objects, zmin, zmax,
                      1 if log_uniform else 0, int(checker[0]), int(checker[1]), noise, objs)
    return Scene(objs, n_objects, seed, Wv, Hv, f)


def render(scene: Scene, eye_x: float, W: int | None = None, H: int | None = None, x_off: int = 0,
           y_off: int = 0, nthreads: int = 0, out_rgba=None, out_depth=None):
    """Ray-cast one eye at (eye_x, 0, 0).

    Returns (rgba uint8 [H, W, 4], depth float32 [H, W]) for the window of the
    virtual frame that starts at (x_off, y_off).  Principal point: the centre
    of the virtual frame.
    """
    W = scene.Wv if W is None else W
    H = scene.Hv if H is None else H
    rgba = np.empty((H, W, 4), dtype=np.uint8) if out_rgba is None else out_rgba
    depth = np.empty((H, W), dtype=np.float32) if out_depth is None else out_depth
    assert rgba.shape == (H, W, 4) and rgba.dtype == np.uint8 and rgba.flags.c_contiguous
    assert depth.shape == (H, W) and depth.dtype == np.float32 and depth.flags.c_contiguous
    lib().ys_render(scene.objects, scene.n, W, H, x_off, y_off, scene.f, 0.5 * scene.Wv,
                    0.5 * scene.Hv, float(eye_x), scene.seed & 0xFFFFFFFFFFFFFFFF, scene.Hv,
                    BACKGROUND_DEPTH, rgba.ctypes.data, depth.ctypes.data, nthreads)
    return rgba, depth


def render_near(scene: Scene, eye_x: float, near_m: float, W: int | None = None, H: int | None = None,
                x_off: int = 0, y_off: int = 0, nthreads: int = 0):
    """The near field of one eye, as a conventional renderer would draw it for
    the near-object hybrid: every pixel whose nearest surface lies closer
    than near_m (its FP32 depth below near_m) gets that surface's colour and
    depth; every other pixel RGBA 0 and depth +inf."""
    W = scene.Wv if W is None else W
    H = scene.Hv if H is None else H
    rgba = np.empty((H, W, 4), dtype=np.uint8)
    depth = np.empty((H, W), dtype=np.float32)
    near = float(np.float32(near_m))
    lib().ys_render(scene.objects, scene.n, W, H, x_off, y_off, scene.f, 0.5 * scene.Wv,
                    0.5 * scene.Hv, float(eye_x), scene.seed & 0xFFFFFFFFFFFFFFFF, scene.Hv,
                    near, rgba.ctypes.data, depth.ctypes.data, nthreads)
    miss = ~(depth < np.float32(near))
    rgba[miss] = 0
    depth[miss] = np.inf
    return rgba, depth


def render_pair(scene: Scene, baseline_m: float, **kw):
    """(left rgba, left depth, right rgba, right depth); right eye at +baseline."""
    l_rgba, l_depth = render(scene, 0.0, **kw)
    r_rgba, r_depth = render(scene, baseline_m, **kw)
    return l_rgba, l_depth, r_rgba, r_depth


def scene_from_objects(objects, Wv: int, Hv: int, f: float, seed: int = 0) -> Scene:
    """A scene from explicit objects: dicts with kind, c, h, texel, cell, rgb, noise."""
    arr = (_Obj * max(len(objects), 1))()
    for i, o in enumerate(objects):
        arr[i].kind = int(o.get("kind", BOX))
        arr[i].id = int(o.get("id", i + 1))
        for k in range(3):
            arr[i].c[k] = float(o["c"][k])
            arr[i].h[k] = float(o["h"][k])
            arr[i].rgb[k] = int(o.get("rgb", (128, 128, 128))[k])
        arr[i].texel = float(o.get("texel", 1.0))
        arr[i].cell = float(o.get("cell", 0.0))
        arr[i].noise = int(o.get("noise", 16))
    return Scene(arr, len(objects), seed, Wv, Hv, f)
