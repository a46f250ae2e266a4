"""ORACLE -- test infrastructure only.  numpy wrapper over ``reproject.c``.

The C file carries the statement of what is computed and the passages it
follows (Section 5 O1/O2, Section 6 reprojection equation and Algorithms 1-2,
Section 7 Algorithm 3 and the Patcher figure, Section 9 PSNR).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "reproject.c")
LIB = os.path.join(_HERE, "liboracle_reproject.so")

TARGET_RIGHT, TARGET_LEFT = 0, 1
FILL_NONE, FILL_NEAREST_BG, FILL_PATCHER, FILL_SIDE_ONLY = 0, 1, 3, 101

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"])
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        L.oracle_reproject.restype = ctypes.c_int
        L.oracle_reproject.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_float, ctypes.c_float, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
        L.oracle_reproject_lowres.restype = ctypes.c_int
        L.oracle_reproject_lowres.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_float, ctypes.c_float, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]
        L.oracle_reproject_pose.restype = ctypes.c_int
        L.oracle_reproject_pose.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]
        L.oracle_project_pose.restype = ctypes.c_int
        L.oracle_project_pose.argtypes = [ctypes.c_float, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float)]
        L.oracle_reproject_hybrid.restype = ctypes.c_int
        L.oracle_reproject_hybrid.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_float, ctypes.c_float, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
        L.oracle_fill_holes.restype = ctypes.c_int
        L.oracle_fill_holes.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.oracle_disparity.restype = ctypes.c_int
        L.oracle_disparity.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32)]
        L.oracle_hole_sse.restype = None
        L.oracle_hole_sse.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
        _lib = L
    return _lib


def disparity(z: float, baseline_m: float, focal_px: float, width: int):
    """Rounded disparity of one depth, or None when the pixel is not splatted."""
    bf = np.float32(np.float32(baseline_m) * np.float32(focal_px))
    d = ctypes.c_int32(0)
    rc = lib().oracle_disparity(float(np.float32(z)), float(bf), width, ctypes.byref(d))
    return None if rc != 0 else int(d.value)


def reproject(src_rgba: np.ndarray, src_depth: np.ndarray, baseline_m: float, focal_px: float,
              target_eye: int = TARGET_RIGHT, fill_mode: int = FILL_NEAREST_BG, nthreads: int = 1):
    """(dst_rgba [H,W,4] u8, dst_depth [H,W] f32, dst_mask [H,W] u8)."""
    src_rgba = np.ascontiguousarray(src_rgba, dtype=np.uint8)
    src_depth = np.ascontiguousarray(src_depth, dtype=np.float32)
    H, W = src_depth.shape
    assert src_rgba.shape == (H, W, 4)
    dst = np.empty_like(src_rgba)
    dz = np.empty_like(src_depth)
    mk = np.empty((H, W), dtype=np.uint8)
    rc = lib().oracle_reproject(src_rgba.ctypes.data, src_depth.ctypes.data, W, H,
                                float(np.float32(baseline_m)), float(np.float32(focal_px)),
                                target_eye, fill_mode, dst.ctypes.data, dz.ctypes.data, mk.ctypes.data,
                                nthreads)
    if rc != 0:
        raise ValueError("oracle_reproject: bad arguments")
    return dst, dz, mk


def reproject_lowres(src_rgba: np.ndarray, src_depth: np.ndarray, baseline_m: float, focal_px: float,
                     target_eye: int = TARGET_RIGHT, fill_mode: int = FILL_NEAREST_BG, scale: int = 4,
                     linear: bool = True):
    """Reprojection through a 1/scale intermediate buffer (Section 6 (c), (d)):
    (dst_rgba [H,W,4] u8, dst_depth [H,W] f32, dst_mask [H,W] u8)."""
    src_rgba = np.ascontiguousarray(src_rgba, dtype=np.uint8)
    src_depth = np.ascontiguousarray(src_depth, dtype=np.float32)
    H, W = src_depth.shape
    assert src_rgba.shape == (H, W, 4)
    dst = np.empty_like(src_rgba)
    dz = np.empty_like(src_depth)
    mk = np.empty((H, W), dtype=np.uint8)
    rc = lib().oracle_reproject_lowres(src_rgba.ctypes.data, src_depth.ctypes.data, W, H,
                                       float(np.float32(baseline_m)), float(np.float32(focal_px)), target_eye,
                                       fill_mode, int(scale), int(bool(linear)), dst.ctypes.data, dz.ctypes.data,
                                       mk.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_reproject_lowres: bad arguments")
    return dst, dz, mk


def _pose_arrays(q, t):
    q = np.ascontiguousarray(q, dtype=np.float32).reshape(4)
    t = np.ascontiguousarray(t, dtype=np.float32).reshape(3)
    return q, t


def reproject_pose(src_rgba: np.ndarray, src_depth: np.ndarray, focal_px: float, cx: float, cy: float, q, t,
                   fill_mode: int = FILL_NEAREST_BG):
    """Reprojection to an eye at pose (q = (r_x scalar, r_y, r_z, r_w), t) in the
    source eye's camera frame (Section 6): (dst_rgba, dst_depth, dst_mask)."""
    src_rgba = np.ascontiguousarray(src_rgba, dtype=np.uint8)
    src_depth = np.ascontiguousarray(src_depth, dtype=np.float32)
    H, W = src_depth.shape
    assert src_rgba.shape == (H, W, 4)
    q, t = _pose_arrays(q, t)
    dst = np.empty_like(src_rgba)
    dz = np.empty_like(src_depth)
    mk = np.empty((H, W), dtype=np.uint8)
    rc = lib().oracle_reproject_pose(src_rgba.ctypes.data, src_depth.ctypes.data, W, H, float(np.float32(focal_px)),
                                     float(np.float32(cx)), float(np.float32(cy)), q.ctypes.data, t.ctypes.data,
                                     fill_mode, dst.ctypes.data, dz.ctypes.data, mk.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_reproject_pose: bad arguments")
    return dst, dz, mk


def project_pose(z: float, x: int, y: int, width: int, height: int, focal_px: float, cx: float, cy: float, q, t):
    """(target x, target y, target depth) of one source pixel, or None when it is not splatted."""
    q, t = _pose_arrays(q, t)
    xt, yt, zt = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_float(0)
    rc = lib().oracle_project_pose(float(np.float32(z)), x, y, width, height, float(np.float32(focal_px)),
                                   float(np.float32(cx)), float(np.float32(cy)), q.ctypes.data, t.ctypes.data,
                                   ctypes.byref(xt), ctypes.byref(yt), ctypes.byref(zt))
    return None if rc != 0 else (int(xt.value), int(yt.value), float(np.float32(zt.value)))


MASK_NEAR = 3  # hybrid: the pixel comes from the near layer


def reproject_hybrid(src_rgba: np.ndarray, src_depth: np.ndarray, baseline_m: float, focal_px: float,
                     target_eye: int, fill_mode: int, near_m: float, near_rgba: np.ndarray, near_depth: np.ndarray,
                     nthreads: int = 0):
    """Near-object hybrid (Section 11.4): the far field (source depth >=
    near_m) warped and filled, the target eye's near layer over it where its
    depth is below near_m.  (dst_rgba, dst_depth, dst_mask)."""
    src_rgba = np.ascontiguousarray(src_rgba, dtype=np.uint8)
    src_depth = np.ascontiguousarray(src_depth, dtype=np.float32)
    near_rgba = np.ascontiguousarray(near_rgba, dtype=np.uint8)
    near_depth = np.ascontiguousarray(near_depth, dtype=np.float32)
    H, W = src_depth.shape
    assert src_rgba.shape == (H, W, 4) and near_rgba.shape == (H, W, 4) and near_depth.shape == (H, W)
    dst = np.empty_like(src_rgba)
    dz = np.empty_like(src_depth)
    mk = np.empty((H, W), dtype=np.uint8)
    rc = lib().oracle_reproject_hybrid(src_rgba.ctypes.data, src_depth.ctypes.data, W, H,
                                       float(np.float32(baseline_m)), float(np.float32(focal_px)), target_eye,
                                       fill_mode, float(np.float32(near_m)), near_rgba.ctypes.data,
                                       near_depth.ctypes.data, dst.ctypes.data, dz.ctypes.data, mk.ctypes.data,
                                       nthreads)
    if rc != 0:
        raise ValueError("oracle_reproject_hybrid: bad arguments")
    return dst, dz, mk


def fill_holes(rgba: np.ndarray, depth: np.ndarray, mask: np.ndarray, target_eye: int = TARGET_RIGHT,
               fill_mode: int = FILL_NEAREST_BG):
    """Copies of (rgba, depth, mask) with holes (mask != 0) refilled from hits."""
    rgba = np.ascontiguousarray(rgba, dtype=np.uint8).copy()
    depth = np.ascontiguousarray(depth, dtype=np.float32).copy()
    mask = np.ascontiguousarray(mask, dtype=np.uint8).copy()
    H, W = depth.shape
    rc = lib().oracle_fill_holes(rgba.ctypes.data, depth.ctypes.data, mask.ctypes.data, W, H, target_eye,
                                 fill_mode)
    if rc != 0:
        raise ValueError("oracle_fill_holes: bad arguments")
    return rgba, depth, mask


def hole_sse(rgba: np.ndarray, ref: np.ndarray, mask: np.ndarray | None):
    """(sum of squared RGB errors over mask != 0 pixels, pixel count)."""
    rgba = np.ascontiguousarray(rgba, dtype=np.uint8)
    ref = np.ascontiguousarray(ref, dtype=np.uint8)
    n = rgba.shape[0] * rgba.shape[1]
    sse, cnt = ctypes.c_uint64(0), ctypes.c_uint64(0)
    mp = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).ctypes.data
    lib().oracle_hole_sse(rgba.ctypes.data, ref.ctypes.data, mp, n, ctypes.byref(sse), ctypes.byref(cnt))
    return int(sse.value), int(cnt.value)


def psnr_from_sse(sse: int, count_pixels: int, peak: float = 255.0) -> float:
    """PSNR = 10 log10(peak^2 / MSE) over RGB (Section 9, PSNR); MSE 0 gives +inf."""
    if count_pixels == 0:
        return float("nan")
    mse = sse / (3.0 * count_pixels)
    if mse == 0:
        return float("inf")
    return 10.0 * np.log10(peak * peak / mse)
