"""Thin Python binding of libyoro.so (include/yoro.h).

Argument marshalling only: torch CUDA tensors in, their device pointers and
torch's current HIP stream out to the C-ABI.  Every step of the method runs
in the library's HIP kernels; there is no CPU fallback, and loading fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libyoro.so")

TARGET_RIGHT, TARGET_LEFT = 0, 1
FILL_NONE, FILL_NEAREST_BG, FILL_LEARNED, FILL_PATCHER = 0, 1, 2, 3
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE_TOO_SMALL, ERR_DEVICE = 0, 1, 2, 3, 4
MAX_WIDTH, MAX_HEIGHT = 8192, 16384
STATIC_MAX_JOBS = 1024  # YORO_STATIC_MAX_JOBS

# Every symbol include/yoro.h declares (the learned-fill layers of
# include/yoro_nn.h are bound in unet.py).
EXPORTS = (
    "yoro_reproject",
    "yoro_reproject_lowres",
    "yoro_reproject_pose_workspace_bytes",
    "yoro_reproject_pose",
    "yoro_fill_holes",
    "yoro_stereo_batch_workspace_bytes",
    "yoro_stereo_batch_prepare",
    "yoro_stereo_batch_launch",
    "yoro_stereo_batch_launch_lowres",
    "yoro_stereo_batch",
    "yoro_stereo_batch_errors",
    "yoro_stereo_batch_static",
    "yoro_hole_sse",
    "yoro_last_error",
    "yoro_version",
)


# include/yoro_measure.h
MEASURE_EXPORTS = ("yoro_measure_stream",)
# include/yoro_hybrid.h
HYBRID_EXPORTS = ("yoro_reproject_hybrid", "yoro_render_near")
MASK_NEAR = 3


class YoroError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"yoro status {status}: {message}")
        self.status = status


class Job(ctypes.Structure):
    """yoro_job."""

    _fields_ = [
        ("src_rgba", ctypes.c_void_p),
        ("src_depth", ctypes.c_void_p),
        ("dst_rgba", ctypes.c_void_p),
        ("dst_depth", ctypes.c_void_p),
        ("dst_mask", ctypes.c_void_p),
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("baseline_m", ctypes.c_float),
        ("focal_px", ctypes.c_float),
        ("target_eye", ctypes.c_int32),
        ("fill_mode", ctypes.c_int32),
    ]


class Model(ctypes.Structure):
    """yoro_model: bf16 model weights and the network's workspace (device)."""

    _fields_ = [
        ("weights", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


def make_model(weights, workspace) -> Model:
    """A yoro_model over a bf16 weights tensor and a uint8 workspace tensor
    (the caller keeps both alive while the calls that use it are queued)."""
    return Model(weights.data_ptr(), workspace.data_ptr(), workspace.numel() * workspace.element_size())


def _model(model):
    return None if model is None else ctypes.byref(model)


_lib = None


def load():
    """Load libyoro.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libyoro.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
    L.yoro_reproject.argtypes = [vp, vp, i32, i32, f32, f32, i32, i32, vp, vp, vp, vp]
    L.yoro_reproject.restype = i32
    L.yoro_reproject_lowres.argtypes = [vp, vp, i32, i32, f32, f32, i32, i32, i32, i32, vp, vp, vp, vp]
    L.yoro_reproject_lowres.restype = i32
    L.yoro_stereo_batch_launch_lowres.argtypes = [vp, i32, ctypes.c_int64, i32, i32, vp]
    L.yoro_stereo_batch_launch_lowres.restype = i32
    L.yoro_reproject_pose_workspace_bytes.argtypes = [i32, i32]
    L.yoro_reproject_pose_workspace_bytes.restype = ctypes.c_size_t
    L.yoro_reproject_pose.argtypes = [vp, vp, i32, i32, f32, f32, f32, vp, vp, i32, vp, vp, vp, vp,
                                      ctypes.c_size_t, vp]
    L.yoro_reproject_pose.restype = i32
    L.yoro_fill_holes.argtypes = [vp, vp, vp, i32, i32, i32, i32, ctypes.POINTER(Model), vp]
    L.yoro_fill_holes.restype = i32
    L.yoro_stereo_batch_workspace_bytes.argtypes = [i32]
    L.yoro_stereo_batch_workspace_bytes.restype = ctypes.c_size_t
    L.yoro_stereo_batch_prepare.argtypes = [ctypes.POINTER(Job), i32, vp, ctypes.c_size_t, vp]
    L.yoro_stereo_batch_prepare.restype = i32
    L.yoro_stereo_batch_launch.argtypes = [vp, i32, ctypes.c_int64, vp]
    L.yoro_stereo_batch_launch.restype = i32
    L.yoro_stereo_batch.argtypes = [ctypes.POINTER(Job), i32, vp, ctypes.c_size_t, ctypes.POINTER(Model), vp]
    L.yoro_stereo_batch.restype = i32
    L.yoro_stereo_batch_static.argtypes = [ctypes.POINTER(Job), i32, vp]
    L.yoro_stereo_batch_static.restype = i32
    L.yoro_stereo_batch_errors.argtypes = [vp]
    L.yoro_stereo_batch_errors.restype = vp
    L.yoro_hole_sse.argtypes = [vp, vp, vp, i32, i32, vp, vp]
    L.yoro_hole_sse.restype = i32
    L.yoro_reproject_hybrid.argtypes = [vp, vp, i32, i32, f32, f32, i32, i32, f32, vp, vp, vp, vp, vp, vp]
    L.yoro_reproject_hybrid.restype = i32
    f64 = ctypes.c_double
    L.yoro_render_near.argtypes = [vp, i32, i32, i32, i32, i32, f64, f64, f64, f64, f32, vp, vp, vp]
    L.yoro_render_near.restype = i32
    L.yoro_measure_stream.argtypes = [vp, vp, vp, ctypes.c_int64, vp]
    L.yoro_measure_stream.restype = i32
    L.yoro_last_error.argtypes = []
    L.yoro_last_error.restype = ctypes.c_char_p
    L.yoro_version.argtypes = []
    L.yoro_version.restype = i32
    _lib = L
    return L


def _check(status: int):
    if status != OK:
        raise YoroError(status, load().yoro_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, dtype, shape, name):
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{name}: want contiguous CUDA {dtype} {tuple(shape)}, got {t.dtype} "
                         f"{tuple(t.shape)} on {t.device}")


def reproject(src_rgba, src_depth, baseline_m: float, focal_px: float, target_eye: int = TARGET_RIGHT,
              fill_mode: int = FILL_NEAREST_BG, out=None, with_depth: bool = True, with_mask: bool = True,
              stream=None):
    """Warp one frame to the other eye.  Returns (rgba, depth or None, mask or None)."""
    H, W = src_depth.shape
    _need(src_rgba, torch.uint8, (H, W, 4), "src_rgba")
    _need(src_depth, torch.float32, (H, W), "src_depth")
    if out is None:
        dev = src_depth.device
        out = (torch.empty((H, W, 4), dtype=torch.uint8, device=dev),
               torch.empty((H, W), dtype=torch.float32, device=dev) if with_depth else None,
               torch.empty((H, W), dtype=torch.uint8, device=dev) if with_mask else None)
    rgba, depth, mask = out
    _check(load().yoro_reproject(_ptr(src_rgba), _ptr(src_depth), W, H, float(baseline_m), float(focal_px),
                                 int(target_eye), int(fill_mode), _ptr(rgba), _ptr(depth), _ptr(mask),
                                 _stream(stream)))
    return rgba, depth, mask


def reproject_lowres(src_rgba, src_depth, baseline_m: float, focal_px: float, target_eye: int = TARGET_RIGHT,
                     fill_mode: int = FILL_NEAREST_BG, scale: int = 4, linear: bool = True, out=None,
                     with_depth: bool = True, with_mask: bool = True, stream=None):
    """Warp one frame to the other eye through a 1/scale intermediate buffer.
    Returns (rgba, depth or None, mask or None)."""
    H, W = src_depth.shape
    _need(src_rgba, torch.uint8, (H, W, 4), "src_rgba")
    _need(src_depth, torch.float32, (H, W), "src_depth")
    if out is None:
        dev = src_depth.device
        out = (torch.empty((H, W, 4), dtype=torch.uint8, device=dev),
               torch.empty((H, W), dtype=torch.float32, device=dev) if with_depth else None,
               torch.empty((H, W), dtype=torch.uint8, device=dev) if with_mask else None)
    rgba, depth, mask = out
    _check(load().yoro_reproject_lowres(_ptr(src_rgba), _ptr(src_depth), W, H, float(baseline_m), float(focal_px),
                                        int(target_eye), int(fill_mode), int(scale), int(bool(linear)), _ptr(rgba),
                                        _ptr(depth), _ptr(mask), _stream(stream)))
    return rgba, depth, mask


def reproject_pose(src_rgba, src_depth, focal_px: float, cx: float, cy: float, rotation, translation,
                   fill_mode: int = FILL_NEAREST_BG, out=None, workspace=None, with_depth: bool = True,
                   with_mask: bool = True, stream=None):
    """Warp one frame to an eye at pose (rotation = unit quaternion (r_x scalar,
    r_y, r_z, r_w), translation in metres), both in the source eye's camera
    frame.  Returns (rgba, depth or None, mask or None)."""
    H, W = src_depth.shape
    _need(src_rgba, torch.uint8, (H, W, 4), "src_rgba")
    _need(src_depth, torch.float32, (H, W), "src_depth")
    L = load()
    if workspace is None:
        workspace = torch.empty(int(L.yoro_reproject_pose_workspace_bytes(W, H)), dtype=torch.uint8,
                                device=src_depth.device)
    if out is None:
        dev = src_depth.device
        out = (torch.empty((H, W, 4), dtype=torch.uint8, device=dev),
               torch.empty((H, W), dtype=torch.float32, device=dev) if with_depth else None,
               torch.empty((H, W), dtype=torch.uint8, device=dev) if with_mask else None)
    rgba, depth, mask = out
    q = (ctypes.c_float * 4)(*[float(v) for v in rotation])
    t = (ctypes.c_float * 3)(*[float(v) for v in translation])
    _check(L.yoro_reproject_pose(_ptr(src_rgba), _ptr(src_depth), W, H, float(focal_px), float(cx), float(cy),
                                 ctypes.cast(q, ctypes.c_void_p), ctypes.cast(t, ctypes.c_void_p), int(fill_mode),
                                 _ptr(rgba), _ptr(depth), _ptr(mask), _ptr(workspace), workspace.numel(),
                                 _stream(stream)))
    return rgba, depth, mask


def fill_holes(rgba, depth, mask, target_eye: int = TARGET_RIGHT, fill_mode: int = FILL_NEAREST_BG, model=None,
               stream=None):
    """Fill holes (mask != 0) of a warped frame in place (FILL_LEARNED needs
    a Model)."""
    H, W = depth.shape
    _need(rgba, torch.uint8, (H, W, 4), "rgba")
    _need(depth, torch.float32, (H, W), "depth")
    _need(mask, torch.uint8, (H, W), "mask")
    _check(load().yoro_fill_holes(_ptr(rgba), _ptr(depth), _ptr(mask), W, H, int(target_eye), int(fill_mode),
                                  _model(model), _stream(stream)))
    return rgba, depth, mask


def reproject_hybrid(src_rgba, src_depth, baseline_m: float, focal_px: float, target_eye: int, fill_mode: int,
                     near_m: float, near_rgba, near_depth, out=None, with_depth: bool = True, with_mask: bool = True,
                     stream=None):
    """Near-object hybrid (include/yoro_hybrid.h): the far field warped and
    filled, the target eye's near layer over it.  Returns (rgba, depth or
    None, mask or None)."""
    H, W = src_depth.shape
    _need(src_rgba, torch.uint8, (H, W, 4), "src_rgba")
    _need(src_depth, torch.float32, (H, W), "src_depth")
    _need(near_rgba, torch.uint8, (H, W, 4), "near_rgba")
    _need(near_depth, torch.float32, (H, W), "near_depth")
    if out is None:
        dev = src_depth.device
        out = (torch.empty((H, W, 4), dtype=torch.uint8, device=dev),
               torch.empty((H, W), dtype=torch.float32, device=dev) if with_depth else None,
               torch.empty((H, W), dtype=torch.uint8, device=dev) if with_mask else None)
    rgba, depth, mask = out
    _check(load().yoro_reproject_hybrid(_ptr(src_rgba), _ptr(src_depth), W, H, float(baseline_m), float(focal_px),
                                        int(target_eye), int(fill_mode), float(near_m), _ptr(near_rgba),
                                        _ptr(near_depth), _ptr(rgba), _ptr(depth), _ptr(mask), _stream(stream)))
    return rgba, depth, mask


def render_near(objects, n: int, width: int, height: int, focal_px: float, cx: float, cy: float, eye_x: float,
                near_m: float, x_off: int = 0, y_off: int = 0, out=None, stream=None):
    """yoro_render_near: the near layer of one eye.  objects: a CUDA uint8
    tensor holding n yoro_object records (88 bytes each).  Returns (rgba, depth)."""
    if objects.dtype != torch.uint8 or not objects.is_cuda or objects.numel() < 88 * n:
        raise ValueError("render_near: objects must be a CUDA uint8 tensor of n * 88 bytes")
    dev = objects.device
    if out is None:
        out = (torch.empty((height, width, 4), dtype=torch.uint8, device=dev),
               torch.empty((height, width), dtype=torch.float32, device=dev))
    rgba, depth = out
    _check(load().yoro_render_near(_ptr(objects), int(n), int(width), int(height), int(x_off), int(y_off),
                                   float(focal_px), float(cx), float(cy), float(eye_x), float(near_m), _ptr(rgba),
                                   _ptr(depth), _stream(stream)))
    return rgba, depth


def make_job(src_rgba, src_depth, dst_rgba, dst_depth, dst_mask, baseline_m, focal_px,
             target_eye=TARGET_RIGHT, fill_mode=FILL_NEAREST_BG) -> Job:
    H, W = src_depth.shape
    return Job(src_rgba.data_ptr(), src_depth.data_ptr(), dst_rgba.data_ptr(),
               None if dst_depth is None else dst_depth.data_ptr(),
               None if dst_mask is None else dst_mask.data_ptr(), W, H, float(baseline_m), float(focal_px),
               int(target_eye), int(fill_mode))


class StereoBatch:
    """A device-resident job table plus the persistent batched launch.

    ``prepare`` validates the jobs and queues the table upload; ``launch``
    runs them (capture-safe).  Tensors referenced by the jobs must stay alive
    while launches that use them are in flight.
    """

    def __init__(self, jobs, device=None):
        L = load()
        self.n = len(jobs)
        self.jobs = (Job * self.n)(*jobs)
        nbytes = L.yoro_stereo_batch_workspace_bytes(self.n)
        if nbytes == 0:
            raise ValueError("bad job count")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=device or "cuda")
        self.max_width = max(j.width for j in jobs)
        self.total_rows = sum(j.height for j in jobs)

    def prepare(self, stream=None):
        _check(load().yoro_stereo_batch_prepare(self.jobs, self.n, _ptr(self.workspace), self.workspace.numel(),
                                                _stream(stream)))

    def launch(self, stream=None, max_width=None, total_rows=None):
        _check(load().yoro_stereo_batch_launch(_ptr(self.workspace), int(max_width or self.max_width),
                                               int(total_rows or self.total_rows), _stream(stream)))

    def launch_lowres(self, scale: int, linear: bool = True, stream=None, max_width=None):
        """Run the prepared jobs through a 1/scale intermediate buffer."""
        _check(load().yoro_stereo_batch_launch_lowres(_ptr(self.workspace), int(max_width or self.max_width),
                                                      int(self.total_rows), int(scale), int(bool(linear)),
                                                      _stream(stream)))

    def run(self, stream=None, model=None):
        """prepare + launch, then the learned fill of FILL_LEARNED jobs (model)."""
        _check(load().yoro_stereo_batch(self.jobs, self.n, _ptr(self.workspace), self.workspace.numel(),
                                        _model(model), _stream(stream)))

    def errors(self) -> int:
        """Rows the last launch skipped (reads the device counter; synchronises)."""
        return int(self.workspace[12:16].view(torch.int32).item())


def stereo_batch_static(jobs, stream=None):
    """yoro_stereo_batch_static: the batch with the library's fixed job table
    (no device allocation; plain jobs only)."""
    arr = (Job * len(jobs))(*jobs)
    _check(load().yoro_stereo_batch_static(arr, len(jobs), _stream(stream)))


def hole_sse(rgba, ref_rgba, mask=None, out=None, stream=None):
    """(device u64[2]: sum of squared RGB errors over mask != 0, pixel count)."""
    H, W = rgba.shape[:2]
    _need(rgba, torch.uint8, (H, W, 4), "rgba")
    _need(ref_rgba, torch.uint8, (H, W, 4), "ref_rgba")
    if mask is not None:
        _need(mask, torch.uint8, (H, W), "mask")
    if out is None:
        out = torch.empty(2, dtype=torch.int64, device=rgba.device)
    _check(load().yoro_hole_sse(_ptr(rgba), _ptr(ref_rgba), _ptr(mask), W, H, _ptr(out), _stream(stream)))
    return out


def measure_stream(a, b, c, stream=None):
    """yoro_measure_stream: c = a ^ b over int32 tensors of one size (the
    warp's 8 B in / 4 B out per element, nothing computed in between)."""
    for t in (a, b, c):
        if t.dtype != torch.int32 or not t.is_contiguous() or not t.is_cuda or t.numel() != a.numel():
            raise ValueError("measure_stream: want contiguous CUDA int32 tensors of one size")
    _check(load().yoro_measure_stream(_ptr(a), _ptr(b), _ptr(c), a.numel(), _stream(stream)))
    return c


def version() -> int:
    return int(load().yoro_version())
