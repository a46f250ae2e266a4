"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, and rejects bad arguments on the host before touching a device."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(name="yoro.h"):
    text = open(os.path.join(ROOT, "include", name)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(yoro_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    fns = header_functions()
    for name in ("yoro_reproject", "yoro_fill_holes", "yoro_stereo_batch"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    from paper_2506_15183_amd import yoro

    lib = yoro.load()
    for name in header_functions():
        assert hasattr(lib, name), name
    assert set(header_functions()) == set(yoro.EXPORTS)
    assert yoro.version() == 1
    for header in ("yoro_nn.h", "yoro_model.h", "yoro_serve.h", "yoro_measure.h", "yoro_hybrid.h"):
        names = header_functions(header)
        assert names, header
        for name in names:
            assert hasattr(lib, name), name
    from paper_2506_15183_amd import serve

    assert set(header_functions("yoro_serve.h")) == set(serve.EXPORTS)
    assert set(header_functions("yoro_measure.h")) == set(yoro.MEASURE_EXPORTS)
    assert set(header_functions("yoro_hybrid.h")) == set(yoro.HYBRID_EXPORTS)
    # the streaming kernel's host checks: misaligned, overlapping, empty
    L = yoro.load()
    a, b, c = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    assert L.yoro_measure_stream(ctypes.c_void_p(0x100004), b, c, 16, None) == yoro.ERR_INVALID_ARG
    assert L.yoro_measure_stream(a, b, ctypes.c_void_p(0x100010), 16, None) == yoro.ERR_INVALID_ARG
    assert L.yoro_measure_stream(a, b, c, 0, None) == yoro.ERR_INVALID_ARG


def test_nn_host_validation_rejects_without_launching():
    from paper_2506_15183_amd import unet, yoro

    L = unet.nnlib()
    a = ctypes.c_void_p(0x100000)
    b = ctypes.c_void_p(0x200000)
    c = ctypes.c_void_p(0x300000)
    # cin not a multiple of 32
    assert L.yoro_nn_conv3x3(a, 40, 1, 8, 8, 40, b, 32, c, 32, 0, 32, 0, None, 0, None) == yoro.ERR_INVALID_ARG
    # misaligned input
    assert L.yoro_nn_conv3x3(ctypes.c_void_p(0x100002), 32, 1, 8, 8, 32, b, 32, c, 32, 0, 32, 0, None, 0,
                             None) == yoro.ERR_INVALID_ARG
    # ReLU-derivative epilogue without its source
    assert L.yoro_nn_conv3x3(a, 32, 1, 8, 8, 32, b, 32, c, 32, 0, 32, 2, None, 0, None) == yoro.ERR_INVALID_ARG
    # odd pool size, workspace too small
    assert L.yoro_nn_avgpool2(a, 32, 1, 7, 8, 32, b, 32, None) == yoro.ERR_INVALID_ARG
    assert L.yoro_nn_conv3x3_wgrad(a, 32, b, 32, 1, 8, 8, 32, 32, c, a, 16, None) == yoro.ERR_WORKSPACE_TOO_SMALL
    assert L.yoro_nn_adamw(a, b, c, a, 10, 1e-3, 0.9, 0.999, 1e-8, 0.01, 0, None) == yoro.ERR_INVALID_ARG


def test_host_validation_rejects_without_launching():
    from paper_2506_15183_amd import yoro

    L = yoro.load()
    fake = ctypes.c_void_p(0x10000)
    fake2 = ctypes.c_void_p(0x20000000)
    fake3 = ctypes.c_void_p(0x40000000)
    # null required pointer
    assert L.yoro_reproject(None, fake, 8, 8, 0.06, 900.0, 0, 1, fake2, None, None, None) == yoro.ERR_INVALID_ARG
    assert b"required" in L.yoro_last_error()
    # sizes
    assert L.yoro_reproject(fake, fake2, 0, 8, 0.06, 900.0, 0, 1, fake3, None, None, None) == yoro.ERR_INVALID_ARG
    assert L.yoro_reproject(fake, fake2, 8193, 8, 0.06, 900.0, 0, 1, fake3, None, None, None) == yoro.ERR_UNSUPPORTED
    # camera
    for B, f in [(0.0, 900.0), (-0.06, 900.0), (float("inf"), 900.0), (0.06, float("nan"))]:
        assert L.yoro_reproject(fake, fake2, 8, 8, B, f, 0, 1, fake3, None, None, None) == yoro.ERR_INVALID_ARG
    # eye / mode
    assert L.yoro_reproject(fake, fake2, 8, 8, 0.06, 900.0, 2, 1, fake3, None, None, None) == yoro.ERR_INVALID_ARG
    assert L.yoro_reproject(fake, fake2, 8, 8, 0.06, 900.0, 0, 7, fake3, None, None, None) == yoro.ERR_INVALID_ARG
    # alignment
    odd = ctypes.c_void_p(0x10001)
    assert L.yoro_reproject(odd, fake2, 8, 8, 0.06, 900.0, 0, 1, fake3, None, None, None) == yoro.ERR_INVALID_ARG
    # overlap: output inside the source colour
    inside = ctypes.c_void_p(0x10000 + 16)
    assert L.yoro_reproject(fake, fake2, 8, 8, 0.06, 900.0, 0, 1, inside, None, None, None) == yoro.ERR_INVALID_ARG
    assert b"overlap" in L.yoro_last_error()
    # the near-object hybrid: near_m finite and > 0, the near layer present and
    # clear of the outputs, no learned fill
    nr, nd = ctypes.c_void_p(0x60000000), ctypes.c_void_p(0x64000000)
    for nm in (0.0, -1.0, float("nan"), float("inf")):
        assert L.yoro_reproject_hybrid(fake, fake2, 8, 8, 0.06, 900.0, 0, 1, nm, nr, nd, fake3, None, None,
                                       None) == yoro.ERR_INVALID_ARG
    assert L.yoro_reproject_hybrid(fake, fake2, 8, 8, 0.06, 900.0, 0, 1, 1.0, None, nd, fake3, None, None,
                                   None) == yoro.ERR_INVALID_ARG
    assert L.yoro_reproject_hybrid(fake, fake2, 8, 8, 0.06, 900.0, 0, 1, 1.0, fake3, nd, fake3, None, None,
                                   None) == yoro.ERR_INVALID_ARG                        # output over the layer
    assert L.yoro_reproject_hybrid(fake, fake2, 8, 8, 0.06, 900.0, 0, yoro.FILL_LEARNED, 1.0, nr, nd, fake3, None,
                                   None, None) == yoro.ERR_UNSUPPORTED
    assert L.yoro_render_near(None, 3, 8, 8, 0, 0, 900.0, 4.0, 4.0, 0.0, 1.0, fake, fake2, None) == yoro.ERR_INVALID_ARG
    assert L.yoro_render_near(fake3, -1, 8, 8, 0, 0, 900.0, 4.0, 4.0, 0.0, 1.0, fake, fake2, None) == yoro.ERR_INVALID_ARG
    assert L.yoro_render_near(fake3, 3, 8, 8, 0, 0, 0.0, 4.0, 4.0, 0.0, 1.0, fake, fake2, None) == yoro.ERR_INVALID_ARG
    assert L.yoro_render_near(fake3, 3, 8, 8, 0, 0, 900.0, 4.0, 4.0, 0.0, 0.0, fake, fake2, None) == yoro.ERR_INVALID_ARG
    # fill_holes
    assert L.yoro_fill_holes(None, fake2, fake3, 8, 8, 0, 1, None, None) == yoro.ERR_INVALID_ARG
    # the learned fill: only with a model, sizes multiples of 8, workspace large enough
    from paper_2506_15183_amd import unet

    assert L.yoro_reproject(fake, fake2, 8, 8, 0.06, 900.0, 0, yoro.FILL_LEARNED, fake3, None, None,
                            None) == yoro.ERR_UNSUPPORTED
    assert b"model" in L.yoro_last_error()
    mk = ctypes.c_void_p(0x50000000)
    assert L.yoro_fill_holes(fake, fake2, mk, 8, 8, 0, yoro.FILL_LEARNED, None, None) == yoro.ERR_INVALID_ARG
    need = unet.nnlib().yoro_model_workspace_bytes(1, 8, 8)
    assert need > 0
    model = yoro.Model(0x58000000, 0x5C000000, need - 1)
    assert L.yoro_fill_holes(fake, fake2, mk, 8, 8, 0, yoro.FILL_LEARNED, ctypes.byref(model),
                             None) == yoro.ERR_WORKSPACE_TOO_SMALL
    model.workspace_bytes = need
    assert L.yoro_fill_holes(fake, fake2, mk, 12, 8, 0, yoro.FILL_LEARNED, ctypes.byref(model),
                             None) == yoro.ERR_UNSUPPORTED
    bad = yoro.Model(0x58000008, 0x5C000000, need)
    assert L.yoro_fill_holes(fake, fake2, mk, 8, 8, 0, yoro.FILL_LEARNED, ctypes.byref(bad),
                             None) == yoro.ERR_INVALID_ARG                             # misaligned weights
    over = yoro.Model(0x58000000, 0x10000, need)
    assert L.yoro_fill_holes(fake, fake2, mk, 8, 8, 0, yoro.FILL_LEARNED, ctypes.byref(over),
                             None) == yoro.ERR_INVALID_ARG                             # workspace over the frame
    assert b"overlap" in L.yoro_last_error()
    # batch
    assert L.yoro_stereo_batch_workspace_bytes(0) == 0
    assert L.yoro_stereo_batch_workspace_bytes(64) == 64 + 64 * 72
    jobs = (yoro.Job * 2)()
    for j in jobs:
        j.src_rgba, j.src_depth, j.dst_rgba = 0x10000, 0x20000000, 0x40000000
        j.width, j.height, j.baseline_m, j.focal_px, j.target_eye, j.fill_mode = 8, 8, 0.06, 900.0, 0, 1
    ws = ctypes.c_void_p(0x7000000)
    # both jobs write the same output
    assert L.yoro_stereo_batch_prepare(jobs, 2, ws, 4096, None) == yoro.ERR_INVALID_ARG
    assert b"overlap" in L.yoro_last_error()
    assert L.yoro_stereo_batch_prepare(jobs, 2, ws, 8, None) == yoro.ERR_WORKSPACE_TOO_SMALL
    assert L.yoro_stereo_batch_launch(ws, 0, 16, None) == yoro.ERR_INVALID_ARG
    assert L.yoro_stereo_batch_launch(ws, 8, 0, None) == yoro.ERR_INVALID_ARG        # no rows
    assert L.yoro_stereo_batch_launch(ws, 8, 1 << 32, None) == yoro.ERR_INVALID_ARG  # too many rows
    # learned jobs: not through prepare; through yoro_stereo_batch only with a
    # model, dst_depth and dst_mask
    one = (yoro.Job * 1)()
    one[0].src_rgba, one[0].src_depth, one[0].dst_rgba = 0x10000, 0x20000000, 0x40000000
    one[0].width, one[0].height, one[0].baseline_m, one[0].focal_px = 8, 8, 0.06, 900.0
    one[0].target_eye, one[0].fill_mode = 0, yoro.FILL_LEARNED
    assert L.yoro_stereo_batch_prepare(one, 1, ws, 4096, None) == yoro.ERR_UNSUPPORTED
    assert L.yoro_stereo_batch(one, 1, ws, 4096, ctypes.byref(model), None) == yoro.ERR_INVALID_ARG
    assert b"dst_depth" in L.yoro_last_error()
    one[0].dst_depth, one[0].dst_mask = 0x44000000, 0x48000000
    assert L.yoro_stereo_batch(one, 1, ws, 4096, None, None) == yoro.ERR_INVALID_ARG
    model.workspace_bytes = need - 1
    assert L.yoro_stereo_batch(one, 1, ws, 4096, ctypes.byref(model), None) == yoro.ERR_WORKSPACE_TOO_SMALL
    model.workspace_bytes = need
    # the downsampled-buffer calls: scale and linear are checked too
    for scale in (0, 3, 32, -1):
        assert L.yoro_reproject_lowres(fake, fake2, 8, 8, 0.06, 900.0, 0, 1, scale, 1, fake3, None, None,
                                       None) == yoro.ERR_INVALID_ARG
        assert L.yoro_stereo_batch_launch_lowres(ws, 8, 16, scale, 1, None) == yoro.ERR_INVALID_ARG
    assert L.yoro_reproject_lowres(fake, fake2, 8, 8, 0.06, 900.0, 0, 1, 4, 2, fake3, None, None,
                                   None) == yoro.ERR_INVALID_ARG
    assert L.yoro_reproject_lowres(None, fake2, 8, 8, 0.06, 900.0, 0, 1, 4, 1, fake3, None, None,
                                   None) == yoro.ERR_INVALID_ARG
    assert L.yoro_reproject_lowres(fake, fake2, 8, 8, 0.06, 900.0, 0, 3, 4, 1, fake3, None, None,
                                   None) == yoro.ERR_INVALID_ARG   # the Patcher needs depth and mask
    assert L.yoro_stereo_batch_launch_lowres(None, 8, 16, 4, 1, None) == yoro.ERR_INVALID_ARG
    assert L.yoro_stereo_batch_launch_lowres(ws, 8193, 16, 4, 1, None) == yoro.ERR_INVALID_ARG
    assert L.yoro_stereo_batch_launch_lowres(ws, 8, 0, 4, 1, None) == yoro.ERR_INVALID_ARG
    # the general-pose call: a unit quaternion, finite values, a workspace of one u64 per pixel
    assert L.yoro_reproject_pose_workspace_bytes(8, 8) == 512
    assert L.yoro_reproject_pose_workspace_bytes(0, 8) == 0
    q = (ctypes.c_float * 4)(1, 0, 0, 0)
    t = (ctypes.c_float * 3)(0.06, 0, 0)
    wsp = ctypes.c_void_p(0x60000000)
    args = [fake, fake2, 8, 8, 900.0, 4.0, 4.0, q, t, 1, fake3, None, None]
    assert L.yoro_reproject_pose(*args, None, 512, None) == yoro.ERR_INVALID_ARG       # no workspace
    assert L.yoro_reproject_pose(*args, wsp, 511, None) == yoro.ERR_WORKSPACE_TOO_SMALL
    assert L.yoro_reproject_pose(*args, ctypes.c_void_p(0x60000008), 512, None) == yoro.ERR_INVALID_ARG  # alignment
    assert L.yoro_reproject_pose(*args, ctypes.c_void_p(0x40000000), 512, None) == yoro.ERR_INVALID_ARG  # overlap
    q2 = (ctypes.c_float * 4)(1, 0.1, 0, 0)
    assert L.yoro_reproject_pose(fake, fake2, 8, 8, 900.0, 4.0, 4.0, q2, t, 1, fake3, None, None, wsp, 512,
                                 None) == yoro.ERR_INVALID_ARG                          # not a unit quaternion
    assert b"unit quaternion" in L.yoro_last_error()
    assert L.yoro_reproject_pose(fake, fake2, 8, 8, 900.0, float("nan"), 4.0, q, t, 1, fake3, None, None, wsp, 512,
                                 None) == yoro.ERR_INVALID_ARG
    assert L.yoro_reproject_pose(fake, fake2, 8, 8, 900.0, 4.0, 4.0, q, t, 3, fake3, None, None, wsp, 512,
                                 None) == yoro.ERR_INVALID_ARG                          # the Patcher needs depth + mask
