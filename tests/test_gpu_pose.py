"""GPU parity of the reprojection through a general pose (yoro_reproject_pose)
against the oracle, bit-exact: every RGBA byte, depth bit and mask byte.
Random poses (rotations about any axis, translations along any axis), both
fill modes and the Patcher, ray-cast scenes with head motion and toed-in
eyes, random frames with collisions, special depths and ragged sizes up to
the maximum width, the direct path as the special case of a horizontal
translation, and repeat runs (the global atomics decide nothing by order)."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import reproject as orc
from paper_2506_15183_amd.scenes import synth
from paper_2506_15183_amd.scenes.configs import config1_frame, config2_frame

pytestmark = pytest.mark.gpu

IDENT = (1.0, 0.0, 0.0, 0.0)


def _gpu():
    import torch

    from paper_2506_15183_amd import yoro

    return torch, yoro


def quat(angle, axis):
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    return (math.cos(angle / 2), *(math.sin(angle / 2) * axis))


def run_gpu(rgba, depth, f, cx, cy, q, t, fill, with_depth=True, with_mask=True):
    torch, yoro = _gpu()
    a = torch.from_numpy(np.ascontiguousarray(rgba)).cuda()
    d = torch.from_numpy(np.ascontiguousarray(depth)).cuda()
    out = yoro.reproject_pose(a, d, f, cx, cy, q, t, fill, with_depth=with_depth, with_mask=with_mask)
    torch.cuda.synchronize()
    return tuple(None if x is None else x.cpu().numpy() for x in out)


def oracle(rgba, depth, f, cx, cy, q, t, fill):
    if fill == orc.FILL_PATCHER:
        raw = orc.reproject_pose(rgba, depth, f, cx, cy, q, t, orc.FILL_NONE)
        eye = orc.TARGET_RIGHT if np.float32(t[0]) >= 0 else orc.TARGET_LEFT
        return orc.fill_holes(*raw, eye, orc.FILL_PATCHER)
    return orc.reproject_pose(rgba, depth, f, cx, cy, q, t, fill)


def assert_same(g, o, what=""):
    go, gz, gm = g
    oo, oz, om = o
    assert np.array_equal(go, oo), f"rgba differs {what}: {np.argwhere(np.any(go != oo, axis=-1))[:5]}"
    if gz is not None:
        assert np.array_equal(gz.view(np.uint32), oz.view(np.uint32)), f"depth differs {what}"
    if gm is not None:
        assert np.array_equal(gm, om), f"mask differs {what}"


def random_pose(rng, max_angle=0.2, max_t=0.1):
    return quat(rng.uniform(-max_angle, max_angle), rng.normal(size=3)), tuple(rng.uniform(-max_t, max_t, 3))


@pytest.mark.parametrize("spec_fn", [config1_frame, config2_frame])
def test_scenes_head_motion_and_toed_in(cuda, spec_fn):
    spec = spec_fn(0)
    rgba, depth = spec.render_source()
    W, H, f = spec.width, spec.height, spec.focal_px
    cases = [
        (IDENT, (spec.baseline_m, 0.0, 0.0)),                               # parallel stereo
        (quat(math.radians(1.5), (0, 1, 0)), (spec.baseline_m, 0.0, 0.0)),  # toed-in right eye
        (quat(math.radians(3.0), (0.2, 1, 0.1)), (0.02, -0.01, 0.05)),      # head motion
        (quat(math.radians(-2.0), (0, 0, 1)), (-spec.baseline_m, 0.0, 0.0)),
    ]
    for q, t in cases:
        for fill in (orc.FILL_NONE, orc.FILL_NEAREST_BG):
            g = run_gpu(rgba, depth, f, W / 2.0, H / 2.0, q, t, fill)
            o = oracle(rgba, depth, f, W / 2.0, H / 2.0, q, t, fill)
            assert_same(g, o, f"{spec_fn.__name__} q={q} t={t} fill={fill}")


SIZES = [(1, 1), (17, 9), (64, 33), (257, 65), (1000, 40), (2305, 7), (8192, 3)]


@pytest.mark.parametrize("W,H", SIZES)
def test_random_frames_and_poses(cuda, W, H):
    rng = np.random.default_rng(W * 7 + H)
    for case, (levels, special) in enumerate([(3, 0.0), (None, 0.08), (6, 0.03)]):
        rgba, depth = synth.random_frame(300 + W + case, W, H, depth_levels=levels, special_frac=special,
                                         zmin=0.2, zmax=20.0)
        q, t = random_pose(rng)
        f = float(rng.uniform(0.5, 1.5) * max(W, 8))
        cx, cy = float(rng.uniform(0, W)), float(rng.uniform(0, H))
        fill = (orc.FILL_NONE, orc.FILL_NEAREST_BG, orc.FILL_PATCHER)[case]
        g = run_gpu(rgba, depth, f, cx, cy, q, t, fill)
        o = oracle(rgba, depth, f, cx, cy, q, t, fill)
        assert_same(g, o, f"{W}x{H} case={case}")


def test_horizontal_translation_is_the_direct_kernel(cuda):
    torch, yoro = _gpu()
    B, f, W, H = 0.063, 900.0, 1832, 64
    bf = np.float32(np.float32(B) * np.float32(f))
    levels = np.array([np.float32(bf / np.float32(k)) for k in range(1, 200)] + [np.inf], np.float32)
    rng = np.random.default_rng(5)
    d = levels[rng.integers(0, len(levels), (H, W))]
    r = rng.integers(0, 256, (H, W, 4), dtype=np.uint8)
    a, dd = torch.from_numpy(r).cuda(), torch.from_numpy(d).cuda()
    for eye, tx in ((yoro.TARGET_RIGHT, B), (yoro.TARGET_LEFT, -B)):
        direct = yoro.reproject(a, dd, B, f, eye, yoro.FILL_NEAREST_BG)
        via_pose = yoro.reproject_pose(a, dd, f, 900.5, 31.0, IDENT, (tx, 0.0, 0.0), yoro.FILL_NEAREST_BG)
        torch.cuda.synchronize()
        for x, y in zip(direct, via_pose):
            assert torch.equal(x.view(torch.uint8), y.view(torch.uint8))


def test_tall_frame_optional_outputs_and_repeats(cuda):
    rgba, depth = synth.random_frame(11, 33, 4099, depth_levels=4, zmin=0.3, zmax=3.0)
    q, t = quat(0.05, (1, 1, 0)), (0.01, 0.02, -0.03)
    o = oracle(rgba, depth, 40.0, 16.0, 2000.0, q, t, orc.FILL_NEAREST_BG)
    assert_same(run_gpu(rgba, depth, 40.0, 16.0, 2000.0, q, t, orc.FILL_NEAREST_BG), o, "tall")
    g = run_gpu(rgba, depth, 40.0, 16.0, 2000.0, q, t, orc.FILL_NEAREST_BG, with_depth=False, with_mask=False)
    assert g[1] is None and g[2] is None and np.array_equal(g[0], o[0])
    # Many sources meet on few targets (a strong zoom-out): the result does
    # not depend on the order of the atomics.
    rgba, depth = synth.random_frame(12, 512, 256, depth_levels=2, zmin=1.0, zmax=1.2)
    q, t = quat(0.1, (0, 0, 1)), (0.0, 0.0, -3.0)
    first = run_gpu(rgba, depth, 300.0, 256.0, 128.0, q, t, orc.FILL_NEAREST_BG)
    assert_same(first, oracle(rgba, depth, 300.0, 256.0, 128.0, q, t, orc.FILL_NEAREST_BG), "zoom-out")
    for _ in range(3):
        assert_same(run_gpu(rgba, depth, 300.0, 256.0, 128.0, q, t, orc.FILL_NEAREST_BG), first, "repeat")


def test_workspace_reuse_and_errors(cuda):
    torch, yoro = _gpu()
    ws = torch.empty(8 * 300 * 200, dtype=torch.uint8, device="cuda")
    for (W, H) in ((300, 200), (100, 50), (299, 199)):
        rgba, depth = synth.random_frame(W, W, H, depth_levels=5, zmin=0.3, zmax=5.0)
        a, d = torch.from_numpy(rgba).cuda(), torch.from_numpy(depth).cuda()
        q, t = quat(0.03, (0, 1, 0)), (0.05, 0.0, 0.0)
        out = yoro.reproject_pose(a, d, 250.0, W / 2, H / 2, q, t, yoro.FILL_NEAREST_BG, workspace=ws)
        torch.cuda.synchronize()
        assert_same(tuple(x.cpu().numpy() for x in out),
                    oracle(rgba, depth, 250.0, W / 2, H / 2, q, t, orc.FILL_NEAREST_BG), f"{W}x{H}")
    a = torch.zeros((4, 8, 4), dtype=torch.uint8, device="cuda")
    d = torch.ones((4, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(yoro.YoroError) as e:
        yoro.reproject_pose(a, d, 100.0, 4.0, 2.0, (1.0, 0.5, 0.0, 0.0), (0, 0, 0))
    assert e.value.status == yoro.ERR_INVALID_ARG
    with pytest.raises(yoro.YoroError) as e:
        yoro.reproject_pose(a, d, 100.0, 4.0, 2.0, IDENT, (0, 0, 0), workspace=ws[:100])
    assert e.value.status == yoro.ERR_WORKSPACE_TOO_SMALL
