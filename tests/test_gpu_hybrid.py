"""GPU parity of the near-object hybrid (include/yoro_hybrid.h) against the
oracle and the scene generator's ray-caster:

- yoro_render_near against the CPU ray-caster's near field, bit for bit
  (both FP64 in the same operation order, correctly rounded division and
  square root), on seeded scenes, windows with offsets, near distances from
  0.5 m to everything;
- yoro_reproject_hybrid, given the CPU near layer, against
  oracle.reproject_hybrid bit for bit, for the three fills, both eyes,
  ray-cast scenes with near objects and random frames of ragged widths;
- the whole GPU path (near layer and hybrid on the device) against the
  oracle fed the CPU near layer.
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from oracle import reproject as orc
from paper_2506_15183_amd.scenes import raycast, synth
from paper_2506_15183_amd.scenes.configs import FrameSpec, config1_frame, config2_frame

pytestmark = pytest.mark.gpu

R, L = 0, 1


def _gpu():
    import torch

    from paper_2506_15183_amd import yoro

    return torch, yoro


def _objects(torch, sc):
    raw = bytes(memoryview(sc.objects).cast("B"))[: 88 * sc.n]
    return torch.frombuffer(bytearray(raw), dtype=torch.uint8).cuda()


def _near_spec(seed, w, h, n=60):
    # Scenes with near objects: centres log-uniform over [0.3, 8] m.
    return FrameSpec(w, h, 0.063, 900.0, R, n, 0.3, 8.0, True, (4, 32), seed)


def assert_same(g, o, what=""):
    assert np.array_equal(g[0], o[0]), f"rgba differs {what}: {np.argwhere(np.any(g[0] != o[0], axis=-1))[:5]}"
    assert np.array_equal(g[1].view(np.uint32), o[1].view(np.uint32)), f"depth differs {what}"
    if len(g) > 2:
        assert np.array_equal(g[2], o[2]), f"mask differs {what}"


@pytest.mark.parametrize("near", [0.5, 1.0, 3.0, float("inf")])
def test_render_near_matches_cpu_raycaster(cuda, near):
    torch, yoro = _gpu()
    near_pixels = 0
    for spec in (config1_frame(0), _near_spec(11, 640, 480), config2_frame(0)):
        sc = spec.scene()
        objs = _objects(torch, sc)
        for eye_x in (0.0, spec.baseline_m):
            want = raycast.render_near(sc, eye_x, near)
            got = yoro.render_near(objs, sc.n, spec.width, spec.height, sc.f, 0.5 * sc.Wv, 0.5 * sc.Hv, eye_x, near)
            torch.cuda.synchronize()
            assert_same([t.cpu().numpy() for t in got], want, f"{spec.width}x{spec.height} eye {eye_x} near {near}")
            near_pixels += int((want[1] < np.float32(near)).sum())
    assert near_pixels > 1000
    # A window of a larger virtual frame (offsets), as the training windows use.
    spec = _near_spec(12, 1832, 1920)
    sc = spec.scene()
    objs = _objects(torch, sc)
    want = raycast.render_near(sc, 0.0, near, W=300, H=200, x_off=700, y_off=900)
    got = yoro.render_near(objs, sc.n, 300, 200, sc.f, 0.5 * sc.Wv, 0.5 * sc.Hv, 0.0, near, x_off=700, y_off=900)
    torch.cuda.synchronize()
    assert_same([t.cpu().numpy() for t in got], want, "window")


def _run_hybrid(torch, yoro, r, d, B, f, eye, fill, near, nr, nd):
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    out = yoro.reproject_hybrid(T(r), T(d), B, f, eye, fill, near, T(nr), T(nd))
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


@pytest.mark.parametrize("fill", [orc.FILL_NONE, orc.FILL_NEAREST_BG, orc.FILL_PATCHER])
@pytest.mark.parametrize("eye", [R, L])
def test_hybrid_matches_oracle_on_scenes(cuda, fill, eye):
    torch, yoro = _gpu()
    for spec, near in ((_near_spec(21, 512, 384), 1.0), (_near_spec(22, 1000, 300), 2.5), (config1_frame(4), 4.0)):
        spec.target_eye = eye
        sc = spec.scene()
        r, d = spec.render_source()
        nr, nd = raycast.render_near(sc, spec.target_eye_x(), near)
        assert (d < near).any() and (nd < near).any()
        g = _run_hybrid(torch, yoro, r, d, spec.baseline_m, spec.focal_px, eye, fill, near, nr, nd)
        o = orc.reproject_hybrid(r, d, spec.baseline_m, spec.focal_px, eye, fill, near, nr, nd)
        assert_same(g, o, f"{spec.width}x{spec.height} near {near}")
        assert (o[2] == orc.MASK_NEAR).any()


@pytest.mark.parametrize("W", [1, 17, 65, 257, 1000, 2160, 4097])
def test_hybrid_random_frames(cuda, W):
    torch, yoro = _gpu()
    rng = np.random.default_rng(W)
    H = 5
    r, d = synth.random_frame(900 + W, W, H, depth_levels=6, special_frac=0.03, zmin=0.3, zmax=8.0)
    nr = rng.integers(0, 256, size=(H, W, 4), dtype=np.uint8)
    nd = np.where(rng.random((H, W)) < 0.2, rng.uniform(0.1, 0.9, (H, W)), np.inf).astype(np.float32)
    nd[rng.random((H, W)) < 0.02] = np.nan                     # no near surface either
    for eye in (R, L):
        for fill in (orc.FILL_NONE, orc.FILL_NEAREST_BG, orc.FILL_PATCHER):
            g = _run_hybrid(torch, yoro, r, d, 0.063, 900.0, eye, fill, 0.8, nr, nd)
            o = orc.reproject_hybrid(r, d, 0.063, 900.0, eye, fill, 0.8, nr, nd)
            assert_same(g, o, f"W={W} eye={eye} fill={fill}")


def test_hybrid_whole_gpu_path(cuda):
    torch, yoro = _gpu()
    spec = config2_frame(2)
    sc = spec.scene()
    near = 1.0
    r, d = spec.render_source()
    objs = _objects(torch, sc)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    nr_g, nd_g = yoro.render_near(objs, sc.n, spec.width, spec.height, sc.f, 0.5 * sc.Wv, 0.5 * sc.Hv,
                                  spec.target_eye_x(), near)
    g = yoro.reproject_hybrid(T(r), T(d), spec.baseline_m, spec.focal_px, spec.target_eye, orc.FILL_NEAREST_BG, near,
                              nr_g, nd_g)
    torch.cuda.synchronize()
    nr, nd = raycast.render_near(sc, spec.target_eye_x(), near)
    o = orc.reproject_hybrid(r, d, spec.baseline_m, spec.focal_px, spec.target_eye, orc.FILL_NEAREST_BG, near, nr, nd)
    assert_same([t.cpu().numpy() for t in g], o, "C2 frame")
    assert (o[2] == orc.MASK_NEAR).sum() > 1000
