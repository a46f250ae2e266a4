"""Pins of the oracle's reprojection through a general pose (Section 6: the
rotation matrix of a unit quaternion, the view and projection matrices and
M = (VP_src)^-1 VP_tgt, under the readings stated in oracle/reproject.c):

- the identity pose is the identity image;
- a pure horizontal translation by the baseline is the (pinned) direct path,
  bit for bit, for both eyes, on depths whose disparity is integral;
- a rotation by 90 degrees about the optical axis turns the image by 90
  degrees (fixes the quaternion's component order and the transpose);
- moving forward by half the distance of a plane magnifies it by 2 (fixes the
  perspective divide and the translation's sign);
- points at infinity only rotate; points behind the target eye are dropped;
- the two-dimensional depth test equals brute force over all sources on tiny
  frames.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import reproject as O
from paper_2506_15183_amd.scenes import synth

IDENT = (1.0, 0.0, 0.0, 0.0)


def pose(r, d, f, cx, cy, q, t, fill=O.FILL_NONE):
    return O.reproject_pose(r, d, f, cx, cy, q, t, fill)


def test_identity_pose_is_the_identity():
    r, d = synth.random_frame(1, 57, 23, special_frac=0.15, zmin=0.1, zmax=40.0)
    out, z, m = pose(r, d, 300.0, 20.3, 11.7, IDENT, (0, 0, 0))
    ok = (d > 0) | np.isposinf(d)
    ok &= ~np.isnan(d)
    assert np.array_equal(m, np.where(ok, 0, 1).astype(np.uint8))
    assert np.array_equal(out[ok], r[ok])
    assert np.array_equal(z[ok].view(np.uint32), d[ok].view(np.uint32))
    assert (out[~ok] == 0).all()


@pytest.mark.parametrize("eye", [O.TARGET_RIGHT, O.TARGET_LEFT])
@pytest.mark.parametrize("fill", [O.FILL_NONE, O.FILL_NEAREST_BG])
def test_horizontal_translation_is_the_direct_path(eye, fill):
    B, f, W, H = 0.064, 200.0, 96, 20
    bf = np.float32(np.float32(B) * np.float32(f))
    levels = [np.float32(bf / np.float32(k)) for k in range(1, 41)] + [np.float32(np.inf)]
    for k, z in enumerate(levels[:-1]):
        assert O.disparity(float(z), B, f, W) == k + 1
    rng = np.random.default_rng(7)
    d = np.array(levels, np.float32)[rng.integers(0, len(levels), (H, W))]
    r = rng.integers(0, 256, (H, W, 4), dtype=np.uint8)
    want = O.reproject(r, d, B, f, eye, fill)
    t = (B, 0.0, 0.0) if eye == O.TARGET_RIGHT else (-B, 0.0, 0.0)
    got = pose(r, d, f, 41.5, 9.25, IDENT, t, fill)
    assert np.array_equal(got[0], want[0])
    assert np.array_equal(got[1].view(np.uint32), want[1].view(np.uint32))
    assert np.array_equal(got[2], want[2])


@pytest.mark.parametrize("N", [40, 41])
def test_rotation_about_the_optical_axis_turns_the_image(N):
    # q = (cos 45, 0, 0, sin 45): 90 degrees about z (r_w is the z part).
    # X_t = R^T X gives x' - c = y - c, y' - c = -(x - c), with c = (N-1)/2:
    # pixel (x, y) lands on (y, N-1-x).
    rng = np.random.default_rng(N)
    r = rng.integers(0, 256, (N, N, 4), dtype=np.uint8)
    d = rng.uniform(0.5, 30.0, (N, N)).astype(np.float32)
    h = math.sqrt(0.5)
    c = (N - 1) / 2.0
    out, z, m = pose(r, d, 250.0, c, c, (h, 0.0, 0.0, h), (0, 0, 0))
    assert (m == 0).all()
    for y in range(N):
        for x in range(N):
            assert np.array_equal(out[N - 1 - x, y], r[y, x])
            assert z[N - 1 - x, y] == d[y, x]
    # The opposite rotation turns it back the other way.
    out2, _, _ = pose(r, d, 250.0, c, c, (h, 0.0, 0.0, -h), (0, 0, 0))
    for y in range(N):
        for x in range(N):
            assert np.array_equal(out2[x, N - 1 - y], r[y, x])


def test_moving_forward_magnifies_a_plane():
    # A plane at z = 2 seen from 1 m further forward: Z_t = 1 and every
    # offset from the principal point doubles, so the hits sit on every
    # other pixel and carry the source pixel halfway to the centre.
    W, H, cx, cy = 64, 48, 32.0, 24.0
    rng = np.random.default_rng(3)
    r = rng.integers(0, 256, (H, W, 4), dtype=np.uint8)
    d = np.full((H, W), 2.0, np.float32)
    out, z, m = pose(r, d, 300.0, cx, cy, IDENT, (0.0, 0.0, 1.0))
    for yt in range(H):
        for xt in range(W):
            if (xt - 32) % 2 == 0 and (yt - 24) % 2 == 0:
                assert m[yt, xt] == 0 and z[yt, xt] == 1.0
                assert np.array_equal(out[yt, xt], r[(yt + 24) // 2, (xt + 32) // 2])
            else:
                assert m[yt, xt] == 1


def test_points_at_infinity_only_rotate_and_points_behind_are_dropped():
    W, H = 30, 30
    rng = np.random.default_rng(4)
    r = rng.integers(0, 256, (H, W, 4), dtype=np.uint8)
    d = np.full((H, W), np.inf, np.float32)
    out, z, m = pose(r, d, 200.0, 14.5, 14.5, IDENT, (0.5, -0.2, 0.3))
    assert (m == 0).all() and np.array_equal(out, r) and np.isposinf(z).all()
    h = math.sqrt(0.5)
    out, _, _ = pose(r, d, 200.0, 14.5, 14.5, (h, 0.0, 0.0, h), (0.5, -0.2, 0.3))
    assert np.array_equal(out[W - 1 - 3, 5], r[5, 3])
    # A plane 2 m ahead, the target eye 5 m forward: everything is behind it.
    d = np.full((H, W), 2.0, np.float32)
    _, _, m = pose(r, d, 200.0, 14.5, 14.5, IDENT, (0.0, 0.0, 5.0))
    assert (m == 1).all()
    _, _, m = pose(r, d, 200.0, 14.5, 14.5, IDENT, (0.0, 0.0, 5.0), O.FILL_NEAREST_BG)
    assert (m == 2).all()


@pytest.mark.parametrize("seed", range(6))
def test_depth_test_is_brute_force_over_all_sources(seed):
    rng = np.random.default_rng(100 + seed)
    W, H = 11, 7
    r = rng.integers(0, 256, (H, W, 4), dtype=np.uint8)
    d = rng.choice(np.array([0.4, 0.7, 1.5, 3.0, np.inf, -1.0], np.float32), size=(H, W))
    ang = rng.uniform(-0.3, 0.3)
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    q = (math.cos(ang / 2), *(math.sin(ang / 2) * axis))
    t = tuple(rng.uniform(-0.2, 0.2, 3))
    f, cx, cy = 9.0, 5.0, 3.0
    out, z, m = pose(r, d, f, cx, cy, q, t)
    # Brute force: every target pixel looks at every source pixel.
    landed = {}
    for y in range(H):
        for x in range(W):
            p = O.project_pose(float(d[y, x]), x, y, W, H, f, cx, cy, q, t)
            if p is not None:
                landed.setdefault((p[1], p[0]), []).append((np.float32(p[2]).view(np.uint32), y * W + x, p[2]))
    assert any(len(v) > 1 for v in landed.values())  # the case has collisions
    for yt in range(H):
        for xt in range(W):
            cand = landed.get((yt, xt))
            if not cand:
                assert m[yt, xt] == 1 and not out[yt, xt].any()
                continue
            zb, idx, zt = min(cand)
            assert m[yt, xt] == 0
            assert np.array_equal(out[yt, xt], r.reshape(-1, 4)[idx])
            assert z[yt, xt].view(np.uint32) == zb


def test_fill_is_the_row_fill_of_the_unfilled_result():
    rng = np.random.default_rng(9)
    r, d = synth.random_frame(9, 80, 30, depth_levels=6, zmin=0.3, zmax=5.0)
    for t in ((0.06, 0.01, 0.02), (-0.06, 0.0, -0.1)):
        q = (0.999, 0.02, -0.03, 0.01)
        n = math.sqrt(sum(v * v for v in q))
        q = tuple(v / n for v in q)
        raw = pose(r, d, 120.0, 40.0, 15.0, q, t)
        filled = pose(r, d, 120.0, 40.0, 15.0, q, t, O.FILL_NEAREST_BG)
        eye = O.TARGET_RIGHT if t[0] >= 0 else O.TARGET_LEFT
        want = O.fill_holes(*raw, eye, O.FILL_NEAREST_BG)
        for a, b in zip(filled, want):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    del rng


def test_bad_arguments():
    r, d = synth.random_frame(1, 8, 8)
    with pytest.raises(ValueError):
        pose(r, d, 100.0, 4.0, 4.0, IDENT, (0, 0, 0), O.FILL_PATCHER)
