"""Pins of the oracle's near-object hybrid (Section 11.4, Impact of Object
Distance: nearer than a minimum distance, objects are rendered
conventionally, the method handles the rest), under the reading stated in
oracle/reproject.c: the far field (source depth >= D) is warped and filled,
the target eye's near layer (depth < D, from the ray-caster) wins wherever
it exists.

- D below every depth with an empty near layer: the plain path bit for bit.
- D beyond every depth: nothing is warped; every pixel where the target eye
  sees a surface is the ray-cast target eye, every other one an unfillable
  hole.
- A near sphere over a far textured plane at integer disparity d: each
  target pixel is, independently of the oracle's code, the ray-cast sphere
  where the target eye sees the sphere, else source pixel x + d (or x - d)
  when that one is plane, else a hole; and the hole count is exactly the
  plane pixels the source eye lost behind the sphere that the target eye
  sees.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import reproject as orc
from paper_2506_15183_amd.scenes import raycast
from paper_2506_15183_amd.scenes.configs import config1_frame

R, L = orc.TARGET_RIGHT, orc.TARGET_LEFT


def _empty_layer(H, W):
    return np.zeros((H, W, 4), np.uint8), np.full((H, W), np.inf, np.float32)


@pytest.mark.parametrize("fill", [orc.FILL_NONE, orc.FILL_NEAREST_BG, orc.FILL_PATCHER])
def test_nothing_near_is_the_plain_path(fill):
    spec = config1_frame(2)
    r, d = spec.render_source()
    assert d.min() > 0.25
    nr, nd = _empty_layer(*d.shape)
    for near in (0.0, 0.25):
        h = orc.reproject_hybrid(r, d, spec.baseline_m, spec.focal_px, spec.target_eye, fill, near, nr, nd)
        p = orc.reproject(r, d, spec.baseline_m, spec.focal_px, spec.target_eye, fill)
        assert np.array_equal(h[0], p[0]) and np.array_equal(h[2], p[2])
        assert np.array_equal(h[1].view(np.uint32), p[1].view(np.uint32))
        assert not (h[2] == orc.MASK_NEAR).any()


@pytest.mark.parametrize("eye", [R, L])
def test_everything_near_is_the_rendered_target_eye(eye):
    spec = config1_frame(3)
    spec.target_eye = eye
    sc = spec.scene()
    r, d = spec.render_source()
    tr, td = spec.render_target()
    near = np.inf
    nr, nd = raycast.render_near(sc, spec.target_eye_x(), near)
    out, dz, mk = orc.reproject_hybrid(r, d, spec.baseline_m, spec.focal_px, eye, orc.FILL_NEAREST_BG, near, nr, nd)
    seen = td < raycast.BACKGROUND_DEPTH
    assert seen.any() and (~seen).any()
    assert (mk[seen] == orc.MASK_NEAR).all()
    assert np.array_equal(out[seen], tr[seen]) and np.array_equal(dz[seen], td[seen])
    # No source pixel is far: every other pixel is a hole with no hit in its row.
    assert (mk[~seen] == 2).all() and (out[~seen] == 0).all()


def _sphere_over_plane(eye, W=160, H=96):
    B, f, zp = 0.064, 200.0, 2.56          # plane disparity B f / z = 5 exactly
    d = 5
    plane = dict(kind=raycast.BOX, c=(0.0, 0.0, zp + 1.0), h=(40.0, 40.0, 1.0), texel=zp / f,
                 rgb=(120, 90, 60), noise=16, id=1)
    sphere = dict(kind=raycast.SPHERE, c=(0.02, -0.01, 0.4), h=(0.06, 0.0, 0.0), texel=0.4 / f,
                  cell=8 * 0.4 / f, rgb=(30, 200, 90), noise=16, id=2)
    sc = raycast.scene_from_objects([plane, sphere], W, H, f, seed=9)
    src_x, tgt_x = (0.0, B) if eye == R else (B, 0.0)
    return sc, B, f, d, src_x, tgt_x


@pytest.mark.parametrize("eye", [R, L])
@pytest.mark.parametrize("near", [0.5, 1.5])
def test_near_sphere_over_a_plane(eye, near):
    sc, B, f, d, src_x, tgt_x = _sphere_over_plane(eye)
    sr, sd = raycast.render(sc, src_x)
    tr, td = raycast.render(sc, tgt_x)
    nr, nd = raycast.render_near(sc, tgt_x, near)
    H, W = sd.shape
    is_sphere_src = sd < near
    assert is_sphere_src.sum() > 200 and np.all(sd[~is_sphere_src] == np.float32(2.56))
    out, dz, mk = orc.reproject_hybrid(sr, sd, B, f, eye, orc.FILL_NONE, near, nr, nd)
    # The characterisation, pixel by pixel.
    step = d if eye == R else -d                       # target x receives source x + step
    for y in range(H):
        for x in range(W):
            xs = x + step
            if td[y, x] < near:                      # the target eye sees the sphere
                assert mk[y, x] == orc.MASK_NEAR and np.array_equal(out[y, x], tr[y, x]), (y, x)
            elif 0 <= xs < W and not is_sphere_src[y, xs]:
                assert mk[y, x] == 0 and np.array_equal(out[y, x], sr[y, xs]), (y, x)
            else:
                assert mk[y, x] == 1 and (out[y, x] == 0).all(), (y, x)
    # Holes: the border band of width d plus the plane the sphere hid in the
    # source eye that the target eye sees, and those are not empty.
    xs = np.arange(W) + step
    inside = (xs >= 0) & (xs < W)
    hidden = np.zeros((H, W), bool)
    hidden[:, inside] = is_sphere_src[:, xs[inside]]
    lost = hidden & ~(td < near)
    assert lost.sum() > 0
    assert (mk == 1).sum() == lost.sum() + H * d
    # The sphere's pixels are exactly the ray-cast target eye (colour and depth).
    near_px = mk == orc.MASK_NEAR
    assert np.array_equal(out[near_px], tr[near_px]) and np.array_equal(dz[near_px], td[near_px])


def test_fill_acts_on_the_far_field_only():
    # With the nearest-background fill every far-field hole takes a plane
    # pixel (depth 2.56), never the sphere's, and the near layer is untouched.
    sc, B, f, d, src_x, tgt_x = _sphere_over_plane(R)
    sr, sd = raycast.render(sc, src_x)
    nr, nd = raycast.render_near(sc, tgt_x, 1.0)
    out, dz, mk = orc.reproject_hybrid(sr, sd, B, f, R, orc.FILL_NEAREST_BG, 1.0, nr, nd)
    assert (mk == 1).any()
    assert np.all(dz[mk == 1] == np.float32(2.56))
    assert np.array_equal(out[mk == orc.MASK_NEAR], nr[mk == orc.MASK_NEAR])
