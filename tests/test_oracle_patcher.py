"""Pins of the oracle's Patcher fill (Section 7, Algorithm 3 with the weight
function of Equation 7, under the readings stated in oracle/reproject.c):
closed forms on hand-built rows, the foreground skip, the neighbouring rows,
agreement with the nearest-background fill on everything but the colour,
mirror symmetry between the eyes, and a kernel as wide as the
disocclusion (no cap on its width)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import reproject as O
from paper_2506_15183_amd.scenes import config1_frame, config2_frame, synth


def frame(cols, depths, mask, alpha=255):
    """1-row (or n-row) frame from per-pixel grey levels, depths and mask."""
    cols = np.atleast_2d(np.asarray(cols, dtype=np.uint8))
    H, W = cols.shape
    rgba = np.zeros((H, W, 4), np.uint8)
    rgba[..., 0] = cols
    rgba[..., 1] = cols
    rgba[..., 2] = cols
    rgba[..., 3] = alpha
    return rgba, np.atleast_2d(np.asarray(depths, np.float32)), np.atleast_2d(np.asarray(mask, np.uint8))


def patch(rgba, depth, mask, eye=O.TARGET_RIGHT):
    return O.fill_holes(rgba, depth, mask, eye, O.FILL_PATCHER)


def test_two_samples_closed_form():
    # Hits at 0 (near: foreground), 3, 4, 5 (far); holes at 1, 2.  Synthesising
    # the right eye, the background edge is R = 3, the run width is 2, and
    # the kernel samples columns 3 and 4 (width 2, one row).
    rgba, depth, mask = frame([50, 0, 0, 200, 100, 7], [1.0, np.inf, np.inf, 10.0, 10.0, 10.0], [0, 1, 1, 0, 0, 0])
    out, z, m = patch(rgba, depth, mask)
    for x, dist in ((1, 2), (2, 1)):
        t = dist / 2.0                       # distance from the edge / run width
        f = 0.5 + 0.3 * t                    # w / w_rem
        w1, w2 = f, (1 - f) * f
        want = round((200 * w1 + 100 * w2) / (w1 + w2))
        assert out[0, x, 0] == want and out[0, x, 1] == want and out[0, x, 2] == want
        assert z[0, x] == 10.0 and m[0, x] == 1 and out[0, x, 3] == 255
    assert out[0, 1, 0] == 183 and out[0, 2, 0] == 174   # 176/0.96 and 152.75/0.8775
    # Hits are left as they were.
    assert np.array_equal(out[0, [0, 3, 4, 5]], rgba[0, [0, 3, 4, 5]])


def test_foreground_samples_are_skipped():
    # Column 4 is nearer than the edge (depth 2 < 10): it is not sampled, so
    # only the edge itself contributes.
    rgba, depth, mask = frame([50, 0, 0, 200, 100, 7], [1.0, np.inf, np.inf, 10.0, 2.0, 10.0], [0, 1, 1, 0, 0, 0])
    out, _, _ = patch(rgba, depth, mask)
    assert out[0, 1, 0] == 200 and out[0, 2, 0] == 200


def test_kernel_width_is_the_disocclusion_width():
    # Section 7: the kernel is as wide as the disocclusion in the hole's row.
    # One-pixel hole: the kernel is one column wide, so the far sample (40)
    # never counts.
    rgba, depth, mask = frame([50, 0, 200, 40], [1.0, np.inf, 10.0, 10.0], [0, 1, 0, 0])
    assert patch(rgba, depth, mask)[0][0, 1, 0] == 200
    # A 20-pixel hole (columns 1..20) whose background edge is column 21:
    # every column past the edge is foreground (depth 2, skipped) except one
    # background sample of level 0 at edge + k.  The kernel spans columns
    # edge .. edge + 19, so for k <= 19 the hole at distance dist from the
    # edge is the closed form 200 f / (f + (1 - f) f) = 200 / (2 - f) with
    # f = 0.5 + 0.3 dist / 20, and for k = 20 the sample is outside the
    # kernel and the fill is the edge alone.
    W = 64
    edge = 21

    def run(bg_col):
        cols = np.full(W, 100)
        depths = np.full(W, 2.0, np.float32)
        mk = np.zeros(W, np.uint8)
        cols[0], depths[0] = 50, 1.0
        mk[1:21] = 1
        depths[edge], cols[edge] = 10.0, 200
        depths[bg_col], cols[bg_col] = 10.0, 0
        return patch(*frame(cols, depths, mk))[0][0, 1:21, 0]

    dist = edge - np.arange(1, 21)
    want = np.array([np.round(200.0 / (2.0 - (0.5 + 0.3 * d / 20.0))) for d in dist])
    for k in (1, 15, 16, 19):
        assert np.array_equal(run(edge + k), want), k
    assert (run(edge + 20) == 200).all()
    assert (want < 200).all() and (want != want[0]).any()


def test_wide_disocclusion_reaches_far_samples():
    # A 300-pixel hole: a lone background sample 250 columns past the edge
    # is still inside the kernel, and the closed form above holds with
    # t = dist / 300 (the FP32 arithmetic can move a value by at most one
    # level against the real-valued closed form, at exact halves).
    W = 600
    cols = np.full(W, 100)
    depths = np.full(W, 2.0, np.float32)
    mk = np.zeros(W, np.uint8)
    cols[0], depths[0] = 50, 1.0
    mk[1:301] = 1
    edge = 301
    depths[edge], cols[edge] = 10.0, 200
    depths[edge + 250], cols[edge + 250] = 10.0, 0
    got = patch(*frame(cols, depths, mk))[0][0, 1:301, 0].astype(int)
    dist = edge - np.arange(1, 301)
    exact = 200.0 / (2.0 - (0.5 + 0.3 * dist / 300.0))
    assert np.abs(got - exact).max() <= 0.5 + 1e-4
    assert (got < 200).all()


def test_deep_kernel_weights_underflow_to_exact_zero():
    # A 400-pixel hole over a background whose rows y, y - 1, y + 1 are all
    # hits: the remaining weight shrinks by a factor in [0.2, 0.5] per
    # accepted sample, into the subnormals, until a sample's weight rounds to
    # exactly zero, after which every further weight is zero.  Levels 255 / 0
    # in alternating columns give a geometric series with a closed form.
    W, H = 900, 3
    cols = np.zeros((H, W), np.int64)
    cols[:, ::2] = 255
    depths = np.full((H, W), 10.0, np.float32)
    mk = np.zeros((H, W), np.uint8)
    mk[1, 0:400] = 1                  # hole run at the row's start: edge is R = 400
    rgba, depth, mask = frame(cols, depths, mk)
    rgba[1, 0:400] = 0
    out, z, m = patch(rgba, depth, mask)
    assert (m[1, :400] == 1).all() and (z[1, :400] == 10.0).all()
    # The edge column 400 holds 255 in all three rows; the next columns
    # alternate.  With f = 0.5 + 0.3 t the weights of the first three
    # samples (all 255) sum to 1 - (1 - f)^3, and the next three (0) only
    # add to the normaliser.  Check the leading terms against the closed
    # form of the infinite sum, which the FP32 loop reaches to within one
    # level.
    for x in (0, 100, 399):
        t = (400 - x) / 400.0
        r = 1.0 - (0.5 + 0.3 * t)      # w_rem factor per accepted sample
        # level 255 on columns 400, 402, ... (3 samples per column), 0 between:
        # sum over column pairs of r^(6p) (1 - r^3) 255, normalised by 1.
        exact = 255.0 * (1.0 - r ** 3) / (1.0 - r ** 6)
        assert abs(int(out[1, x, 0]) - exact) <= 0.5 + 1e-3, (x, out[1, x, 0], exact)


def test_uniform_background_is_reproduced_exactly():
    rng = np.random.default_rng(0)
    for level in (0, 1, 77, 128, 254, 255):
        W, H = 64, 5
        depth = np.full((H, W), 20.0, np.float32)
        mask = (rng.random((H, W)) < 0.3).astype(np.uint8)
        cols = np.full((H, W), level)
        rgba, depth, mask = frame(cols, depth, mask)
        rgba[mask != 0] = 0
        out, _, m = patch(rgba, depth, mask)
        filled = m == 1
        assert filled.any() and (out[filled][:, :3] == level).all()


def test_neighbouring_rows_are_sampled():
    # Three rows; the middle row's hole at column 1 has its edge at column 2.
    # Rows above and below hold other levels at column 2: the kernel
    # (rows y, y-1, y+1) mixes them with weights f, f(1-f), f(1-f)^2.
    cols = [[10, 10, 60, 10], [50, 0, 200, 200], [10, 10, 90, 10]]
    depths = [[10, 10, 10, 10], [1.0, np.inf, 10.0, 10.0], [10, 10, 10, 10]]
    mask = [[0, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 0]]
    out, _, _ = patch(*frame(cols, depths, mask))
    f = 0.5 + 0.3 * 1.0                       # t = 1 / 1
    w = [f, (1 - f) * f, (1 - f) ** 2 * f]     # samples: (2, y), (2, y-1), (2, y+1)
    want = round((200 * w[0] + 60 * w[1] + 90 * w[2]) / sum(w))
    assert out[1, 1, 0] == want


def test_empty_row_and_single_sided_holes():
    rgba, depth, mask = frame([[0, 0, 0], [9, 0, 0]], [[np.inf] * 3, [5.0, np.inf, np.inf]], [[1, 1, 1], [0, 1, 1]])
    out, z, m = patch(rgba, depth, mask)
    assert (m[0] == 2).all() and (out[0] == 0).all() and np.isinf(z[0]).all()
    # Row 1: only a left hit; its column is the edge, the kernel runs left.
    assert (m[1, 1:] == 1).all() and (out[1, 1:, 0] == 9).all() and (z[1, 1:] == 5.0).all()


@pytest.mark.parametrize("spec_fn", [config1_frame, config2_frame])
def test_patcher_agrees_with_plain_fill_except_colour(spec_fn):
    spec = spec_fn(0)
    r, d = spec.render_source()
    plain = O.reproject(r, d, spec.baseline_m, spec.focal_px, spec.target_eye, O.FILL_NEAREST_BG)
    pat = O.reproject(r, d, spec.baseline_m, spec.focal_px, spec.target_eye, O.FILL_PATCHER)
    assert np.array_equal(plain[2], pat[2])                       # same holes, same mask values
    assert np.array_equal(plain[1].view(np.uint32), pat[1].view(np.uint32))  # edge depth = plain choice
    hits = plain[2] == 0
    assert np.array_equal(plain[0][hits], pat[0][hits])           # hits untouched
    assert np.array_equal(plain[0][..., 3], pat[0][..., 3])       # alpha from the edge
    holes = plain[2] == 1
    assert (plain[0][holes] != pat[0][holes]).any()               # and the colours do change


def test_mirror_symmetry_between_eyes():
    r, d = synth.random_frame(3, 96, 24, depth_levels=6, zmin=0.5, zmax=8.0)
    B, f = 0.064, 200.0
    right = O.reproject(r, d, B, f, O.TARGET_RIGHT, O.FILL_PATCHER)
    left_of_mirror = O.reproject(r[:, ::-1].copy(), d[:, ::-1].copy(), B, f, O.TARGET_LEFT, O.FILL_PATCHER)
    assert np.array_equal(right[0], left_of_mirror[0][:, ::-1])
    assert np.array_equal(right[2], left_of_mirror[2][:, ::-1])
