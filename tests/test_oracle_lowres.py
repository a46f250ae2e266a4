"""Pins of the oracle's reprojection through a downsampled intermediate buffer
(Section 6 (c) resolution-independent buffers, (d) linear interpolation along
the row), under the readings stated in oracle/reproject.c:

- scale 1 is the direct path, bit for bit;
- the texel scatter is the direct path run on the frame of block centres with
  focal length f / k (exact for a power-of-two k), and every full-resolution
  pixel samples the source column its texel's disparity names;
- the fill is the direct path's fill applied to the unfilled result;
- hand-worked rows for the interpolated shift, for both eyes, and the
  one-surface rule that turns it off across a depth step.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import reproject as O
from paper_2506_15183_amd.scenes import config1_frame, synth

SCALES = (1, 2, 4, 8, 16)


def lowres(r, d, B, f, eye, fill, k, linear):
    return O.reproject_lowres(r, d, B, f, eye, fill, k, linear)


@pytest.mark.parametrize("eye", [O.TARGET_RIGHT, O.TARGET_LEFT])
@pytest.mark.parametrize("fill", [O.FILL_NONE, O.FILL_NEAREST_BG])
@pytest.mark.parametrize("linear", [False, True])
def test_scale_one_is_the_direct_path(eye, fill, linear):
    frames = [synth.random_frame(11, 97, 13, depth_levels=5, special_frac=0.1, zmin=0.05, zmax=5.0),
              synth.random_frame(12, 64, 7, zmin=0.3, zmax=50.0)]
    spec = config1_frame(0)
    frames.append(spec.render_source())
    for (r, d) in frames:
        want = O.reproject(r, d, 0.064, 200.0, eye, fill)
        got = lowres(r, d, 0.064, 200.0, eye, fill, 1, linear)
        assert np.array_equal(got[0], want[0])
        assert np.array_equal(got[1].view(np.uint32), want[1].view(np.uint32))
        assert np.array_equal(got[2], want[2])


@pytest.mark.parametrize("k", [2, 4, 8, 16])
@pytest.mark.parametrize("eye", [O.TARGET_RIGHT, O.TARGET_LEFT])
def test_texels_follow_the_direct_path_on_block_centres(k, eye):
    """Without interpolation: texel (i, j) is pixel (k i + k/2, k j + k/2),
    its record is what the direct path gives the small frame of those pixels
    with focal f / k (B f / k / z = (B f / z) / k exactly for a power of two,
    and q / k < W / k iff q < W), and pixel (x, y) of block (i, j) takes the
    source column x -+ roundf(B f / z) of that record's depth, or is a hole
    when that column is off the row."""
    W, H, B, f = 16 * 12, 16 * 3, 0.064, 200.0
    r, d = synth.random_frame(20 + k, W, H, depth_levels=7, special_frac=0.05, zmin=0.2, zmax=8.0)
    c = k // 2
    sr = np.ascontiguousarray(r[c::k, c::k])
    sd = np.ascontiguousarray(d[c::k, c::k])
    _, zs, ms = O.reproject(sr, sd, B, f / k, eye, O.FILL_NONE)
    out, z, m = lowres(r, d, B, f, eye, O.FILL_NONE, k, False)
    sign = 1 if eye == O.TARGET_RIGHT else -1
    checked = 0
    for y in range(H):
        for x in range(W):
            i, j = x // k, y // k
            if ms[j, i] != 0:
                assert m[y, x] == 1 and np.isinf(z[y, x]) and not out[y, x].any()
                continue
            dd = O.disparity(float(zs[j, i]), B, f, W)
            assert dd is not None
            xs = x + sign * dd
            if not 0 <= xs < W:
                assert m[y, x] == 1
                continue
            assert m[y, x] == 0
            assert z[y, x].view(np.uint32) == zs[j, i].view(np.uint32)
            assert np.array_equal(out[y, x], r[y, xs])
            checked += 1
    assert checked > W * H // 3


@pytest.mark.parametrize("k", SCALES)
@pytest.mark.parametrize("eye", [O.TARGET_RIGHT, O.TARGET_LEFT])
def test_fill_is_the_direct_fill_of_the_unfilled_result(k, eye):
    r, d = synth.random_frame(40 + k, 150, 37, depth_levels=9, special_frac=0.02, zmin=0.1, zmax=10.0)
    for linear in (False, True):
        raw = lowres(r, d, 0.064, 200.0, eye, O.FILL_NONE, k, linear)
        filled = lowres(r, d, 0.064, 200.0, eye, O.FILL_NEAREST_BG, k, linear)
        want = O.fill_holes(*raw, eye, O.FILL_NEAREST_BG)
        for a, b in zip(filled, want):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def worked_frame(zs_by_block, k, W, H, bf_depth_scale=1.0):
    """Rows of W pixels whose k-blocks hold the given depths; colour R of
    pixel (x, y) is 10 y + x so a sampled column can be read back."""
    d = np.repeat(np.asarray(zs_by_block, np.float32), k)[None, :].repeat(H, axis=0)
    r = np.zeros((H, W, 4), np.uint8)
    r[..., 0] = (10 * np.arange(H)[:, None] + np.arange(W)[None, :]).astype(np.uint8)
    r[..., 3] = 255
    return r, np.ascontiguousarray(d)


def sampled_columns(out, m, y):
    return [int(out[y, x, 0]) - 10 * y if m[y, x] == 0 else None for x in range(out.shape[1])]


def test_interpolated_shift_worked_example_right_eye():
    # B f = 19; depths 4.75 (q = 4) and 4 (q = 4.75), both exact.  k = 4,
    # texel centres at x = 2, 6, 10, 14; texel disparity roundf(q / 4) = 1,
    # so texels 1, 2, 3 land on 0, 1, 2 and target texel 3 is empty.
    # Shifts of target texels 0, 1, 2: 4, 4.75, 4.75.  Pixel x reads
    # u = (x - 2) / 4; e.g. x = 4: f = 0.5, s = 4 + 0.5 * 0.75 = 4.375 -> 4,
    # column 8 (the nearest texel alone gives 4.75 -> 5, column 9).  x = 10:
    # texel 3 is empty, no interpolation, 4.75 -> 5, column 15; x = 11 would
    # read column 16, off the row.
    r, d = worked_frame([4.75, 4.75, 4.0, 4.0], 4, 16, 4)
    lin = lowres(r, d, 1.0, 19.0, O.TARGET_RIGHT, O.FILL_NONE, 4, True)
    near = lowres(r, d, 1.0, 19.0, O.TARGET_RIGHT, O.FILL_NONE, 4, False)
    tail = [None] * 5
    for y in range(4):
        assert sampled_columns(lin[0], lin[2], y) == [4, 5, 6, 7, 8, 10, 11, 12, 13, 14, 15] + tail
        assert sampled_columns(near[0], near[2], y) == [4, 5, 6, 7, 9, 10, 11, 12, 13, 14, 15] + tail
    # Depth is the nearest texel's: target texel 0 holds source texel 1
    # (4.75), texels 1 and 2 hold 4.0.
    assert list(lin[1][0, :11]) == [4.75] * 4 + [4.0] * 7
    assert np.isinf(lin[1][0, 11:]).all() and (lin[2][0, 11:] == 1).all()


def test_interpolated_shift_worked_example_left_eye():
    # Same frame, left eye: texels 0, 1, 2 land on 1, 2, 3; target texel 0 is
    # empty.  Shifts of target texels 1, 2, 3: 4, 4, 4.75; source column
    # x - roundf(s).  x = 12: f = 0.5 between texels 2 and 3, s = 4.375 -> 4,
    # column 8 (nearest: texel 3, 4.75 -> 5, column 7).
    r, d = worked_frame([4.75, 4.75, 4.0, 4.0], 4, 16, 4)
    lin = lowres(r, d, 1.0, 19.0, O.TARGET_LEFT, O.FILL_NONE, 4, True)
    near = lowres(r, d, 1.0, 19.0, O.TARGET_LEFT, O.FILL_NONE, 4, False)
    head = [None] * 4
    for y in range(4):
        assert sampled_columns(lin[0], lin[2], y) == head + [0, 1, 2, 3, 4, 5, 6, 7, 8, 8, 9, 10]
        assert sampled_columns(near[0], near[2], y) == head + [0, 1, 2, 3, 4, 5, 6, 7, 7, 8, 9, 10]


def test_no_interpolation_across_a_depth_step():
    # B f = 24: depths 6 (q = 4) and 4 (q = 6) differ by 2 pixels of shift,
    # more than one surface allows: the interpolated path is the nearest one.
    r, d = worked_frame([6.0, 6.0, 4.0, 4.0, 6.0, 6.0, 4.0, 4.0], 4, 32, 4)
    lin = lowres(r, d, 1.0, 24.0, O.TARGET_RIGHT, O.FILL_NONE, 4, True)
    near = lowres(r, d, 1.0, 24.0, O.TARGET_RIGHT, O.FILL_NONE, 4, False)
    for a, b in zip(lin, near):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    # ... while a one-pixel step is interpolated.
    r, d = worked_frame([6.0, 6.0, 4.8, 4.8, 6.0, 6.0, 4.8, 4.8], 4, 32, 4)
    lin = lowres(r, d, 1.0, 24.0, O.TARGET_RIGHT, O.FILL_NONE, 4, True)
    near = lowres(r, d, 1.0, 24.0, O.TARGET_RIGHT, O.FILL_NONE, 4, False)
    assert not np.array_equal(lin[0], near[0])


@pytest.mark.parametrize("k", [2, 4, 8, 16])
def test_ragged_frame_edges(k):
    # Widths and heights that are not multiples of k: the last block is cut,
    # its centre clamped to the frame; every output is still defined and
    # hits carry a source pixel of their own row.
    W, H = 16 * 5 + 3, 2 * k + 1
    r, d = synth.random_frame(60 + k, W, H, depth_levels=4, zmin=0.3, zmax=6.0)
    out, z, m = lowres(r, d, 0.064, 200.0, O.TARGET_RIGHT, O.FILL_NONE, k, True)
    assert set(np.unique(m)) <= {0, 1}
    for y in range(H):
        row = {bytes(r[y, x]) for x in range(W)}
        for x in np.nonzero(m[y] == 0)[0]:
            assert bytes(out[y, x]) in row
    # The last block row is cut to the single row H - 1 and its centre is
    # clamped to it: that row comes out as the one-row frame of itself.
    one = lowres(r[H - 1:], d[H - 1:], 0.064, 200.0, O.TARGET_RIGHT, O.FILL_NONE, k, True)
    assert np.array_equal(out[H - 1], one[0][0]) and np.array_equal(m[H - 1], one[2][0])


def test_constant_depth_plane_is_a_uniform_shift():
    # One depth everywhere: every texel shifts by roundf(q / k), every pixel
    # of a hit block samples x + roundf(q): the direct path's image wherever
    # the block is hit.
    W, H, B, f, z = 128, 16, 0.064, 200.0, 0.6
    rng = np.random.default_rng(5)
    r = rng.integers(0, 256, (H, W, 4), dtype=np.uint8)
    d = np.full((H, W), z, np.float32)
    direct = O.reproject(r, d, B, f, O.TARGET_RIGHT, O.FILL_NONE)
    dd = O.disparity(z, B, f, W)
    for k in SCALES:
        dk = O.disparity(z, B, f / k, W // k)
        out, zz, m = lowres(r, d, B, f, O.TARGET_RIGHT, O.FILL_NONE, k, True)
        for x in range(W):
            hit_block = x // k + dk < W // k
            hit = hit_block and x + dd < W
            assert (m[:, x] == (0 if hit else 1)).all()
            if hit:
                assert np.array_equal(out[:, x], direct[0][:, x])


def test_bad_scale_is_rejected():
    r, d = synth.random_frame(1, 8, 8)
    for k in (0, 3, 32, -2):
        with pytest.raises(ValueError):
            lowres(r, d, 0.064, 200.0, O.TARGET_RIGHT, O.FILL_NONE, k, True)


def test_a_shift_of_a_full_row_is_never_splatted():
    # A ragged width (83 = 5 * 16 + 3) lets roundf(q / 16) fall inside the
    # buffer row for q just past the frame width: the direct path's rule
    # (q < W) skips such a texel, and any pixel that read its shift would
    # sample a column off the row, so every pixel is a hole.  Just below the
    # width the shift reaches the far edge of the row.
    W, H, B, f = 83, 4, 0.064, 200.0
    bf = np.float32(np.float32(B) * np.float32(f))
    r = np.full((H, W, 4), 9, np.uint8)
    for q, any_hit in ((83.5, False), (78.0, True)):
        z = np.float32(bf / np.float32(q))
        d = np.full((H, W), z, np.float32)
        for eye in (O.TARGET_RIGHT, O.TARGET_LEFT):
            _, _, m = lowres(r, d, B, f, eye, O.FILL_NONE, 16, True)
            assert (m == 0).any() == any_hit
