"""GPU parity of the reprojection through a downsampled intermediate buffer
(yoro_reproject_lowres, yoro_stereo_batch_launch_lowres) against the oracle,
bit-exact: every RGBA byte, depth bit and mask byte.  Scales 1-16, with and
without the interpolated shift, both eyes, every fill mode, ray-cast scenes,
random frames with forced collisions, special depths and ragged widths and
heights, tall frames (units of several rows), the 64-frame mixed batch, graph
replay and the skipped-row count."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import reproject as orc
from paper_2506_15183_amd.scenes import synth
from paper_2506_15183_amd.scenes.configs import config1_frame, config2_frame, config3_frames

pytestmark = pytest.mark.gpu

R, L = 0, 1
SCALES = (1, 2, 4, 8, 16)


def _gpu():
    import torch

    from paper_2506_15183_amd import yoro

    return torch, yoro


def run_gpu(rgba, depth, B, f, eye, fill, k, linear, with_depth=True, with_mask=True):
    torch, yoro = _gpu()
    a = torch.from_numpy(np.ascontiguousarray(rgba)).cuda()
    d = torch.from_numpy(np.ascontiguousarray(depth)).cuda()
    out = yoro.reproject_lowres(a, d, B, f, eye, fill, k, linear, with_depth=with_depth, with_mask=with_mask)
    torch.cuda.synchronize()
    return tuple(None if t is None else t.cpu().numpy() for t in out)


def oracle(rgba, depth, B, f, eye, fill, k, linear):
    if fill == orc.FILL_PATCHER:
        raw = orc.reproject_lowres(rgba, depth, B, f, eye, orc.FILL_NONE, k, linear)
        return orc.fill_holes(*raw, eye, orc.FILL_PATCHER)
    return orc.reproject_lowres(rgba, depth, B, f, eye, fill, k, linear)


def assert_same(g, o, what=""):
    go, gz, gm = g
    oo, oz, om = o
    assert np.array_equal(go, oo), f"rgba differs {what}: {np.argwhere(np.any(go != oo, axis=-1))[:5]}"
    if gz is not None:
        assert np.array_equal(gz.view(np.uint32), oz.view(np.uint32)), f"depth differs {what}"
    if gm is not None:
        assert np.array_equal(gm, om), f"mask differs {what}"


@pytest.mark.parametrize("spec_fn", [config1_frame, config2_frame])
@pytest.mark.parametrize("k", SCALES)
def test_scenes(cuda, spec_fn, k):
    spec = spec_fn(0)
    rgba, depth = spec.render_source()
    for eye in (R, L):
        for linear in (False, True):
            g = run_gpu(rgba, depth, spec.baseline_m, spec.focal_px, eye, orc.FILL_NEAREST_BG, k, linear)
            o = oracle(rgba, depth, spec.baseline_m, spec.focal_px, eye, orc.FILL_NEAREST_BG, k, linear)
            assert_same(g, o, f"{spec_fn.__name__} k={k} eye={eye} linear={linear}")


# Widths across wave (64), workgroup (256) and pixels-per-thread boundaries
# and the maximum; heights cut the last block row.
WIDTHS = [1, 2, 17, 63, 64, 65, 257, 1000, 1832, 2160, 4097, 8192]


@pytest.mark.parametrize("W", WIDTHS)
def test_random_frames(cuda, W):
    for k in SCALES:
        H = 2 * k + 3 if W <= 2160 else k + 1
        for case, (levels, special) in enumerate([(3, 0.0), (None, 0.08), (7, 0.02)]):
            rgba, depth = synth.random_frame(900 + 7 * W + 31 * k + case, W, H, depth_levels=levels,
                                             special_frac=special, zmin=0.05 if W > 512 else 0.3, zmax=30.0)
            for eye in (R, L):
                fill = orc.FILL_NEAREST_BG if case != 1 else orc.FILL_NONE
                linear = (case + eye) % 2 == 0
                g = run_gpu(rgba, depth, 0.063, 900.0, eye, fill, k, linear)
                o = oracle(rgba, depth, 0.063, 900.0, eye, fill, k, linear)
                assert_same(g, o, f"W={W} H={H} k={k} case={case} eye={eye}")


def test_scale_one_is_the_direct_kernel(cuda):
    torch, yoro = _gpu()
    spec = config2_frame(2)
    rgba, depth = spec.render_source()
    a = torch.from_numpy(rgba).cuda()
    d = torch.from_numpy(depth).cuda()
    for eye in (R, L):
        direct = yoro.reproject(a, d, spec.baseline_m, spec.focal_px, eye, yoro.FILL_NEAREST_BG)
        low = yoro.reproject_lowres(a, d, spec.baseline_m, spec.focal_px, eye, yoro.FILL_NEAREST_BG, 1, True)
        torch.cuda.synchronize()
        for x, y in zip(direct, low):
            assert torch.equal(x.view(torch.uint8), y.view(torch.uint8))


def test_patcher_fill_and_optional_outputs(cuda):
    spec = config1_frame(1)
    rgba, depth = spec.render_source()
    for k in (2, 8):
        for eye in (R, L):
            g = run_gpu(rgba, depth, spec.baseline_m, spec.focal_px, eye, orc.FILL_PATCHER, k, True)
            o = oracle(rgba, depth, spec.baseline_m, spec.focal_px, eye, orc.FILL_PATCHER, k, True)
            assert_same(g, o, f"patcher k={k} eye={eye}")
    g = run_gpu(rgba, depth, spec.baseline_m, spec.focal_px, R, orc.FILL_NEAREST_BG, 4, True, False, False)
    o = oracle(rgba, depth, spec.baseline_m, spec.focal_px, R, orc.FILL_NEAREST_BG, 4, True)
    assert g[1] is None and g[2] is None and np.array_equal(g[0], o[0])


def test_degenerate_rows_and_tall_frames(cuda):
    W, H = 700, 32
    rgba, depth = synth.random_frame(6, W, H)
    depth[0:8, :] = np.nan        # a block row with no geometry
    depth[8:16, :] = np.inf       # identity
    depth[16:24, :] = 1e-30       # every shift beyond the row
    depth[24:28, ::2] = -2.0
    depth[28:, :] = 0.2
    for k in SCALES:
        for eye in (R, L):
            for fill in (orc.FILL_NONE, orc.FILL_NEAREST_BG):
                assert_same(run_gpu(rgba, depth, 0.063, 900.0, eye, fill, k, True),
                            oracle(rgba, depth, 0.063, 900.0, eye, fill, k, True), f"k={k} eye={eye} fill={fill}")
    # Tall frames: enough block rows that a unit spans several rows.
    for (W, H, k) in [(40, 12000, 2), (33, 16384, 4), (96, 16000, 16)]:
        rgba, depth = synth.random_frame(W + k, W, H, depth_levels=5, zmin=0.1, zmax=4.0)
        assert_same(run_gpu(rgba, depth, 0.064, 200.0, R, 1, k, True),
                    oracle(rgba, depth, 0.064, 200.0, R, 1, k, True), f"{W}x{H} k={k}")
    rgba, depth = synth.random_frame(8, 1, 1)
    assert_same(run_gpu(rgba, depth, 0.064, 200.0, L, 1, 16, True), oracle(rgba, depth, 0.064, 200.0, L, 1, 16, True))


def test_deterministic_repeats(cuda):
    rgba, depth = synth.random_frame(3, 1832, 64, depth_levels=3, zmin=0.05, zmax=1.0)
    first = run_gpu(rgba, depth, 0.063, 900.0, R, 1, 4, True)
    for _ in range(4):
        assert_same(run_gpu(rgba, depth, 0.063, 900.0, R, 1, 4, True), first)


def _batch(specs):
    torch, yoro = _gpu()
    frames, dev = [], []
    for s in specs:
        rgba, depth = s.render_source()
        frames.append((rgba, depth))
        H, W = depth.shape
        dev.append((torch.from_numpy(rgba).cuda(), torch.from_numpy(depth).cuda(),
                    torch.empty((H, W, 4), dtype=torch.uint8, device="cuda"),
                    torch.empty((H, W), dtype=torch.float32, device="cuda"),
                    torch.empty((H, W), dtype=torch.uint8, device="cuda")))
    return frames, dev


@pytest.mark.parametrize("k,linear", [(2, True), (4, False), (16, True)])
def test_batch_mixed_resolutions(cuda, k, linear):
    """Every frame of the 64-frame mixed-resolution batch, bit-exact."""
    torch, yoro = _gpu()
    specs = config3_frames()
    frames, dev = _batch(specs)
    jobs = [yoro.make_job(d[0], d[1], d[2], d[3], d[4], s.baseline_m, s.focal_px, L if i % 3 == 0 else R, 1)
            for i, (s, d) in enumerate(zip(specs, dev))]
    batch = yoro.StereoBatch(jobs)
    batch.prepare()
    batch.launch_lowres(k, linear)
    torch.cuda.synchronize()
    assert batch.errors() == 0
    for i, (s, (rgba, depth), d) in enumerate(zip(specs, frames, dev)):
        o = orc.reproject_lowres(rgba, depth, s.baseline_m, s.focal_px, L if i % 3 == 0 else R, 1, k, linear)
        assert_same(tuple(x.cpu().numpy() for x in d[2:]), o, f"frame {i} {s.width}x{s.height}")


def test_batch_graph_replay_and_skipped_rows(cuda):
    torch, yoro = _gpu()
    specs = config3_frames(n_per_size=1)
    frames, dev = _batch(specs)
    jobs = [yoro.make_job(d[0], d[1], d[2], d[3], d[4], s.baseline_m, s.focal_px, R, 1)
            for s, d in zip(specs, dev)]
    batch = yoro.StereoBatch(jobs)
    want = [orc.reproject_lowres(r, z, s.baseline_m, s.focal_px, R, 1, 8, True) for s, (r, z) in zip(specs, frames)]
    st = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        batch.prepare(stream=st)
        batch.launch_lowres(8, True, stream=st)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=st):
            batch.prepare(stream=st)
            batch.launch_lowres(8, True, stream=st)
    for rep in range(3):
        for d in dev:
            d[2].zero_(); d[3].zero_(); d[4].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for w, d in zip(want, dev):
            assert_same(tuple(x.cpu().numpy() for x in d[2:]), w, f"replay {rep}")
    # A launch laid out for narrower rows skips (and counts) the wider frames' rows.
    batch.prepare()
    batch.launch_lowres(8, True, max_width=1024)
    torch.cuda.synchronize()
    assert batch.errors() == sum(s.height for s in specs if s.width > 1024)
