"""GPU tests of the serving loop (yoro_serve_run): every admitted frame is
processed, a frame's result inside a mixed batch equals the same frame warped
alone (bit-exact), the learned refinement runs under its policy and equals
the stand-alone tiled learned fill, the fallback keeps the plain fill, and
rejected headsets are not processed."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _mods():
    import torch

    from paper_2506_15183_amd import serve, unet, yoro
    from paper_2506_15183_amd.scenes.configs import HeadsetSpec, FrameSpec

    return torch, serve, unet, yoro, HeadsetSpec, FrameSpec


SIZES = ((256, 256), (320, 264), (384, 256))


def _headsets(HeadsetSpec, n, rates=(240.0, 300.0, 200.0)):
    out = []
    for i in range(n):
        w, h = SIZES[i % len(SIZES)]
        out.append(HeadsetSpec(i, rates[i % len(rates)], w, h, i % 2, 0.06 + 0.002 * i, 700.0 + 40 * i,
                               0.0005 * i))
    return out


def _frames(FrameSpec):
    cache = {}

    def frames(h, slot):
        key = (h.width, h.height, h.target_eye, slot)
        if key not in cache:
            spec = FrameSpec(h.width, h.height, 0.063, 900.0, h.target_eye, 40, 0.3, 50.0, True, (4, 32),
                             1000 + hash(key) % 100000)
            cache[key] = spec.render_source()
        return cache[key]

    return frames


def _last_per_output(trace, res, n_outputs, n_headsets):
    """(headset, output) -> index of the last processed arrival written there."""
    last = {}
    count = [0] * n_headsets
    for k in range(len(trace)):
        if res["path"][k] == 4:
            continue
        h = int(trace["headset"][k])
        last[(h, count[h] % n_outputs)] = k
        count[h] += 1
    return last


def _plain_alone(yoro, srv, h, slot):
    src_rgba, src_depth = srv.pools[h.index][slot]
    return yoro.reproject(src_rgba, src_depth, h.baseline_m, h.focal_px, h.target_eye, yoro.FILL_NEAREST_BG)


def test_plain_serving_processes_every_frame_and_matches_alone(cuda):
    torch, serve, unet, yoro, HeadsetSpec, FrameSpec = _mods()
    hs = _headsets(HeadsetSpec, 6)
    cfg = serve.Config(budget_bytes=10**10, n_sources=3, n_outputs=2, max_batch=4, max_in_flight=2)
    srv = serve.Server(hs, cfg, _frames(FrameSpec))
    trace = serve.make_trace(hs, 0.5, cfg.n_sources, seed=1)
    res = srv.run(trace, serve.PLAIN)
    assert (res["path"] == serve.PATH_PLAIN).all()
    t = trace["t_ns"]
    assert (res["launch_ns"] >= t).all() and (res["done_ns"] >= res["launch_ns"]).all()
    assert (res["batch_frames"] >= 1).all() and (res["batch_frames"] <= cfg.max_batch).all()
    lat = (res["done_ns"] - t) / 1e6
    assert lat.max() < 200.0, lat.max()
    s = serve.summarize(trace, res, hs, 0.5)
    assert s["processed"] == len(trace) and s["p99_ms"] >= s["p50_ms"] > 0
    for (hi, o), k in _last_per_output(trace, res, cfg.n_outputs, len(hs)).items():
        h = hs[hi]
        want = _plain_alone(yoro, srv, h, int(trace["source"][k]))
        got = srv.outs[hi][o]
        for g, w in zip(got, want):
            assert torch.equal(g, w), (hi, o, k)


def test_burst_arrivals_batch_together_and_match_alone(cuda):
    """Eight headsets of three resolutions whose frames arrive in bursts at
    the same instants: the loop batches frames of different sizes into one
    launch (some batches hold three or more frames), and every frame's
    result equals the same frame warped alone, bit for bit."""
    torch, serve, unet, yoro, HeadsetSpec, FrameSpec = _mods()
    hs = _headsets(HeadsetSpec, 8, rates=(50.0,))
    bursts = 4  # YORO_SERVE_MAX_OUTPUTS: each arrival keeps its own output set
    cfg = serve.Config(budget_bytes=10**10, n_sources=3, n_outputs=bursts, max_batch=8, max_in_flight=1)
    srv = serve.Server(hs, cfg, _frames(FrameSpec))
    trace = np.zeros(bursts * len(hs), serve.ARRIVAL_DTYPE)
    for b in range(bursts):
        for i in range(len(hs)):
            a = trace[b * len(hs) + i]
            a["t_ns"] = 10_000_000 + b * 20_000_000  # every headset at the same instant
            a["headset"] = i
            a["source"] = (b + i) % cfg.n_sources
    res = srv.run(trace, serve.PLAIN)
    assert (res["path"] == serve.PATH_PLAIN).all()
    assert (res["batch_frames"] >= 3).sum() >= 3, res["batch_frames"]
    # A batch mixes resolutions: some launch holds frames of two sizes or more.
    mixed = False
    for t in np.unique(res["launch_ns"]):
        sizes = {(hs[int(h)].width, hs[int(h)].height) for h in trace["headset"][res["launch_ns"] == t]}
        mixed |= len(sizes) >= 2
    assert mixed
    # Each arrival has its own output set (n_outputs = bursts): check every frame.
    count = [0] * len(hs)
    for k in range(len(trace)):
        hi = int(trace["headset"][k])
        o = count[hi] % cfg.n_outputs
        count[hi] += 1
        want = _plain_alone(yoro, srv, hs[hi], int(trace["source"][k]))
        for g, w in zip(srv.outs[hi][o], want):
            assert torch.equal(g, w), (hi, o, k, int(res["batch_frames"][k]))


def test_admission_rejects_what_does_not_fit(cuda):
    torch, serve, unet, yoro, HeadsetSpec, FrameSpec = _mods()
    hs = _headsets(HeadsetSpec, 3)
    cfg = serve.Config(n_sources=2, n_outputs=1, max_batch=2, max_in_flight=2)
    need = [serve.headset_bytes(h, 2, 1) for h in hs]
    probe = serve.Server(hs[:1], serve.Config(budget_bytes=10**10, n_sources=2, n_outputs=1, max_batch=2,
                                              max_in_flight=2), _frames(FrameSpec))
    cfg.budget_bytes = probe.ws_bytes + need[0] + need[1] + need[2] - 1  # one byte short for the last
    srv = serve.Server(hs, cfg, _frames(FrameSpec))
    assert srv.admitted.tolist() == [True, True, False]
    trace = serve.make_trace(hs, 0.2, cfg.n_sources, seed=2)
    res = srv.run(trace, serve.PLAIN)
    rejected = trace["headset"] == 2
    assert (res["path"][rejected] == serve.PATH_REJECTED).all()
    assert (res["path"][~rejected] == serve.PATH_PLAIN).all() and (res["done_ns"][~rejected] > 0).all()


def _strong_net(unet, seed):
    p = unet.init_params(seed)
    p[-1] = p[-1] * 100.0
    return unet.UNet("cuda", params=p)


def _learned_want(net, cfg, rgba, depth, mask):
    """The stand-alone learned fill the loop's refinement must equal: hole
    tiles, or full-width bands."""
    if cfg.band > 0:
        return net.fill_bands(rgba, depth, mask, band=cfg.band, halo=cfg.halo)
    return net.fill_tiles(rgba, depth, mask, chunk=cfg.chunk)[0]


@pytest.mark.parametrize("band", [0, 256])
def test_learned_policy_refines_and_falls_back(cuda, band):
    torch, serve, unet, yoro, HeadsetSpec, FrameSpec = _mods()
    hs = _headsets(HeadsetSpec, 4, rates=(60.0, 50.0, 40.0))
    net = _strong_net(unet, 8)
    cfg = serve.Config(budget_bytes=10**10, n_sources=2, n_outputs=2, max_batch=4, max_in_flight=2, chunk=4,
                       learned_max_hole_fraction=1.0, band=band)
    srv = serve.Server(hs, cfg, _frames(FrameSpec), model=net)
    trace = serve.make_trace(hs, 0.4, cfg.n_sources, seed=3)
    res = srv.run(trace, serve.LEARNED)
    paths = res["path"]
    assert np.isin(paths, [serve.PATH_LEARNED, serve.PATH_BUSY]).all()
    assert (paths == serve.PATH_LEARNED).sum() >= 1
    counted = res["holes"] >= 0
    assert (res["holes"][counted] > 0).all() and (res["holes"][paths == serve.PATH_LEARNED] > 0).all()
    assert (res["done_ns"] >= res["launch_ns"]).all()
    checked = 0
    for (hi, o), k in _last_per_output(trace, res, cfg.n_outputs, len(hs)).items():
        h = hs[hi]
        rgba, depth, mask = _plain_alone(yoro, srv, h, int(trace["source"][k]))
        if res["holes"][k] >= 0:
            assert int(res["holes"][k]) == int((mask != 0).sum())
        if paths[k] == serve.PATH_LEARNED:
            want = _learned_want(net, cfg, rgba, depth, mask)
            checked += 1
        else:
            want = rgba
        got = srv.outs[hi][o]
        assert torch.equal(got[0], want), (hi, o, k, int(paths[k]))
        assert torch.equal(got[1], depth) and torch.equal(got[2], mask)
    assert checked >= 1
    # Threshold 0: every frame with a hole falls back to the plain fill.
    srv.cfg.learned_max_hole_fraction = 0.0
    res0 = srv.run(trace, serve.LEARNED)
    assert (res0["path"] == serve.PATH_FALLBACK).all()
    for (hi, o), k in _last_per_output(trace, res0, cfg.n_outputs, len(hs)).items():
        want = _plain_alone(yoro, srv, hs[hi], int(trace["source"][k]))[0]
        assert torch.equal(srv.outs[hi][o][0], want)


def test_refinement_interval_budget(cuda):
    """Refinements start at least learned_min_interval_ns apart: over a
    trace shorter than the interval exactly one frame is refined."""
    torch, serve, unet, yoro, HeadsetSpec, FrameSpec = _mods()
    hs = _headsets(HeadsetSpec, 3, rates=(120.0, 90.0, 72.0))
    net = _strong_net(unet, 9)
    cfg = serve.Config(budget_bytes=10**10, n_sources=2, n_outputs=2, max_batch=4, max_in_flight=2, chunk=4,
                       learned_max_hole_fraction=1.0, learned_min_interval_ms=10_000.0)
    srv = serve.Server(hs, cfg, _frames(FrameSpec), model=net)
    trace = serve.make_trace(hs, 0.3, cfg.n_sources, seed=4)
    res = srv.run(trace, serve.LEARNED)
    assert (res["path"] == serve.PATH_LEARNED).sum() == 1
    assert ((res["path"] == serve.PATH_LEARNED) | (res["path"] == serve.PATH_BUSY)).all()
    assert (res["done_ns"] >= res["launch_ns"]).all()


@pytest.mark.parametrize("band", [0, 256])
def test_progressive_refinement_releases_at_the_warp(cuda, band):
    """Progressive mode: every frame is released with the plain fill when its
    warp completes (done_ns); a refined frame is upgraded in place later
    (refined_ns), and the output it leaves equals the stand-alone tiled
    learned fill."""
    torch, serve, unet, yoro, HeadsetSpec, FrameSpec = _mods()
    hs = _headsets(HeadsetSpec, 4, rates=(60.0, 50.0, 40.0))
    net = _strong_net(unet, 8)
    cfg = serve.Config(budget_bytes=10**10, n_sources=2, n_outputs=2, max_batch=4, max_in_flight=2, chunk=4,
                       learned_max_hole_fraction=1.0, progressive=True, band=band)
    srv = serve.Server(hs, cfg, _frames(FrameSpec), model=net)
    trace = serve.make_trace(hs, 0.4, cfg.n_sources, seed=3)
    res = srv.run(trace, serve.LEARNED)
    paths = res["path"]
    refined = paths == serve.PATH_LEARNED
    assert np.isin(paths, [serve.PATH_LEARNED, serve.PATH_BUSY]).all() and refined.sum() >= 1
    assert (res["done_ns"] >= res["launch_ns"]).all()
    assert (res["refined_ns"][refined] > res["done_ns"][refined]).all()
    assert (res["refined_ns"][~refined] == -1).all()
    checked = 0
    for (hi, o), k in _last_per_output(trace, res, cfg.n_outputs, len(hs)).items():
        rgba, depth, mask = _plain_alone(yoro, srv, hs[hi], int(trace["source"][k]))
        want = _learned_want(net, cfg, rgba, depth, mask) if refined[k] else rgba
        checked += int(refined[k])
        assert torch.equal(srv.outs[hi][o][0], want), (hi, o, k, int(paths[k]))
    assert checked >= 1
    s = serve.summarize(trace, res, hs, 0.4)
    assert s["refined_upgrade_p50_ms"] > 0 and s["refined_fraction"] > 0
