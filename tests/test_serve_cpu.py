"""Host logic of the serving loop: admission under a budget, the arrival
trace, the headset recipe, workspace sizing and argument checks (no GPU)."""
from __future__ import annotations

import collections
import ctypes

import numpy as np
import pytest

from paper_2506_15183_amd import serve, yoro
from paper_2506_15183_amd.scenes.configs import SERVE_SIZES, config5_headsets


def test_admission_is_greedy_in_order_within_the_budget():
    assert serve.admit([3, 4, 5, 1], 10, 1).tolist() == [True, True, False, True]
    assert serve.admit([3, 4, 5, 1], 100).all()
    assert not serve.admit([3, 4], 2).any()
    assert serve.admit([], 10).size == 0
    assert serve.admit([5, 5], 10, 0).all() and serve.admit([5, 5], 10, 1).tolist() == [True, False]
    with pytest.raises(ValueError):
        serve.admit([1], -1)
    # The recipe's 32 headsets do not all fit 8 GB: admission binds.
    hs = config5_headsets()
    need = [serve.headset_bytes(h, 8, 3) for h in hs]
    ok = serve.admit(need, 8 * 10**9)
    assert 0 < ok.sum() < len(hs) and sum(np.array(need)[ok]) <= 8 * 10**9


def test_headset_recipe_is_balanced_and_seeded():
    hs = config5_headsets(32, seed=0)
    assert collections.Counter(h.rate_hz for h in hs) == {72.0: 11, 90.0: 11, 120.0: 10}
    assert collections.Counter((h.width, h.height) for h in hs) == {s: n for s, n in zip(SERVE_SIZES, (11, 11, 10))}
    assert {h.target_eye for h in hs} == {0, 1}
    assert all(0.055 <= h.baseline_m <= 0.072 and 600 <= h.focal_px <= 1100 and 0 <= h.phase_s < 1 / h.rate_hz
               for h in hs)
    assert [h.baseline_m for h in config5_headsets(32, seed=0)] == [h.baseline_m for h in hs]
    assert [h.baseline_m for h in config5_headsets(32, seed=1)] != [h.baseline_m for h in hs]


def test_trace_follows_each_display_clock_with_exponential_jitter():
    hs = config5_headsets(32)
    T = 20.0
    tr = serve.make_trace(hs, T, n_sources=8, seed=3)
    assert np.all(np.diff(tr["t_ns"]) >= 0) and tr["t_ns"].min() >= 0 and tr["t_ns"].max() < T * 1e9
    jit = []
    for i, h in enumerate(hs):
        a = tr[tr["headset"] == i]
        assert abs(len(a) - h.rate_hz * T) <= 2
        k = np.arange(len(a))
        assert np.array_equal(a["source"], k % 8)
        jit.append(a["t_ns"] / 1e9 - (h.phase_s + k / h.rate_hz))
    jit = np.concatenate(jit)
    assert jit.min() >= -1e-9
    assert abs(jit.mean() - 1e-3) < 5e-5 and abs(np.median(jit) - np.log(2) * 1e-3) < 5e-5
    assert abs(len(tr) / T - sum(h.rate_hz for h in hs)) < 5
    assert np.array_equal(serve.make_trace(hs, 2.0, 8, seed=3), serve.make_trace(hs, 2.0, 8, seed=3))


def test_workspace_sizes_and_option_checks():
    L = serve.lib()
    o = serve.Options()
    o.max_batch, o.max_in_flight, o.policy = 16, 4, serve.PLAIN
    plain = L.yoro_serve_workspace_bytes(ctypes.byref(o), 2160, 2160)
    assert plain >= 4 * yoro.load().yoro_stereo_batch_workspace_bytes(16)
    assert L.yoro_serve_host_bytes(ctypes.byref(o), 2160, 2160) >= 0
    o.policy = serve.LEARNED  # without a model, workspace or stream: refused
    o.tile, o.halo, o.chunk = 128, 64, 8
    assert L.yoro_serve_workspace_bytes(ctypes.byref(o), 2160, 2160) == 0
    o.model_weights, o.learned_workspace, o.learned_stream = 256, 256, 256
    learned = L.yoro_serve_workspace_bytes(ctypes.byref(o), 2160, 2160)
    assert learned > plain  # tile counts per slot and the crop plan
    assert L.yoro_serve_host_bytes(ctypes.byref(o), 2160, 2160) >= 4 * 16 * 17 * 17 * 4
    o.progressive = 2  # only 0 or 1
    assert L.yoro_serve_workspace_bytes(ctypes.byref(o), 2160, 2160) == 0
    o.progressive = 1
    assert L.yoro_serve_workspace_bytes(ctypes.byref(o), 2160, 2160) == learned
    # Bands: a multiple of the tile, at least twice the halo.
    for band, ok in ((256, True), (384, True), (200, False), (128, True), (-128, False)):
        o.band = band
        assert (L.yoro_serve_workspace_bytes(ctypes.byref(o), 2160, 2160) == learned) == ok, band
    o.halo = 72
    assert L.yoro_serve_workspace_bytes(ctypes.byref(o), 2160, 2160) == 0  # 2 halo > 128
    o.halo, o.band = 64, 0
    o.max_batch = 0
    assert L.yoro_serve_workspace_bytes(ctypes.byref(o), 2160, 2160) == 0


def test_run_rejects_bad_arguments_before_touching_the_device():
    L = serve.lib()
    o = serve.Options()
    o.max_batch, o.max_in_flight, o.policy = 4, 2, serve.PLAIN
    hs = (serve.Headset * 1)()
    hs[0].width, hs[0].height, hs[0].n_sources, hs[0].first_source = 64, 64, 1, 0
    hs[0].admitted, hs[0].n_outputs = 1, 1
    hs[0].dst_rgba[0] = 0x1000
    src = (serve.Source * 1)(serve.Source(0x2000, 0x3000))
    res = np.zeros(2, serve.RESULT_DTYPE)
    host = ctypes.create_string_buffer(1024)

    def run(arr, ws_bytes=1 << 20, opts=o, h=hs):
        a = np.ascontiguousarray(arr, serve.ARRIVAL_DTYPE)
        return L.yoro_serve_run(h, 1, src, 1, a.ctypes.data, len(a), ctypes.byref(opts), 0x4000, ws_bytes,
                                ctypes.addressof(host), 1024, None, res.ctypes.data)

    good = np.array([(0, 0, 0), (10, 0, 0)], serve.ARRIVAL_DTYPE)
    unsorted = np.array([(10, 0, 0), (0, 0, 0)], serve.ARRIVAL_DTYPE)
    bad_src = np.array([(0, 0, 1)], serve.ARRIVAL_DTYPE)
    bad_headset = np.array([(0, 1, 0)], serve.ARRIVAL_DTYPE)
    assert run(unsorted) == yoro.ERR_INVALID_ARG
    assert run(bad_src) == yoro.ERR_INVALID_ARG
    assert run(bad_headset) == yoro.ERR_INVALID_ARG
    assert run(good, ws_bytes=16) == yoro.ERR_WORKSPACE_TOO_SMALL
    hs[0].n_outputs = 0
    assert run(good) == yoro.ERR_INVALID_ARG
    hs[0].n_outputs = 1
    o.policy = serve.LEARNED
    assert run(good) == yoro.ERR_INVALID_ARG  # no model
    assert b"options" in yoro.load().yoro_last_error()
