"""Serving many headsets on one GPU: binding of include/yoro_serve.h plus the
workload around it (arrival traces, resident frame pools, admission under an
HBM budget, latency summaries).

    python -m paper_2506_15183_amd.serve --seconds 60

Each headset renders its dominant eye at 72, 90 or 120 Hz and needs the other
eye (the paper targets 90-120 frames per second per eye pair, Sections 1
and 12).  Frame k of a headset with rate r arrives at t0 + k / r + delta_k,
delta_k ~ Exp(mean 1 ms): the display clock plus a random render-completion
delay.  A headset owns a pool of resident source frames (used round-robin)
and a few output sets; the library's loop (yoro_serve_run) does the
batching, launching and completion tracking in native code.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import sys
from dataclasses import dataclass

import numpy as np
import torch

from . import yoro
from .scenes.configs import HeadsetSpec, config5_headsets, config5_pool_frame

PLAIN, LEARNED = 0, 1
PATH_PLAIN, PATH_LEARNED, PATH_FALLBACK, PATH_BUSY, PATH_REJECTED = 0, 1, 2, 3, 4
PATH_NAMES = ("plain", "learned", "fallback", "busy", "rejected")
MAX_OUTPUTS = 4

EXPORTS = ("yoro_serve_workspace_bytes", "yoro_serve_host_bytes", "yoro_serve_admit", "yoro_serve_run")


class Source(ctypes.Structure):
    _fields_ = [("rgba", ctypes.c_void_p), ("depth", ctypes.c_void_p)]


class Headset(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("baseline_m", ctypes.c_float), ("focal_px", ctypes.c_float),
        ("target_eye", ctypes.c_int32),
        ("first_source", ctypes.c_int32), ("n_sources", ctypes.c_int32),
        ("admitted", ctypes.c_int32), ("n_outputs", ctypes.c_int32),
        ("dst_rgba", ctypes.c_void_p * MAX_OUTPUTS),
        ("dst_depth", ctypes.c_void_p * MAX_OUTPUTS),
        ("dst_mask", ctypes.c_void_p * MAX_OUTPUTS),
    ]


class Arrival(ctypes.Structure):
    _fields_ = [("t_ns", ctypes.c_int64), ("headset", ctypes.c_int32), ("source", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [
        ("max_batch", ctypes.c_int32), ("max_in_flight", ctypes.c_int32), ("policy", ctypes.c_int32),
        ("learned_max_hole_fraction", ctypes.c_float),
        ("model_weights", ctypes.c_void_p), ("learned_workspace", ctypes.c_void_p),
        ("learned_workspace_bytes", ctypes.c_size_t),
        ("tile", ctypes.c_int32), ("halo", ctypes.c_int32), ("chunk", ctypes.c_int32),
        ("learned_stream", ctypes.c_void_p),
        ("learned_min_interval_ns", ctypes.c_int64),
        ("progressive", ctypes.c_int32),
        ("band", ctypes.c_int32),
    ]


class Result(ctypes.Structure):
    _fields_ = [("launch_ns", ctypes.c_int64), ("done_ns", ctypes.c_int64), ("path", ctypes.c_int32),
                ("batch_frames", ctypes.c_int32), ("holes", ctypes.c_int64), ("refined_ns", ctypes.c_int64)]


RESULT_DTYPE = np.dtype([("launch_ns", "<i8"), ("done_ns", "<i8"), ("path", "<i4"), ("batch_frames", "<i4"),
                         ("holes", "<i8"), ("refined_ns", "<i8")])
ARRIVAL_DTYPE = np.dtype([("t_ns", "<i8"), ("headset", "<i4"), ("source", "<i4")])
assert RESULT_DTYPE.itemsize == ctypes.sizeof(Result) and ARRIVAL_DTYPE.itemsize == ctypes.sizeof(Arrival)

_lib = None


def lib():
    global _lib
    if _lib is None:
        L = yoro.load()
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.yoro_serve_workspace_bytes.argtypes = [ctypes.POINTER(Options), i32, i32]
        L.yoro_serve_workspace_bytes.restype = sz
        L.yoro_serve_host_bytes.argtypes = [ctypes.POINTER(Options), i32, i32]
        L.yoro_serve_host_bytes.restype = sz
        L.yoro_serve_admit.argtypes = [vp, i32, i64, i64, vp]
        L.yoro_serve_admit.restype = i32
        L.yoro_serve_run.argtypes = [ctypes.POINTER(Headset), i32, ctypes.POINTER(Source), i32, vp, i64,
                                     ctypes.POINTER(Options), vp, sz, vp, sz, vp, vp]
        L.yoro_serve_run.restype = i32
        _lib = L
    return _lib


def admit(nbytes, budget: int, reserved: int = 0):
    """Greedy in-order admission (yoro_serve_admit): bool array."""
    b = np.ascontiguousarray(nbytes, dtype=np.int64)
    out = np.zeros(len(b), dtype=np.int32)
    n = lib().yoro_serve_admit(b.ctypes.data, len(b), int(budget), int(reserved), out.ctypes.data)
    if n < 0:
        raise ValueError("bad admission arguments")
    return out.astype(bool)


def make_trace(headsets, seconds: float, n_sources: int, seed: int = 0, jitter_ms: float = 1.0):
    """Arrivals (structured array sorted by time) of every headset over
    [0, seconds): t_k = phase + k / rate + Exp(jitter_ms), and no earlier
    than t_(k-1)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, h in enumerate(headsets):
        k = np.arange(int(np.ceil((seconds - h.phase_s) * h.rate_hz)) + 1)
        t = h.phase_s + k / h.rate_hz + rng.exponential(jitter_ms * 1e-3, size=k.size)
        t = np.maximum.accumulate(t)  # a frame is not ready before the previous one
        keep = t < seconds
        a = np.zeros(int(keep.sum()), ARRIVAL_DTYPE)
        a["t_ns"] = np.round(t[keep] * 1e9).astype(np.int64)
        a["headset"] = i
        a["source"] = k[keep] % n_sources
        parts.append(a)
    tr = np.concatenate(parts) if parts else np.zeros(0, ARRIVAL_DTYPE)
    return tr[np.argsort(tr["t_ns"], kind="stable")]


def headset_bytes(h, n_sources: int, n_outputs: int) -> int:
    """Resident bytes of one headset: its source pool (RGBA8 + FP32 depth) and
    output sets (RGBA8 + FP32 depth + u8 mask)."""
    px = h.width * h.height
    return n_sources * px * 8 + n_outputs * px * 9


@dataclass
class Config:
    budget_bytes: int = 8 * 10**9
    n_sources: int = 8
    n_outputs: int = 3
    max_batch: int = 64
    max_in_flight: int = 4
    tile: int = 128
    halo: int = 64
    chunk: int = 8
    learned_max_hole_fraction: float = 0.05
    learned_min_interval_ms: float = 0.0
    # Learned policy: release every frame at its warp and refine it in place
    # afterwards (latency = first delivery; refined_ns marks the upgrade).
    progressive: bool = False
    # Learned policy: 0 refines 128-pixel hole tiles (each in a crop with
    # `halo` pixels of context), > 0 the full-width bands of this many rows
    # that hold holes (a multiple of `tile`).  512-row bands refine a sparse
    # 1832x1920 frame in about 5 ms against about 8 ms for its hole tiles
    # (whose crops overlap), and reserve less memory than the tile plan.
    band: int = 512


class Server:
    """Resident pools and outputs of the admitted headsets, the loop's
    workspaces, and runs of yoro_serve_run over arrival traces."""

    def __init__(self, headsets, cfg: Config = Config(), frames=None, device="cuda", model=None, log=None):
        self.h = list(headsets)
        self.cfg = cfg
        self.device = torch.device(device)
        self.model = model
        L = lib()
        self.stream = torch.cuda.Stream(device=self.device)
        self.lstream = torch.cuda.Stream(device=self.device)
        self.lws = None
        opts = self._options(LEARNED if model is not None else PLAIN)
        max_w = max(h.width for h in self.h)
        max_h = max(h.height for h in self.h)
        self.ws_bytes = L.yoro_serve_workspace_bytes(ctypes.byref(opts), max_w, max_h)
        self.host_bytes = L.yoro_serve_host_bytes(ctypes.byref(opts), max_w, max_h)
        self.learned_bytes = 0
        if model is not None:
            from . import unet

            N = unet.nnlib()
            if cfg.band > 0:
                self.learned_bytes = max(N.yoro_model_bands_workspace_bytes(h.width, h.height, cfg.band, cfg.halo)
                                         for h in self.h)
            else:
                tiles = -(-max_w // cfg.tile) * -(-max_h // cfg.tile)
                self.learned_bytes = N.yoro_model_tiles_workspace_bytes(tiles, cfg.chunk, cfg.tile, cfg.halo)
        reserved = self.ws_bytes + self.learned_bytes + (model.wf.numel() * 2 if model is not None else 0)
        need = [headset_bytes(h, cfg.n_sources, cfg.n_outputs) for h in self.h]
        self.admitted = admit(need, cfg.budget_bytes, reserved)
        self.resident_bytes = int(np.sum(np.array(need)[self.admitted])) + reserved
        if log:
            log(f"admitted {int(self.admitted.sum())} of {len(self.h)} headsets, "
                f"{self.resident_bytes / 1e9:.2f} GB resident of {cfg.budget_bytes / 1e9:.1f} GB")
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)
        self.host = torch.empty(max(self.host_bytes, 256), dtype=torch.uint8, pin_memory=True)
        self.lws = torch.empty(max(self.learned_bytes, 256), dtype=torch.uint8, device=self.device)
        # Resident buffers.
        self.pools, self.outs = [], []
        self.sources = []
        self.table = (Headset * len(self.h))()
        for i, h in enumerate(self.h):
            T = self.table[i]
            T.width, T.height, T.baseline_m, T.focal_px = h.width, h.height, h.baseline_m, h.focal_px
            T.target_eye, T.admitted = h.target_eye, int(self.admitted[i])
            T.first_source, T.n_sources, T.n_outputs = len(self.sources), cfg.n_sources, cfg.n_outputs
            pool, outs = [], []
            for s in range(cfg.n_sources):
                if self.admitted[i]:
                    rgba, depth = frames(h, s)
                    r = torch.from_numpy(rgba).to(self.device)
                    d = torch.from_numpy(depth).to(self.device)
                    pool.append((r, d))
                    self.sources.append((r.data_ptr(), d.data_ptr()))
                else:
                    self.sources.append((0, 0))
            if self.admitted[i]:
                for o in range(cfg.n_outputs):
                    rgba = torch.empty((h.height, h.width, 4), dtype=torch.uint8, device=self.device)
                    depth = torch.empty((h.height, h.width), dtype=torch.float32, device=self.device)
                    mask = torch.empty((h.height, h.width), dtype=torch.uint8, device=self.device)
                    outs.append((rgba, depth, mask))
                    T.dst_rgba[o], T.dst_depth[o], T.dst_mask[o] = rgba.data_ptr(), depth.data_ptr(), mask.data_ptr()
            self.pools.append(pool)
            self.outs.append(outs)
        if not self.admitted.any():
            raise RuntimeError("no headset fits the budget")
        self.src_table = (Source * len(self.sources))(*[Source(*s) for s in self.sources])
        torch.cuda.synchronize()

    def _options(self, policy):
        c = self.cfg
        o = Options()
        o.max_batch, o.max_in_flight, o.policy = c.max_batch, c.max_in_flight, policy
        o.learned_max_hole_fraction = c.learned_max_hole_fraction
        o.learned_min_interval_ns = int(c.learned_min_interval_ms * 1e6)
        o.progressive = int(bool(c.progressive))
        o.tile, o.halo, o.chunk, o.band = c.tile, c.halo, c.chunk, c.band
        if policy == LEARNED:
            o.model_weights = self.model.wf.data_ptr()
            # (sizing happens before the workspace exists: any non-null address)
            o.learned_workspace = self.lws.data_ptr() if self.lws is not None else 256
            o.learned_workspace_bytes = self.learned_bytes if self.lws is not None else 0
            o.learned_stream = self.lstream.cuda_stream
        return o

    def run(self, trace, policy: int = PLAIN):
        """Runs a trace in real time; returns the per-arrival results."""
        if policy == LEARNED and self.model is None:
            raise ValueError("the learned policy needs a model")
        tr = np.ascontiguousarray(trace, dtype=ARRIVAL_DTYPE)
        res = np.zeros(len(tr), RESULT_DTYPE)
        opts = self._options(policy)
        torch.cuda.synchronize()
        yoro._check(lib().yoro_serve_run(self.table, len(self.h), self.src_table, len(self.sources),
                                         tr.ctypes.data, len(tr), ctypes.byref(opts), self.ws.data_ptr(),
                                         self.ws_bytes, self.host.data_ptr(), self.host_bytes,
                                         self.stream.cuda_stream, res.ctypes.data))
        return res


def run_interleaved(server, trace, policies, rounds: int = 2):
    """Runs the trace once per policy per round, the policies alternating
    (plain, learned, plain, learned, ...), and pools each policy's arrivals
    and results: slow drifts of the host then affect every policy alike.
    Returns {policy: (trace, results)} to pass to summarize with
    seconds * rounds."""
    runs = {p: ([], []) for p in policies}
    for _ in range(rounds):
        for p in policies:
            runs[p][0].append(trace)
            runs[p][1].append(server.run(trace, p))
    return {p: (np.concatenate(t), np.concatenate(r)) for p, (t, r) in runs.items()}


def summarize(trace, res, headsets, seconds: float):
    """Latency percentiles (ms, completion - arrival, over processed frames),
    throughput and frame counts by path."""
    done = res["path"] != PATH_REJECTED
    lat = (res["done_ns"][done] - trace["t_ns"][done]) / 1e6
    px = np.array([h.width * h.height for h in headsets], dtype=np.int64)[trace["headset"][done]]
    span = max(seconds, (res["done_ns"][done].max() if done.any() else 0) / 1e9)
    out = {
        "frames": int(len(trace)), "processed": int(done.sum()),
        "paths": {PATH_NAMES[p]: int((res["path"] == p).sum()) for p in range(5) if (res["path"] == p).any()},
        "p50_ms": round(float(np.percentile(lat, 50)), 4) if lat.size else None,
        "p99_ms": round(float(np.percentile(lat, 99)), 4) if lat.size else None,
        "max_ms": round(float(lat.max()), 4) if lat.size else None,
        "mpix_per_s": round(float(px.sum()) / span / 1e6, 1),
        "frames_per_s": round(float(done.sum()) / span, 1),
        "mean_batch_frames": round(float(res["batch_frames"][done].mean()), 3) if done.any() else None,
    }
    refined = res["path"][done] == PATH_LEARNED
    if refined.any():
        out["refined_fraction"] = round(float(refined.mean()), 5)
        out["learned_frames_p50_ms"] = round(float(np.percentile(lat[refined], 50)), 4)
        out["learned_frames_p99_ms"] = round(float(np.percentile(lat[refined], 99)), 4)
        out["learned_frames_max_ms"] = round(float(lat[refined].max()), 4)
        out["p99_plain_path_frames_ms"] = round(float(np.percentile(lat[~refined], 99)), 4)
        up = res["refined_ns"][done][refined]
        if (up >= 0).any():  # progressive: time from arrival to the refined upgrade
            t_up = (up[up >= 0] - trace["t_ns"][done][refined][up >= 0]) / 1e6
            out["refined_upgrade_p50_ms"] = round(float(np.percentile(t_up, 50)), 4)
            out["refined_upgrade_p99_ms"] = round(float(np.percentile(t_up, 99)), 4)
            out["refined_upgrade_max_ms"] = round(float(t_up.max()), 4)
    holes = res["holes"][done]
    if (holes >= 0).any():
        frac = holes[holes >= 0] / px[holes >= 0]
        out["hole_fraction_p50"] = round(float(np.median(frac)), 4)
        out["hole_fraction_min"] = round(float(frac.min()), 4)
    return out


def pool_renderer(n_threads: int = 0, sparse: bool = False):
    """Pool frames shared by headsets of the same resolution and eye (each
    headset still holds its own resident copy)."""
    cache = {}

    def frames(h: HeadsetSpec, slot: int):
        key = (h.width, h.height, h.target_eye, slot)
        if key not in cache:
            spec = config5_pool_frame(h.width, h.height, h.target_eye, slot, sparse=sparse)
            cache[key] = spec.render_source(nthreads=n_threads)
        return cache[key]

    return frames


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--headsets", type=int, default=32)
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--budget-gb", type=float, default=8.0)
    ap.add_argument("--learned", action="store_true", help="also run the learned policy with its fallback")
    ap.add_argument("--weights", default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--sparse", action="store_true", help="scenes with few holes (U{20..60} objects, depth >= 2 m)")
    ap.add_argument("--learned-interval-ms", type=float, default=0.0)
    ap.add_argument("--progressive", action="store_true",
                    help="learned policy: release frames at the warp, refine them in place afterwards")
    ap.add_argument("--band", type=int, default=Config.band,
                    help="learned policy: refine full-width bands of this many rows (0: 128-pixel hole tiles)")
    a = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    hs = config5_headsets(a.headsets, a.seed)
    model = None
    if a.learned:
        from . import train, unet

        model = unet.UNet("cuda", params=train.load_weights(a.weights or train.DEFAULT_WEIGHTS))
    cfg = Config(budget_bytes=int(a.budget_gb * 1e9), learned_min_interval_ms=a.learned_interval_ms,
                 progressive=a.progressive, band=a.band)
    srv = Server(hs, cfg, pool_renderer(sparse=a.sparse), model=model, log=log)
    trace = make_trace(hs, a.seconds, cfg.n_sources, seed=a.seed)
    log(f"{len(trace)} arrivals over {a.seconds} s")
    out = {"headsets": len(hs), "admitted": int(srv.admitted.sum()), "resident_gb": round(srv.resident_bytes / 1e9, 3)}
    out["plain"] = summarize(trace, srv.run(trace, PLAIN), hs, a.seconds)
    log(json.dumps(out["plain"]))
    if model is not None:
        out["learned"] = summarize(trace, srv.run(trace, LEARNED), hs, a.seconds)
        log(json.dumps(out["learned"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
