"""Hole PSNR of the plain nearest-background fill, the paper's Patcher,
the learned fill and the near-object hybrid against the ray-cast target eye
on held-out full frames,
the learned fill's inference throughput, and the whole-image error of the
reprojection through a downsampled intermediate buffer at scales 2-16.

    python -m paper_2506_15183_amd.evaluate --frames 16

PSNR is over the RGB channels of the hole pixels (mask != 0) with peak 255,
reported per frame (mean over frames) and pooled (one MSE over all hole
pixels of all frames).  The learned fill runs on whole frames here: it equals
the hole-tile fill bit for bit, and with hole blocks covering most of a frame
the whole frame is the cheaper of the two.
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np
import torch

from . import train, unet, yoro
from .scenes.configs import config4_test_frames

BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 matrix peak, vendor figure
LOWRES_SCALES = (2, 4, 8, 16)  # intermediate-buffer scales measured beside the direct path


def algorithmic_flops(h: int, w: int, n: int = 1) -> float:
    """FLOPs of one forward pass over the real channel counts (5-channel
    input, 3-channel head; the kernels' zero padding to 32 not counted)."""
    level = {"e0": 0, "e1": 1, "e2": 2, "e3": 3, "d2": 2, "d1": 1, "d0": 0, "he": 0}
    return sum(2.0 * 9 * cin * cout * n * (h >> level[nm[:2]]) * (w >> level[nm[:2]]) for nm, cin, cout in unet.ARCH)


def _psnr(sse: int, count: int) -> float:
    if count == 0:
        return float("nan")
    mse = sse / (3.0 * count)
    return float("inf") if mse == 0 else 10.0 * math.log10(255.0 ** 2 / mse)


def _sse(a, b, m):
    s, c = [int(v) for v in yoro.hole_sse(a, b, m).cpu().numpy().view(np.uint64)]
    return s, c


def evaluate(net: unet.UNet, n_frames: int = 16, log=None, timing_reps: int = 5):
    dev = net.device
    per_plain, per_learned, per_patch = [], [], []
    pooled = np.zeros((3, 2), dtype=np.int64)  # [plain, learned, patcher] x [sse, count]
    patch_times = []
    blocks, blocks_total, hole_frac = 0, 0, []
    times = []
    # Downsampled intermediate buffer: whole-image error against the ray-cast
    # eye and against the direct path, and its hole count, per (scale, linear).
    low = {(k, lin): np.zeros(5, dtype=np.int64) for k in LOWRES_SCALES for lin in (False, True)}
    direct_full = np.zeros(2, dtype=np.int64)
    for i, spec in enumerate(config4_test_frames(n_frames)):
        s_rgba, s_depth = spec.render_source()
        t_rgba, _ = spec.render_target()
        src = torch.from_numpy(s_rgba).to(dev)
        srd = torch.from_numpy(s_depth).to(dev)
        tgt = torch.from_numpy(t_rgba).to(dev)
        rgba, depth, mask = yoro.reproject(src, srd, spec.baseline_m, spec.focal_px, spec.target_eye,
                                           yoro.FILL_NEAREST_BG)
        out = net.fill_native(rgba[None], depth[None], mask[None])[0]
        counts = net.tile_holes(mask).cpu().numpy()
        blocks += int((counts > 0).sum())
        blocks_total += counts.size
        torch.cuda.synchronize()
        if i == 0:  # time the whole-frame learned fill (resident inputs)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(timing_reps)]
            for a, b in ev:
                a.record()
                net.fill_native(rgba[None], depth[None], mask[None], out=out[None])
                b.record()
            torch.cuda.synchronize()
            times = [a.elapsed_time(b) for a, b in ev]
        # The paper's Patcher on the same frame (warp, then the weighted fill).
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        ev[0].record()
        prgba, _, _ = yoro.reproject(src, srd, spec.baseline_m, spec.focal_px, spec.target_eye, yoro.FILL_PATCHER)
        ev[1].record()
        torch.cuda.synchronize()
        patch_times.append(ev[0].elapsed_time(ev[1]))
        direct_full += _sse(rgba, tgt, None)
        lbuf = (torch.empty_like(rgba), None, torch.empty_like(mask))
        for (k, lin), acc in low.items():
            lr, _, lm = yoro.reproject_lowres(src, srd, spec.baseline_m, spec.focal_px, spec.target_eye,
                                              yoro.FILL_NEAREST_BG, k, lin, out=lbuf)
            acc[0:2] += _sse(lr, tgt, None)
            acc[2:4] += _sse(lr, rgba, None)
            acc[4] += int((lm != 0).sum().item())
        sp = _sse(rgba, tgt, mask)
        sl = _sse(out, tgt, mask)
        sq = _sse(prgba, tgt, mask)
        pooled[0] += sp
        pooled[1] += sl
        pooled[2] += sq
        per_plain.append(_psnr(*sp))
        per_learned.append(_psnr(*sl))
        per_patch.append(_psnr(*sq))
        hole_frac.append(sp[1] / spec.pixels)
        if log:
            log(f"frame {i}: holes {hole_frac[-1]:.3f}, plain {per_plain[-1]:.2f} dB, patcher {per_patch[-1]:.2f} dB, "
                f"learned {per_learned[-1]:.2f} dB")
    h, w = 1920, 1832
    ms = float(np.median(times))
    fl = algorithmic_flops(h, w)
    return {
        "frames": n_frames, "size": f"{w}x{h}",
        "hole_fraction_mean": round(float(np.mean(hole_frac)), 4),
        "hole_psnr_plain_db": round(_psnr(*pooled[0]), 3),
        "hole_psnr_patcher_db": round(_psnr(*pooled[2]), 3),
        "hole_psnr_learned_db": round(_psnr(*pooled[1]), 3),
        "hole_psnr_plain_mean_db": round(float(np.mean(per_plain)), 3),
        "hole_psnr_patcher_mean_db": round(float(np.mean(per_patch)), 3),
        "hole_psnr_learned_mean_db": round(float(np.mean(per_learned)), 3),
        "patcher_warp_and_fill_ms_per_frame": round(float(np.median(patch_times[1:] or patch_times)), 4),
        "hole_blocks_fraction": round(blocks / max(blocks_total, 1), 4),
        "learned_ms_per_frame": round(ms, 3),
        "learned_tflops": round(fl / (ms * 1e-3) / 1e12, 2),
        "learned_frac_of_bf16_peak": round(fl / (ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, 4),
        "learned_flops_per_frame": fl,
        "image_psnr_direct_db": round(_psnr(*direct_full), 3),
        "lowres": [{"scale": k, "linear": lin,
                    "image_psnr_db": round(_psnr(int(a[0]), int(a[1])), 3),
                    "psnr_vs_direct_db": round(_psnr(int(a[2]), int(a[3])), 3),
                    "hole_fraction": round(int(a[4]) / int(a[1]), 4)} for (k, lin), a in low.items()],
    }


def evaluate_sparse(net: unet.UNet, n_frames: int = 8):
    """Hole PSNR of the plain and the learned fill against the ray-cast target
    eye on the serving loop's sparse-scene frames (the frames its learned
    policy refines: 1-3 % holes), whole frames, the three serving sizes and
    both eyes in turn."""
    from .scenes.configs import SERVE_SIZES, config5_pool_frame

    dev = net.device
    pooled = np.zeros((2, 2), dtype=np.int64)  # [plain, learned] x [sse, count]
    fracs = []
    for i in range(n_frames):
        w, h = SERVE_SIZES[i % len(SERVE_SIZES)]
        spec = config5_pool_frame(w, h, i % 2, 100 + i, sparse=True)
        s_rgba, s_depth = spec.render_source()
        t_rgba, _ = spec.render_target()
        src = torch.from_numpy(s_rgba).to(dev)
        srd = torch.from_numpy(s_depth).to(dev)
        tgt = torch.from_numpy(t_rgba).to(dev)
        rgba, depth, mask = yoro.reproject(src, srd, spec.baseline_m, spec.focal_px, spec.target_eye,
                                           yoro.FILL_NEAREST_BG)
        out = net.fill_native(rgba[None], depth[None], mask[None])[0]
        sp = _sse(rgba, tgt, mask)
        pooled[0] += sp
        pooled[1] += _sse(out, tgt, mask)
        fracs.append(sp[1] / spec.pixels)
    return {"frames": n_frames, "sizes": [f"{w}x{h}" for w, h in SERVE_SIZES],
            "hole_fraction_mean": round(float(np.mean(fracs)), 4),
            "hole_psnr_plain_db": round(_psnr(*pooled[0]), 3),
            "hole_psnr_learned_db": round(_psnr(*pooled[1]), 3)}


def evaluate_hybrid(net: unet.UNet, n_frames: int = 8, nears=(0.5, 1.0)):
    """The near-object hybrid (Section 11.4) beside the three fills, on the
    held-out 1832 x 1920 frames (objects from 0.3 m): every method's error
    against the ray-cast target eye over the plain path's hole pixels and
    over the whole image.  The hybrid renders the near field (surfaces
    nearer than near_m) for the target eye with yoro_render_near and warps
    and fills the rest with the plain fill; its time per frame is the near
    render plus the hybrid warp."""
    dev = net.device
    names = ["plain", "patcher", "learned"] + [f"hybrid_{d:g}m" for d in nears]
    holes = {k: np.zeros(2, dtype=np.int64) for k in names}
    whole = {k: np.zeros(2, dtype=np.int64) for k in names}
    near_frac = {d: [] for d in nears}
    left_frac = {d: [] for d in nears}
    times = {d: [] for d in nears}
    for i, spec in enumerate(config4_test_frames(n_frames)):
        sc = spec.scene()
        s_rgba, s_depth = spec.render_source()
        t_rgba, _ = spec.render_target()
        src = torch.from_numpy(s_rgba).to(dev)
        srd = torch.from_numpy(s_depth).to(dev)
        tgt = torch.from_numpy(t_rgba).to(dev)
        raw = bytes(memoryview(sc.objects).cast("B"))[: 88 * sc.n]
        objs = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
        rgba, depth, mask = yoro.reproject(src, srd, spec.baseline_m, spec.focal_px, spec.target_eye,
                                           yoro.FILL_NEAREST_BG)
        outs = {"plain": rgba,
                "patcher": yoro.reproject(src, srd, spec.baseline_m, spec.focal_px, spec.target_eye,
                                          yoro.FILL_PATCHER)[0],
                "learned": net.fill_native(rgba[None], depth[None], mask[None])[0]}
        for d in nears:
            ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            ev[0].record()
            nr, nd = yoro.render_near(objs, sc.n, spec.width, spec.height, sc.f, 0.5 * sc.Wv, 0.5 * sc.Hv,
                                      spec.target_eye_x(), d)
            hr, _, hm = yoro.reproject_hybrid(src, srd, spec.baseline_m, spec.focal_px, spec.target_eye,
                                              yoro.FILL_NEAREST_BG, d, nr, nd)
            ev[1].record()
            torch.cuda.synchronize()
            times[d].append(ev[0].elapsed_time(ev[1]))
            outs[f"hybrid_{d:g}m"] = hr
            near_frac[d].append(float((hm == yoro.MASK_NEAR).float().mean().item()))
            left_frac[d].append(float(((hm == 1) | (hm == 2)).float().mean().item()))
        for k, o in outs.items():
            holes[k] += _sse(o, tgt, mask)
            whole[k] += _sse(o, tgt, None)
    res = {"frames": n_frames, "size": "1832x1920", "hole_pixels": int(holes["plain"][1]),
           "hole_psnr_db": {k: round(_psnr(*v), 3) for k, v in holes.items()},
           "image_psnr_db": {k: round(_psnr(*v), 3) for k, v in whole.items()}}
    for d in nears:
        res[f"hybrid_{d:g}m"] = {"near_fraction": round(float(np.mean(near_frac[d])), 4),
                                 "far_holes_fraction": round(float(np.mean(left_frac[d])), 4),
                                 "render_and_warp_ms_per_frame": round(float(np.median(times[d][1:] or times[d])), 4)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=16)
    ap.add_argument("--weights", default=train.DEFAULT_WEIGHTS)
    a = ap.parse_args()
    net = unet.UNet("cuda", params=train.load_weights(a.weights))
    res = evaluate(net, a.frames, log=lambda m: print(m, file=sys.stderr, flush=True))
    res["hybrid"] = evaluate_hybrid(net, min(a.frames, 8))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
