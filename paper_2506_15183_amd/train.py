"""Train and evaluate the learned hole filler on seeded ray-cast windows.

Data: 256 x 256 windows of virtual 1832 x 1920 frames (scenes of 50..300
boxes and spheres, depth log-uniform on [0.3, 50] m, B ~ U[0.055, 0.072] m,
f ~ U[600, 1100] px).  The left eye is ray-cast over the window plus the
margin its sources come from, warped to the right eye by ``yoro_reproject``
with the plain nearest-background fill (on the GPU), and cropped to the
window; the label is the ray-cast right eye.  Loss: L1 over hole pixels.
Optimiser: AdamW (lr 1e-3, betas 0.9/0.999, eps 1e-8, weight decay 0.01).

    python -m paper_2506_15183_amd.train --windows 20000 --epochs 1 --out weights.npz

Weights are written as an .npz of bfloat16 bit patterns (uint16), one array
per layer in the network's order, loadable with numpy (no pickle).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import unet as U
from . import yoro
from .scenes.configs import training_window

WINDOW = 256
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "unet_windows256.npz")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_windows(indices, split: str, device, nthreads: int = 0):
    """(plain rgba [n,256,256,4] u8, depth f32, mask u8, target rgba u8) on the device."""
    n = len(indices)
    rgba = torch.empty((n, WINDOW, WINDOW, 4), dtype=torch.uint8, device=device)
    depth = torch.empty((n, WINDOW, WINDOW), dtype=torch.float32, device=device)
    mask = torch.empty((n, WINDOW, WINDOW), dtype=torch.uint8, device=device)
    target = torch.empty((n, WINDOW, WINDOW, 4), dtype=torch.uint8, device=device)
    for k, idx in enumerate(indices):
        win = training_window(int(idx), split, WINDOW)
        (s_rgba, s_depth), (t_rgba, _) = win.render(nthreads=nthreads)
        src_rgba = torch.from_numpy(s_rgba).to(device)
        src_depth = torch.from_numpy(s_depth).to(device)
        out, dz, mk = yoro.reproject(src_rgba, src_depth, win.spec.baseline_m, win.spec.focal_px,
                                     win.spec.target_eye, yoro.FILL_NEAREST_BG)
        rgba[k] = out[:, :WINDOW]
        depth[k] = dz[:, :WINDOW]
        mask[k] = mk[:, :WINDOW]
        target[k] = torch.from_numpy(t_rgba).to(device)
    return rgba, depth, mask, target


def flops_per_step(n: int, h: int, w: int) -> float:
    """Matrix-core FLOPs of one training step (forward, input and weight
    gradients) over the padded channel counts the kernels compute."""
    level = {"e0": 0, "e1": 1, "e2": 2, "e3": 3, "d2": 2, "d1": 1, "d0": 0, "he": 0}
    total = 0.0
    for name, cin, cout in U.ARCH:
        cin_p = U._pad32(cin)
        cout_p = U._pad32(cout)
        lev = level[name[:2]]
        pix = n * (h >> lev) * (w >> lev)
        f = 2.0 * 9 * cin_p * cout_p * pix
        total += f * (2 if name == "e0a" else 3)  # no input gradient for the first layer
    return total


def flops_forward(n: int, h: int, w: int) -> float:
    level = {"e0": 0, "e1": 1, "e2": 2, "e3": 3, "d2": 2, "d1": 1, "d0": 0, "he": 0}
    return sum(2.0 * 9 * U._pad32(cin) * U._pad32(cout) * n * (h >> level[nm[:2]]) * (w >> level[nm[:2]])
               for nm, cin, cout in U.ARCH)


def hole_psnr(out_rgba, target, mask):
    """Pooled hole PSNR over a batch (exact integer SSE on the GPU)."""
    sse, cnt = 0, 0
    for k in range(out_rgba.shape[0]):
        r = yoro.hole_sse(out_rgba[k], target[k], mask[k])
        s, c = [int(v) for v in r.cpu().numpy().view(np.uint64)]
        sse += s
        cnt += c
    if cnt == 0:
        return float("nan"), 0
    mse = sse / (3.0 * cnt)
    return (float("inf") if mse == 0 else 10.0 * math.log10(255.0 ** 2 / mse)), cnt


def evaluate(net: U.UNet, data, batch: int = 16):
    rgba, depth, mask, target = data
    out = torch.empty_like(rgba)
    for i in range(0, rgba.shape[0], batch):
        sl = slice(i, i + batch)
        net.fill(rgba[sl], depth[sl], mask[sl], out=out[sl])
    torch.cuda.synchronize()
    p_plain, n_holes = hole_psnr(rgba, target, mask)
    p_learned, _ = hole_psnr(out, target, mask)
    return {"hole_psnr_plain_db": round(p_plain, 3), "hole_psnr_learned_db": round(p_learned, 3),
            "hole_pixels": n_holes, "windows": int(rgba.shape[0])}


def save_weights(net: U.UNet, path: str):
    params = net.get_params()
    arrs = {}
    for (name, _, _), p in zip(U.ARCH, params):
        f = p.astype(np.float32)
        u = f.view(np.uint32).astype(np.uint64)
        arrs[name] = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, **arrs)


def load_weights(path: str = DEFAULT_WEIGHTS):
    """Canonical FP32 parameter list from a weights file (values exactly bf16)."""
    z = np.load(path, allow_pickle=False)
    return [(z[name].astype(np.uint32) << 16).view(np.float32) for name, _, _ in U.ARCH]


def train(windows=20000, epochs=1, batch=16, lr=1e-3, seed=0, val=500, out=None, chunk=1024, log_every=100,
          time_limit=None):
    dev = torch.device("cuda")
    net = U.UNet(dev, seed=seed)
    rng = np.random.default_rng(seed)
    t0 = time.time()
    log(f"rendering {val} validation windows")
    vdata = make_windows(range(val), "val", dev)
    before = evaluate(net, vdata)
    log(f"untrained: {before}  ({time.time() - t0:.1f}s)")
    fl = flops_per_step(batch, WINDOW, WINDOW)
    steps, t_train, losses = 0, 0.0, []
    stopped = False
    for ep in range(epochs):
        order = rng.permutation(windows)
        for c0 in range(0, windows, chunk):
            tg = time.time()
            data = make_windows(order[c0:c0 + chunk], "train", dev)
            torch.cuda.synchronize()
            log(f"epoch {ep} chunk {c0 // chunk}: rendered {data[0].shape[0]} windows in {time.time() - tg:.1f}s")
            for i in range(0, data[0].shape[0] - batch + 1, batch):
                sl = slice(i, i + batch)
                ts = time.time()
                loss = net.train_step(data[0][sl], data[1][sl], data[2][sl], data[3][sl], lr=lr)
                steps += 1
                if steps % log_every == 0:
                    losses.append(float(loss.item()))
                    log(f"step {steps} loss {losses[-1]:.5f}")
                torch.cuda.synchronize()
                t_train += time.time() - ts
                if time_limit and t_train > time_limit:
                    stopped = True
                    break
            del data
            if stopped:
                break
        if stopped:
            break
    after = evaluate(net, vdata)
    res = {"steps": steps, "batch": batch, "train_seconds": round(t_train, 2),
           "ms_per_step": round(1e3 * t_train / max(steps, 1), 3),
           "tflops_achieved": round(fl * steps / max(t_train, 1e-9) / 1e12, 2), "flops_per_step": fl,
           "losses": losses, "before": before, "after": after, "wall_seconds": round(time.time() - t0, 1)}
    log(json.dumps(res))
    if out:
        save_weights(net, out)
    return net, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--windows", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--val", type=int, default=500)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--time-limit", type=float, default=None, help="stop training after this many GPU seconds")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    _, res = train(a.windows, a.epochs, a.batch, a.lr, a.seed, a.val, a.out, time_limit=a.time_limit)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
