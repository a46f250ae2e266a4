"""Profiling helpers: counter runs and rocprofv3 summaries.

Workflow (each step its own process; the GPU steps under rocprofv3):

  1. rocprofv3 --kernel-trace --stats -d OUT/trace -o t -- python bench.py --no-cpu-baseline --no-single-frame --serve-seconds 0 --eval-frames 0 --no-lowres
  2. rocprofv3 --pmc FETCH_SIZE -d OUT/fetch -o f -- python -m paper_2506_15183_amd.profiling counters
  3. rocprofv3 --pmc WRITE_SIZE -d OUT/write -o w -- python -m paper_2506_15183_amd.profiling counters
  4. python -m paper_2506_15183_amd.profiling summarize OUT > profiles/<kernel>_<workload>.md
     (summarize-lowres OUT for the downsampled-buffer kernel)

The ``counters`` workload launches the batched warp kernel a few times on the
64-frame batch and, for calibration, a plain elementwise kernel that reads
and writes a known number of bytes: each counter is scaled by (bytes the copy moves) /
(what the counter reports for the copy), so ``traffic`` is in real bytes.
"""
from __future__ import annotations

import glob
import hashlib
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# The warp kernel's source: its own file and the row machinery it includes.
KERNEL_SOURCES = (os.path.join(HERE, "csrc", "warp_fill.hip"), os.path.join(HERE, "csrc", "row_common.h"))
WARP_KERNEL = "warp_batch_kernel"
LOWRES_KERNEL = "lowres_batch_kernel"
LOWRES_SOURCES = (os.path.join(HERE, "csrc", "lowres.hip"), os.path.join(HERE, "csrc", "row_common.h"))
LOWRES_COUNTED = (4, 16)  # scales whose HBM counters the counters workload takes
COPY_BYTES = 1 << 30


def kernel_source_sha() -> str:
    """Short hash of the kernel source the counters were taken on."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _sha(paths) -> str:
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def lowres_lds_bytes(max_width: int, k: int) -> int:
    """Dynamic LDS of the downsampled-buffer kernel (as the library sizes it):
    the row's keys, hit masks, hole counter and list, plus the texel slots."""
    wl = (max_width + 63) & ~63
    hl = (wl + 255) // 256 * 256
    slots = (((max_width + k - 1) // k) + 63) & ~63
    return (wl + 64) * 8 + (wl // 64) * 8 + 16 + hl * 2 + slots * 8


def counters_workload(launches: int = 5) -> None:
    import torch

    from . import workloads

    dev = torch.device("cuda:0")
    # The benchmark's own batch (RGBA output only).
    batch = workloads.rgba_only_batch(dev).batch
    batch.prepare()
    for _ in range(launches):
        batch.launch()
    # The same batch through the downsampled intermediate buffer.
    for k in LOWRES_COUNTED:
        for _ in range(launches):
            batch.launch_lowres(k, True)
    # The calibration kernel: an elementwise pass that reads and writes
    # COPY_BYTES each (torch's bitwise_not on int32).
    a = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    for _ in range(launches):
        torch.bitwise_not(a, out=b)
    torch.cuda.synchronize()
    print(f"counters workload done: {launches} warp launches, {launches} copies of {COPY_BYTES} B", flush=True)


def learned_workload(frames: int = 4, steps: int = 4) -> None:
    """Whole-frame learned fill of a 1832 x 1920 frame, then training steps on
    16 windows of 256 x 256 (seeded synthetic inputs, committed weights)."""
    import numpy as np
    import torch

    from . import train, unet

    net = unet.UNet("cuda", params=train.load_weights(train.DEFAULT_WEIGHTS))
    rng = np.random.default_rng(0)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    h, w = 1920, 1832
    rgba = T(rng.integers(0, 256, (1, h, w, 4), dtype=np.uint8))
    depth = T(np.exp(rng.uniform(np.log(0.3), np.log(50), (1, h, w))).astype(np.float32))
    mask = T((rng.random((1, h, w)) < 0.2).astype(np.uint8))
    out = torch.empty_like(rgba)
    for _ in range(frames):
        net.fill_native(rgba, depth, mask, out=out)
    n = 16
    batch = [T(rng.integers(0, 256, (n, 256, 256, 4), dtype=np.uint8)),
             T(np.exp(rng.uniform(np.log(0.3), np.log(50), (n, 256, 256))).astype(np.float32)),
             T((rng.random((n, 256, 256)) < 0.2).astype(np.uint8)),
             T(rng.integers(0, 256, (n, 256, 256, 4), dtype=np.uint8))]
    for _ in range(steps):
        net.train_step(*batch)
    torch.cuda.synchronize()
    print(f"learned workload done: {frames} frames, {steps} training steps", flush=True)


def summarize_learned(trace_dir: str) -> str:
    """Per-layer kernel durations of the last whole-frame forward pass and the
    kernel totals of the last training step, from a kernel trace of
    ``learned_workload``."""
    c = _db(trace_dir)
    rows = list(c.execute("select name, duration from kernels order by start"))

    def short(n):
        n = n.replace("void ", "").replace("yoro::(anonymous namespace)::", "")
        return n.split("(")[0]

    # The whole-frame forwards come first (each ends with the composite), the
    # training steps after them (each starts by packing its input).
    ends = [i for i, (n, _) in enumerate(rows) if short(n).startswith("composite_kernel")]
    starts = [i for i, (n, _) in enumerate(rows) if short(n).startswith("unet_input")]
    lines = ["# Learned fill kernels: one 1832x1920 forward pass and one training step", "",
             "Commands (from the repository root, on one MI355X; OUT=the output directory):", "", "```",
             "rocprofv3 --kernel-trace --stats -d $OUT -o l -- python -m paper_2506_15183_amd.profiling learned",
             "python -m paper_2506_15183_amd.profiling summarize-learned $OUT", "```", "",
             "## Forward pass (last whole-frame fill), in order", "",
             "FLOPs per convolution over the channels the kernels compute (padded to 32, the head's 16-wide tile).",
             "", "| # | step | kernel | us | TFLOP/s |", "|---|---|---|---|---|"]
    steps = ["e0a (packs the input)", "e0b (+ 2x2 pool)", "e1a", "e1b (+ 2x2 pool)", "e2a", "e2b (+ 2x2 pool)", "e3a",
             "e3b", "d2a (upsampling load)", "d2b", "d2c", "d1a (upsampling load)", "d1b", "d1c",
             "d0a (upsampling load)", "d0b", "d0c", "head", "composite"]
    lev = {"e0": 0, "e1": 1, "e2": 2, "e3": 3, "d2": 2, "d1": 1, "d0": 0, "he": 0}
    cin = {"e0a": 32, "e0b": 32, "e1a": 32, "e1b": 64, "e2a": 64, "e2b": 128, "e3a": 128, "e3b": 256, "d2a": 256,
           "d2b": 256, "d2c": 128, "d1a": 128, "d1b": 128, "d1c": 64, "d0a": 64, "d0b": 64, "d0c": 32, "head": 32}
    cout = {"e0a": 32, "e0b": 32, "e1a": 64, "e1b": 64, "e2a": 128, "e2b": 128, "e3a": 256, "e3b": 256, "d2a": 128,
            "d2b": 128, "d2c": 128, "d1a": 64, "d1b": 64, "d1c": 64, "d0a": 32, "d0b": 32, "d0c": 32, "head": 16}
    # The last whole-frame forward: the kernels after the previous composite.
    n_fwd = len([e for e in ends if not starts or e < starts[0]])
    i0 = ends[n_fwd - 2] + 1 if n_fwd >= 2 else 0
    total = 0.0
    k = 0
    for name, dur in rows[i0:]:
        nm = short(name)
        total += dur
        st = steps[k] if k < len(steps) else "?"
        key = st.split(" ")[0]
        tf = ""
        if key in cin:
            px = (1920 >> lev[key[:2]]) * (1832 >> lev[key[:2]])
            tf = f"{2.0 * 9 * cin[key] * cout[key] * px / dur / 1e3:.0f}"
        lines.append(f"| {k} | {st} | `{nm}` | {dur / 1000:.1f} | {tf} |")
        k += 1
        if nm.startswith("composite"):
            break
    lines += ["", f"forward total: {total / 1000:.1f} us", "", "## Training step (last), kernel totals", "",
              "| kernel | calls | us |", "|---|---|---|"]
    last = starts[-1]
    agg = {}
    for name, dur in rows[last:]:
        nm = short(name)
        if nm.startswith("at::") or "rocclr" in nm:
            continue
        a = agg.setdefault(nm, [0, 0.0])
        a[0] += 1
        a[1] += dur
    for nm, (cnt, d) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| `{nm}` | {cnt} | {d / 1000:.1f} |")
    lines += ["", f"training step total: {sum(v[1] for v in agg.values()) / 1000:.1f} us", ""]
    return "\n".join(lines)


def _db(path_dir: str) -> sqlite3.Connection:
    files = glob.glob(os.path.join(path_dir, "**", "*_results.db"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no rocpd database under {path_dir}")
    return sqlite3.connect(files[0])


def _counter_means(path_dir: str, counter: str):
    """(mean counter value per dispatch of the warp kernel, of the copy kernel)."""
    c = _db(path_dir)
    warp, copy = [], []
    for name, cname, val in c.execute("select kernel_name, counter_name, value from counters_collection"):
        if cname != counter:
            continue
        if WARP_KERNEL in name:
            warp.append(val)
        elif "bitwise_not" in name.lower() or "bitwisenot" in name.lower():
            copy.append(val)
    if not warp or not copy:
        raise RuntimeError(f"{counter}: found {len(warp)} warp and {len(copy)} copy dispatches")
    return sum(warp) / len(warp), sum(copy) / len(copy)


def _trace_stats(path_dir: str):
    """[(kernel name, calls, median ns, mean ns, min ns)] from the per-dispatch trace, longest first."""
    c = _db(path_dir)
    per = {}
    for name, dur in c.execute("select name, duration from kernels"):
        per.setdefault(name, []).append(float(dur))
    rows = []
    for name, d in per.items():
        d = sorted(d)
        rows.append((name, len(d), d[len(d) // 2], sum(d) / len(d), d[0]))
    rows.sort(key=lambda r: -r[1] * r[3])
    return rows


def summarize(out_dir: str, pixels: int, algo_bytes_per_px: int = 12) -> str:
    trace = _trace_stats(os.path.join(out_dir, "trace"))
    fw, fc = _counter_means(os.path.join(out_dir, "fetch"), "FETCH_SIZE")
    ww, wc = _counter_means(os.path.join(out_dir, "write"), "WRITE_SIZE")
    fetch_scale = COPY_BYTES / (fc * 1024.0)
    write_scale = COPY_BYTES / (wc * 1024.0)
    fetch_bytes = fw * 1024.0 * fetch_scale
    write_bytes = ww * 1024.0 * write_scale
    traffic = fetch_bytes + write_bytes
    algo = algo_bytes_per_px * pixels
    warp_rows = [r for r in trace if WARP_KERNEL in r[0]]
    lines = [
        "# warp_batch_kernel on the 64-frame mixed-resolution batch",
        "",
        "Commands (from the repository root, on one MI355X; OUT=the output directory):",
        "",
        "```",
        "rocprofv3 --kernel-trace --stats -d $OUT/trace -o t -- python bench.py --no-cpu-baseline --no-single-frame --serve-seconds 0 --eval-frames 0 --no-lowres",
        "rocprofv3 --pmc FETCH_SIZE -d $OUT/fetch -o f -- python -m paper_2506_15183_amd.profiling counters",
        "rocprofv3 --pmc WRITE_SIZE -d $OUT/write -o w -- python -m paper_2506_15183_amd.profiling counters",
        "python -m paper_2506_15183_amd.profiling summarize $OUT",
        "```",
        "",
        "## Kernel trace (top kernels)",
        "",
        "| kernel | calls | median ns | mean ns | min ns |",
        "|---|---|---|---|---|",
    ]
    for name, calls, med, mean, mn in trace[:8]:
        short = name if len(name) < 90 else name[:87] + "..."
        lines.append(f"| `{short}` | {calls} | {med:.0f} | {mean:.0f} | {mn:.0f} |")
    lines += [
        "",
        "## HBM traffic per launch (FETCH_SIZE, WRITE_SIZE)",
        "",
        f"Calibration: an elementwise pass reading and writing {COPY_BYTES} B reports FETCH_SIZE = {fc:.0f} KiB and WRITE_SIZE = "
        f"{wc:.0f} KiB per dispatch, so the scale factors are fetch x{fetch_scale:.4f}, write x{write_scale:.4f}.",
        "",
        f"- warp kernel FETCH_SIZE {fw:.0f} KiB -> {fetch_bytes / 1e9:.4f} GB read",
        f"- warp kernel WRITE_SIZE {ww:.0f} KiB -> {write_bytes / 1e9:.4f} GB written",
        f"- algorithmic bytes per launch: {algo_bytes_per_px} B x {pixels} px = {algo / 1e9:.4f} GB",
        f"- measured / algorithmic: {traffic / algo:.4f}",
        "",
        "Machine-readable (read by bench.py):",
        "",
        f"traffic_bytes_per_launch: {traffic:.0f}",
        f"kernel_median_ns: {warp_rows[0][2]:.0f}" if warp_rows else "kernel_median_ns: nan",
        f"kernel_source_sha: {kernel_source_sha()}",
        "",
    ]
    return "\n".join(lines)


def summarize_lowres(out_dir: str, pixels: int, max_width: int = 2160) -> str:
    """The downsampled-buffer kernel per scale: durations from the bench trace
    (dispatches told apart by their LDS size, which depends on the scale) and
    HBM bytes from the counter runs."""
    scales = (1, 2, 4, 8, 16)
    lds = {lowres_lds_bytes(max_width, k): k for k in scales}

    def scale_of(size):
        return lds[min(lds, key=lambda b: abs(b - size))]

    c = _db(os.path.join(out_dir, "trace"))
    dur = {k: [] for k in scales}
    for name, size, d in c.execute("select name, lds_size, duration from kernels"):
        if LOWRES_KERNEL in name:
            dur[scale_of(size)].append(float(d))
    counted = {}
    for cname, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        cc = _db(os.path.join(out_dir, sub))
        vals, copy = {k: [] for k in scales}, []
        for name, size, cn, v in cc.execute(
                "select kernel_name, lds_block_size, counter_name, value from counters_collection"):
            if cn != cname:
                continue
            if LOWRES_KERNEL in name:
                vals[scale_of(size)].append(v)
            elif "bitwise_not" in name.lower() or "bitwisenot" in name.lower():
                copy.append(v)
        scale = COPY_BYTES / (sum(copy) / len(copy) * 1024.0)
        for k in scales:
            if vals[k]:
                counted.setdefault(k, {})[cname] = sum(vals[k]) / len(vals[k]) * 1024.0 * scale
    lines = [
        "# lowres_batch_kernel (downsampled intermediate buffer) on the 64-frame mixed-resolution batch",
        "",
        "Commands (from the repository root, on one MI355X; OUT=the output directory):",
        "",
        "```",
        "rocprofv3 --kernel-trace --stats -d $OUT/trace -o t -- python bench.py --no-cpu-baseline --no-single-frame --serve-seconds 0 --eval-frames 0 --no-lowres",
        "rocprofv3 --pmc FETCH_SIZE -d $OUT/fetch -o f -- python -m paper_2506_15183_amd.profiling counters",
        "rocprofv3 --pmc WRITE_SIZE -d $OUT/write -o w -- python -m paper_2506_15183_amd.profiling counters",
        "python -m paper_2506_15183_amd.profiling summarize-lowres $OUT",
        "```",
        "",
        "RGBA output only, interpolated shift, one unit = one block row of k rows.",
        "Scale 1 runs the direct warp kernel (its own summary), so its row is absent here.",
        "Algorithmic bytes per pixel: 4 B gathered + 4 B written + 4/k^2 B of block-centre depth.",
        "Counter bytes are scaled as for the warp kernel (copy-kernel calibration).",
        "",
        "| k | dispatches | median us | mean us | algorithmic GB | algorithmic TB/s (mean) | HBM read GB | HBM written GB | HBM / algorithmic |",
        "|---|---|---|---|---|---|---|---|---|",
    ]
    for k in scales:
        d = sorted(dur[k])
        if not d:
            continue
        mean = sum(d) / len(d)
        algo = (8.0 + 4.0 / (k * k)) * pixels
        cnt = counted.get(k, {})
        rd, wr = cnt.get("FETCH_SIZE"), cnt.get("WRITE_SIZE")
        ratio = f"{(rd + wr) / algo:.3f}" if rd is not None and wr is not None else "-"
        lines.append(f"| {k} | {len(d)} | {d[len(d) // 2] / 1e3:.1f} | {mean / 1e3:.1f} | {algo / 1e9:.4f} | "
                     f"{algo / (mean * 1e-9) / 1e12:.2f} | {'-' if rd is None else f'{rd / 1e9:.4f}'} | "
                     f"{'-' if wr is None else f'{wr / 1e9:.4f}'} | {ratio} |")
    lines += ["", f"kernel_source_sha: {_sha(LOWRES_SOURCES)}", ""]
    return "\n".join(lines)


def summarize_pose(out_dir: str) -> str:
    """The general-pose kernels (clear, scatter, resolve) from a kernel trace
    of the bench's single-frame pose timing."""
    trace = _trace_stats(os.path.join(out_dir, "trace"))
    rows = [r for r in trace if "pose_" in r[0]]
    lines = [
        "# pose kernels (reprojection to a general pose) on one 1832x1920 frame",
        "",
        "Commands (from the repository root, on one MI355X; OUT=the output directory):",
        "",
        "```",
        "rocprofv3 --kernel-trace --stats -d $OUT/trace -o p -- python bench.py --no-cpu-baseline --serve-seconds 0 "
        "--eval-frames 0 --no-lowres --steps 5 --warmup 1",
        "python -m paper_2506_15183_amd.profiling summarize-pose $OUT",
        "```",
        "",
        "Head motion of 3 degrees about a tilted axis and 5.5 cm, RGBA output, one call = the three kernels.",
        "",
        "| kernel | calls | median us | mean us | min us |",
        "|---|---|---|---|---|",
    ]
    total = 0.0
    for name, calls, med, mean, mn in rows:
        short = name if len(name) < 90 else name[:87] + "..."
        lines.append(f"| `{short}` | {calls} | {med / 1e3:.1f} | {mean / 1e3:.1f} | {mn / 1e3:.1f} |")
        total += med
    lines += ["", f"sum of medians per call: {total / 1e3:.1f} us", "",
              f"kernel_source_sha: {_sha((os.path.join(HERE, 'csrc', 'pose.hip'), os.path.join(HERE, 'csrc', 'row_common.h')))}",
              ""]
    return "\n".join(lines)


def summarize_warp_counters(path_dir: str) -> str:
    """Mean of every counter per dispatch of the warp batch kernel (a --pmc run
    of the counters workload), one line each."""
    c = _db(path_dir)
    acc = {}
    for name, cname, val in c.execute("select kernel_name, counter_name, value from counters_collection"):
        if WARP_KERNEL in name:
            acc.setdefault(cname, []).append(float(val))
    lines = [f"kernel_source_sha: {kernel_source_sha()}"]
    for k in sorted(acc):
        v = acc[k]
        lines.append(f"{k}: {sum(v) / len(v):.4g} (mean of {len(v)} dispatches)")
    return "\n".join(lines)


def read_summary(path: str):
    """(traffic bytes per launch, kernel source sha) from a committed summary, or (None, None)."""
    if not os.path.exists(path):
        return None, None
    text = open(path).read()
    t = re.search(r"^traffic_bytes_per_launch: (\d+)", text, re.M)
    h = re.search(r"^kernel_source_sha: (\w+)", text, re.M)
    return (int(t.group(1)) if t else None), (h.group(1) if h else None)


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "counters":
        counters_workload()
    elif len(sys.argv) >= 2 and sys.argv[1] == "learned":
        learned_workload()
    elif len(sys.argv) >= 3 and sys.argv[1] == "summarize-learned":
        print(summarize_learned(sys.argv[2]))
    elif len(sys.argv) >= 3 and sys.argv[1] == "summarize-counters":
        print(summarize_warp_counters(sys.argv[2]))
    elif len(sys.argv) >= 3 and sys.argv[1] == "summarize-pose":
        print(summarize_pose(sys.argv[2]))
    elif len(sys.argv) >= 3 and sys.argv[1] == "summarize-lowres":
        sys.path.insert(0, os.path.dirname(HERE))
        from paper_2506_15183_amd.scenes import config3_frames

        print(summarize_lowres(sys.argv[2], sum(s.pixels for s in config3_frames())))
    elif len(sys.argv) >= 3 and sys.argv[1] == "summarize":
        sys.path.insert(0, os.path.dirname(HERE))
        from paper_2506_15183_amd.scenes import config3_frames

        px = sum(s.pixels for s in config3_frames())
        print(summarize(sys.argv[2], px))
    else:
        print(__doc__)
        sys.exit(2)
