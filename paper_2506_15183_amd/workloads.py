"""The timed batch workload, built in one place for the benchmark and for the
GPU test that checks that exact configuration against the oracle.

64 seeded ray-cast frames (16 each of 1024x1024, 1440x1600, 1832x1920,
2160x2160), each warped to the other eye with the nearest-background fill,
RGBA output only (no depth, no mask), as one persistent batched launch.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import yoro
from .scenes import config3_frames


@dataclass
class BatchWorkload:
    specs: list
    frames: list       # host (rgba, depth) per frame, as rendered
    src: list          # device (rgba, depth) per frame
    dst: list          # device RGBA output per frame
    batch: "yoro.StereoBatch"

    @property
    def pixels(self) -> int:
        return sum(s.pixels for s in self.specs)


def rgba_only_batch(device, n_per_size: int = 16) -> BatchWorkload:
    """Render the frames, upload them and build the batch (not yet prepared)."""
    specs = config3_frames(n_per_size=n_per_size)
    frames = [s.render_source() for s in specs]
    src = [(torch.from_numpy(r).to(device), torch.from_numpy(d).to(device)) for r, d in frames]
    dst = [torch.empty((s.height, s.width, 4), dtype=torch.uint8, device=device) for s in specs]
    jobs = [yoro.make_job(a, b, o, None, None, s.baseline_m, s.focal_px, s.target_eye, yoro.FILL_NEAREST_BG)
            for s, (a, b), o in zip(specs, src, dst)]
    return BatchWorkload(specs, frames, src, dst, yoro.StereoBatch(jobs, device=device))
