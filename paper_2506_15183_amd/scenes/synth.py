"""Random frames for parity and edge-case tests (numpy PCG64, seeded).

Depths are drawn from a small set so that several sources of a row collide on
one target, and special values (+inf, NaN, 0, negative, tiny) are sprinkled
in on request, so the depth test and the skip rules are all exercised.
"""
from __future__ import annotations

import numpy as np


def random_frame(seed: int, width: int, height: int, *, depth_levels=None, special_frac: float = 0.0,
                 zmin: float = 0.3, zmax: float = 50.0):
    """(rgba uint8 [H, W, 4], depth float32 [H, W]).

    depth_levels: None draws log-uniform depths in [zmin, zmax]; an int k
    draws from k fixed log-uniform levels (forces equal-depth runs and many
    collisions).  special_frac of the pixels get one of +inf, NaN, 0, -0,
    -1, a tiny positive value (disparity beyond the frame) or 1e6.
    """
    rng = np.random.default_rng(seed)
    rgba = rng.integers(0, 256, size=(height, width, 4), dtype=np.uint8)
    if depth_levels is None:
        depth = np.exp(rng.uniform(np.log(zmin), np.log(zmax), size=(height, width))).astype(np.float32)
    else:
        levels = np.exp(rng.uniform(np.log(zmin), np.log(zmax), size=int(depth_levels))).astype(np.float32)
        depth = levels[rng.integers(0, len(levels), size=(height, width))]
    if special_frac > 0:
        specials = np.array([np.inf, np.nan, 0.0, -0.0, -1.0, 1e-30, 1e6], dtype=np.float32)
        sel = rng.random(size=(height, width)) < special_frac
        depth = depth.copy()
        depth[sel] = specials[rng.integers(0, len(specials), size=int(sel.sum()))]
    return np.ascontiguousarray(rgba), np.ascontiguousarray(depth.astype(np.float32))


def random_rows(seed: int, width: int, height: int, hole_frac: float = 0.3):
    """A warped-looking frame for the stand-alone fill: (rgba, depth, mask).

    mask 0 marks hits, 1 marks holes; hole pixels carry RGBA 0 and depth +inf.
    """
    rng = np.random.default_rng(seed)
    rgba = rng.integers(0, 256, size=(height, width, 4), dtype=np.uint8)
    levels = np.exp(rng.uniform(np.log(0.3), np.log(50.0), size=6)).astype(np.float32)
    depth = levels[rng.integers(0, len(levels), size=(height, width))]
    # Holes come in runs, as disocclusions do.
    mask = np.zeros((height, width), dtype=np.uint8)
    for y in range(height):
        x = 0
        while x < width:
            if rng.random() < hole_frac / 4:
                run = int(rng.integers(1, 24))
                mask[y, x:x + run] = 1
                x += run
            x += 1
    rgba[mask != 0] = 0
    depth = depth.copy()
    depth[mask != 0] = np.inf
    return np.ascontiguousarray(rgba), np.ascontiguousarray(depth.astype(np.float32)), mask
