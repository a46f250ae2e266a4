"""Seeded synthetic inputs: scene recipes, the analytic ray-caster, random frames.

This package is the only code that both the GPU path's tests and the CPU
oracle's tests draw inputs from.  It holds none of the reprojection method's
arithmetic (no disparity, no scatter, no fill): it only makes the rendered
eye's colour + depth G-buffer (Section 3.2) and the true other eye, and random
frames shaped like them.
"""
from .raycast import Scene, render, render_pair, make_scene  # noqa: F401
from .configs import (  # noqa: F401
    FrameSpec,
    config1_frame,
    config2_frame,
    config3_frames,
    training_window,
    frame_seed,
)
from .synth import random_frame, random_rows  # noqa: F401
