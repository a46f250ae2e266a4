"""yoro_stereo_batch_static (the batch with the library's fixed device job
table, for callers that cannot allocate) against yoro_stereo_batch on the
same jobs, bit for bit: two calls in a row, the second with fewer, smaller
frames, so the second reuses a table the first left behind."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2506_15183_amd.scenes.configs import config1_frame, config3_frames

pytestmark = pytest.mark.gpu


def _t():
    import torch

    from paper_2506_15183_amd import yoro

    return torch, yoro


def _jobs(torch, yoro, specs, extra):
    """Inputs and two output sets (reference, static) per frame; frames with
    extra=True also ask for depth and mask."""
    refs, stats, jr, js = [], [], [], []
    for s, ex in zip(specs, extra):
        r, d = s.render_source()
        a, b = torch.from_numpy(r).cuda(), torch.from_numpy(d).cuda()
        for outs, jl in ((refs, jr), (stats, js)):
            o = (torch.full((s.height, s.width, 4), 7, dtype=torch.uint8, device="cuda"),
                 torch.full((s.height, s.width), 7.0, dtype=torch.float32, device="cuda") if ex else None,
                 torch.full((s.height, s.width), 7, dtype=torch.uint8, device="cuda") if ex else None)
            outs.append((a, b, o))
            jl.append(yoro.make_job(a, b, *o, s.baseline_m, s.focal_px, s.target_eye, yoro.FILL_NEAREST_BG))
    return refs, stats, jr, js


def _same(refs, stats):
    for (_, _, o1), (_, _, o2) in zip(refs, stats):
        for t1, t2 in zip(o1, o2):
            if t1 is None:
                continue
            assert np.array_equal(t1.cpu().numpy().view(np.uint8), t2.cpu().numpy().view(np.uint8))


def test_static_batch_equals_workspace_batch_twice(cuda):
    torch, yoro = _t()
    # Call 1: four frames of the four headset sizes, mixed outputs.
    specs = config3_frames(n_per_size=1)
    refs, stats, jr, js = _jobs(torch, yoro, specs, [True, False, True, False])
    yoro.StereoBatch(jr).run()
    yoro.stereo_batch_static(js)
    torch.cuda.synchronize()
    _same(refs, stats)
    # Call 2: two small frames, both eyes: fewer records than the table holds
    # from call 1, so stale records must not be read.
    small = [config1_frame(0), config1_frame(1)]
    small[1].target_eye = 1
    refs2, stats2, jr2, js2 = _jobs(torch, yoro, small, [True, False])
    yoro.StereoBatch(jr2).run()
    yoro.stereo_batch_static(js2)
    torch.cuda.synchronize()
    _same(refs2, stats2)
    # The first call's outputs were not touched by the second.
    _same(refs, stats)


def test_static_batch_limits(cuda):
    torch, yoro = _t()
    spec = config1_frame(0)
    r, d = spec.render_source()
    a, b = torch.from_numpy(r).cuda(), torch.from_numpy(d).cuda()
    outs = [torch.empty_like(a) for _ in range(2)]
    j = yoro.make_job(a, b, outs[0], None, None, spec.baseline_m, spec.focal_px, 0, yoro.FILL_NEAREST_BG)
    L = yoro.load()
    arr = (yoro.Job * (yoro.STATIC_MAX_JOBS + 1))(*([j] * (yoro.STATIC_MAX_JOBS + 1)))
    assert L.yoro_stereo_batch_static(arr, yoro.STATIC_MAX_JOBS + 1, None) == yoro.ERR_INVALID_ARG
    assert b"1024" in L.yoro_last_error()
    jl = yoro.make_job(a, b, outs[1], None, None, spec.baseline_m, spec.focal_px, 0, yoro.FILL_LEARNED)
    with pytest.raises(yoro.YoroError) as ei:
        yoro.stereo_batch_static([jl])
    assert ei.value.status == yoro.ERR_UNSUPPORTED
