"""Host logic of hole-tile inference: the boundary reach of the network
(pinned on the oracle: a crop's outputs far enough from its edges equal the
whole frame's) and the crop placement of tile_plan."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import unet as OU
from paper_2506_15183_amd import unet as U


def test_boundary_reach_value():
    # 2 convs (2) -> pool (1) -> 2 convs (3) -> pool (2) -> 2 convs (4) -> pool (2)
    # -> 2 convs (4) -> up+conv (9) -> 2 convs (11) -> up+conv (23) -> (25)
    # -> up+conv (51) -> (53) -> head (54).
    assert U.boundary_reach() == 54
    assert U.HALO >= U.boundary_reach() and U.HALO % 8 == 0 and U.TILE % 8 == 0


def test_crop_equals_whole_frame_beyond_the_reach():
    """Oracle forward (float64, no rounding) on a 192 x 192 frame and on a
    128 x 128 crop at (32, 32): outputs at least boundary_reach() pixels from
    both crop edges agree; some output closer than that differs."""
    rng = np.random.default_rng(5)
    params = [rng.normal(0, np.sqrt(2.0 / (9 * cin)), size=(9, cout, cin)) for _, cin, cout in OU.LAYERS]
    x = rng.uniform(0, 1, size=(1, 192, 192, 5))
    full, _ = OU.forward(params, x, rounding=False)
    o, c = 32, 128
    part, _ = OU.forward(params, x[:, o:o + c, o:o + c], rounding=False)
    r = U.boundary_reach()
    inner = slice(r, c - r)
    ref = full[:, o:o + c, o:o + c]
    scale = np.abs(ref).max()
    assert np.abs(part[:, inner, inner] - ref[:, inner, inner]).max() <= 1e-12 * scale
    # The reach is not loose by a pooling cell: the band just inside it differs.
    band = np.abs(part - ref)[:, r - 8:r, r:c - r]
    assert band.max() > 1e-6 * scale


@pytest.mark.parametrize("h,w", [(1832, 1920), (1600, 1440), (2160, 2160), (256, 256), (264, 392)])
def test_tile_plan_places_every_crop_inside_and_away_from_the_block(h, w):
    rng = np.random.default_rng(h * 7 + w)
    T, Hh = U.TILE, U.HALO
    ntx, nty = -(-w // T), -(-h // T)
    counts = rng.integers(0, 3, size=ntx * nty) * (rng.uniform(size=ntx * nty) < 0.5)
    counts[0] = counts[-1] = 5
    plan = U.tile_plan(counts, h, w)
    crop = T + 2 * Hh
    assert plan.shape == (int((counts > 0).sum()), 4) and plan.dtype == np.int32
    want = {(int(i % ntx) * T, int(i // ntx) * T) for i in np.flatnonzero(counts)}
    assert {tuple(t) for t in plan[:, 2:].tolist()} == want
    for ox, oy, tx, ty in plan.tolist():
        assert ox % 8 == 0 and oy % 8 == 0
        assert 0 <= ox and ox + crop <= w and 0 <= oy and oy + crop <= h
        bx, by = min(tx + T, w), min(ty + T, h)
        assert ox <= tx and bx <= ox + crop and oy <= ty and by <= oy + crop
        # Each crop edge is a frame edge or at least HALO from the block.
        assert ox == 0 or tx - ox >= Hh
        assert oy == 0 or ty - oy >= Hh
        assert ox + crop == w or ox + crop - bx >= Hh
        assert oy + crop == h or oy + crop - by >= Hh


def test_tile_plan_rejects_small_or_unaligned_frames():
    with pytest.raises(ValueError):
        U.tile_plan(np.ones(4), 200, 200)
    with pytest.raises(ValueError):
        U.tile_plan(np.ones(9), 260, 300)
    assert U.tile_plan(np.zeros(9, np.int32), 384, 384).shape == (0, 4)


def test_library_layer_layout_matches_the_network_table():
    """The library's packed-weight layout (yoro_model_layout) is the one the
    Python sequencer's flat parameter arrays use."""
    import ctypes

    L = U.nnlib()
    cin = (ctypes.c_int32 * 18)()
    cout = (ctypes.c_int32 * 18)()
    off = (ctypes.c_int64 * 19)()
    assert L.yoro_model_layout(cin, cout, off) == 0
    shapes = [(9, U._pad32(co) if name == "head" else co, U._pad32(ci)) for name, ci, co in U.ARCH]
    assert [(9, cout[i], cin[i]) for i in range(18)] == shapes
    sizes = np.cumsum([0] + [int(np.prod(sh)) for sh in shapes])
    assert list(off) == sizes.tolist()
    assert L.yoro_model_weights_bytes() == 2 * sizes[-1]
    # Workspace sizes are defined for multiples of 8 only.
    assert L.yoro_model_workspace_bytes(1, 256, 256) > 0
    assert L.yoro_model_workspace_bytes(1, 250, 256) == 0
    assert L.yoro_model_tiles_workspace_bytes(10, 4, 128, 64) > L.yoro_model_tiles_workspace_bytes(4, 4, 128, 64)
