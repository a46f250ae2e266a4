"""GPU tests of hole-tile inference: the tile kernels against host slicing
and the oracle's composite, and the tiled learned fill against the
whole-frame learned fill (bit-exact: a crop reaching boundary_reach() pixels
past its block computes the same residuals there as the whole frame)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import unet as OU

pytestmark = pytest.mark.gpu


def _t():
    import torch

    from paper_2506_15183_amd import unet as G

    return torch, G


def _frame(rng, h, w, hole_tiles=None, tile=128):
    """Plain-fill-like frame; holes everywhere, or only inside the listed blocks."""
    rgba = rng.integers(0, 256, size=(h, w, 4), dtype=np.uint8)
    depth = np.exp(rng.uniform(np.log(0.2), np.log(80), size=(h, w))).astype(np.float32)
    hole = rng.random((h, w)) < 0.25
    if hole_tiles is not None:
        keep = np.zeros((h, w), bool)
        for tx, ty in hole_tiles:
            keep[ty * tile:(ty + 1) * tile, tx * tile:(tx + 1) * tile] = True
        hole &= keep
    mask = hole.astype(np.uint8) * rng.integers(1, 3, size=(h, w), dtype=np.uint8)
    depth[mask == 2] = np.inf
    return rgba, depth, mask


def _dev(torch, *arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def _strong_head(G, seed):
    """Random weights with the head at full He scale, so residuals move the
    composite by many levels (a differing residual would show)."""
    p = G.init_params(seed)
    p[-1] = p[-1] * 100.0
    return p


def test_tile_kernels_match_host(cuda):
    torch, G = _t()
    L = G.nnlib()
    rng = np.random.default_rng(11)
    h, w, tile, crop = 264, 392, 128, 256
    rgba, depth, mask = _frame(rng, h, w, hole_tiles=[(0, 0), (3, 1), (2, 2)])
    a, d, m = _dev(torch, rgba, depth, mask)
    ntx, nty = -(-w // tile), -(-h // tile)
    counts = torch.full((ntx * nty,), 7, dtype=torch.int32, device="cuda")
    G._ok(L.yoro_nn_tile_holes(G._p(m), w, h, tile, G._p(counts), None))
    want = np.array([[np.count_nonzero(mask[y:y + tile, x:x + tile]) for x in range(0, w, tile)]
                     for y in range(0, h, tile)])
    assert np.array_equal(counts.cpu().numpy().reshape(nty, ntx), want)
    plan = G.tile_plan(counts.cpu().numpy(), h, w)
    k = plan.shape[0]
    assert k == 3
    pd, = _dev(torch, plan)
    cr = torch.empty((k, crop, crop, 4), dtype=torch.uint8, device="cuda")
    cd = torch.empty((k, crop, crop), dtype=torch.float32, device="cuda")
    cm = torch.empty((k, crop, crop), dtype=torch.uint8, device="cuda")
    G._ok(L.yoro_nn_gather_crops(G._p(a), G._p(d), G._p(m), w, h, G._p(pd), k, crop, G._p(cr), G._p(cd), G._p(cm),
                                 None))
    res = rng.normal(0, 0.2, size=(k, crop, crop, 3)).astype(np.float32)
    rd, = _dev(torch, res)
    out = a.clone()
    G._ok(L.yoro_nn_composite_tiles(G._p(rd), G._p(pd), k, crop, tile, G._p(a), G._p(m), w, h, G._p(out), None))
    torch.cuda.synchronize()
    want_out = rgba.copy()
    for i, (ox, oy, tx, ty) in enumerate(plan.tolist()):
        sl = (slice(oy, oy + crop), slice(ox, ox + crop))
        assert np.array_equal(cr[i].cpu().numpy(), rgba[sl])
        assert np.array_equal(cd[i].cpu().numpy(), depth[sl])
        assert np.array_equal(cm[i].cpu().numpy(), mask[sl])
        comp = OU.composite(res[i], rgba[sl], mask[sl])
        bx, by = min(tile, w - tx), min(tile, h - ty)
        want_out[ty:ty + by, tx:tx + bx] = comp[ty - oy:ty - oy + by, tx - ox:tx - ox + bx]
    assert np.array_equal(out.cpu().numpy(), want_out)


def test_crop_residuals_equal_whole_frame_residuals(cuda):
    torch, G = _t()
    rng = np.random.default_rng(12)
    h, w = 384, 512
    rgba, depth, mask = _frame(rng, h, w)
    a, d, m = _dev(torch, rgba[None], depth[None], mask[None])
    net = G.UNet("cuda", params=_strong_head(G, 3))
    b = net.buffers(1, h, w)
    net.forward(a, d, m, b)
    full = b.res.view(h, w, 3).clone()
    ntx, nty = -(-w // G.TILE), -(-h // G.TILE)
    plan = G.tile_plan(np.ones(ntx * nty, np.int32), h, w)
    k, crop = plan.shape[0], G.TILE + 2 * G.HALO
    o, = _dev(torch, plan)
    cr = torch.empty((k, crop, crop, 4), dtype=torch.uint8, device="cuda")
    cd = torch.empty((k, crop, crop), dtype=torch.float32, device="cuda")
    cm = torch.empty((k, crop, crop), dtype=torch.uint8, device="cuda")
    L = G.nnlib()
    G._ok(L.yoro_nn_gather_crops(G._p(a), G._p(d), G._p(m), w, h, G._p(o), k, crop, G._p(cr), G._p(cd), G._p(cm),
                                 None))
    bc = net.buffers(k, crop, crop)
    net.forward(cr, cd, cm, bc)
    part = bc.res.view(k, crop, crop, 3)
    torch.cuda.synchronize()
    for i, (ox, oy, tx, ty) in enumerate(plan.tolist()):
        got = part[i, ty - oy:ty - oy + G.TILE, tx - ox:tx - ox + G.TILE]
        want = full[ty:ty + G.TILE, tx:tx + G.TILE]
        assert torch.equal(got, want), (i, tx, ty)
    # And the reach is real: a crop's own border residuals differ from the frame's.
    ox, oy = plan[k // 2, :2]
    assert oy > 0 and not torch.equal(part[k // 2, :8], full[oy:oy + 8, ox:ox + crop])


@pytest.mark.parametrize("chunk", [32, 2])
def test_fill_tiles_equals_whole_frame_fill(cuda, chunk):
    torch, G = _t()
    rng = np.random.default_rng(13)
    h, w = 520, 648
    blocks = [(0, 0), (4, 0), (2, 2), (5, 4), (1, 3)]
    rgba, depth, mask = _frame(rng, h, w, hole_tiles=blocks)
    a, d, m = _dev(torch, rgba, depth, mask)
    net = G.UNet("cuda", params=_strong_head(G, 4))
    whole = net.fill(a[None], d[None], m[None])[0]
    tiled, k = net.fill_tiles(a, d, m, chunk=chunk)
    torch.cuda.synchronize()
    assert k == len(blocks)
    assert torch.equal(tiled, whole)
    changed = (tiled != a).any(-1).cpu().numpy()
    assert changed.any() and not changed[mask == 0].any()
    # In place (out is the plain frame) gives the same result: every crop is
    # gathered before any block is written.
    inplace = a.clone()
    net.fill_tiles(inplace, d, m, out=inplace, chunk=chunk)
    torch.cuda.synchronize()
    assert torch.equal(inplace, whole)
    # A frame without holes runs no crop and is copied unchanged.
    m0 = torch.zeros_like(m)
    out, k0 = net.fill_tiles(a, d, m0)
    assert k0 == 0 and torch.equal(out, a)


def test_fill_tiles_full_headset_frame(cuda):
    """A 1832 x 1920 frame warped by the plain path: tiled == whole-frame fill."""
    torch, G = _t()
    from paper_2506_15183_amd import yoro
    from paper_2506_15183_amd.scenes.configs import config2_frame

    spec = config2_frame(0)
    rgba, depth = spec.render_source()
    a, d = _dev(torch, rgba, depth)
    out, dz, mk = yoro.reproject(a, d, spec.baseline_m, spec.focal_px, spec.target_eye, yoro.FILL_NEAREST_BG)
    net = G.UNet("cuda", params=_strong_head(G, 5))
    whole = net.fill(out[None], dz[None], mk[None])[0]
    tiled, k = net.fill_tiles(out, dz, mk)
    torch.cuda.synchronize()
    h, w = depth.shape
    assert 0 < k <= (-(-h // G.TILE)) * (-(-w // G.TILE))
    assert torch.equal(tiled, whole)


def test_native_forward_equals_the_python_sequence(cuda):
    """yoro_model_residual / yoro_model_fill (the library's own forward
    sequence) against the Python sequencer over the same layer kernels."""
    torch, G = _t()
    L = G.nnlib()
    rng = np.random.default_rng(14)
    n, h, w = 3, 72, 96
    frames = [_frame(rng, h, w) for _ in range(n)]
    a, d, m = _dev(torch, *[np.stack([f[i] for f in frames]) for i in range(3)])
    net = G.UNet("cuda", params=_strong_head(G, 6))
    b = net.buffers(n, h, w)
    net.forward(a, d, m, b)
    res = torch.empty((n * h * w, 3), dtype=torch.float32, device="cuda")
    nbytes = L.yoro_model_workspace_bytes(n, h, w)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    G._ok(L.yoro_model_residual(G._p(net.wf), G._p(a), G._p(d), G._p(m), n, h, w, G._p(res), G._p(ws), nbytes, None))
    torch.cuda.synchronize()
    assert torch.equal(res, b.res)
    assert torch.equal(net.fill_native(a, d, m), net.fill(a, d, m))
    # Packing FP32 masters through the library gives the same weights.
    wf = torch.empty(L.yoro_model_weights_bytes() // 2, dtype=torch.bfloat16, device="cuda")
    G._ok(L.yoro_model_pack(G._p(net.master), G._p(wf), None))
    torch.cuda.synchronize()
    assert torch.equal(wf.view(torch.int16), net.wf.view(torch.int16))
    # A short workspace is refused before anything runs.
    assert L.yoro_model_fill(G._p(net.wf), G._p(a), G._p(d), G._p(m), n, h, w, G._p(a), G._p(ws), nbytes - 1,
                             None) == 3


@pytest.mark.parametrize("band,halo", [(256, 64), (128, 64), (512, 64)])
def test_fill_bands_equals_whole_frame_fill(cuda, band, halo):
    """Full-width bands (yoro_model_fill_bands), in place and out of place,
    with and without skipped bands, equal the whole-frame learned fill bit for
    bit at the serving sizes (short last bands included)."""
    torch, G = _t()
    rng = np.random.default_rng(band + halo)
    net = G.UNet("cuda", params=_strong_head(G, 5))
    for (w, h) in ((1440, 1600), (1832, 1920), (2160, 2160), (256, 200)):
        rgba, depth, mask = _frame(rng, h, w)
        a, d, m = _dev(torch, rgba, depth, mask)
        want = net.fill_native(a[None], d[None], m[None])[0]
        got = net.fill_bands(a, d, m, band=band, halo=halo)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (w, h)
        inplace = a.clone()
        net.fill_bands(inplace, d, m, out=inplace, band=band, halo=halo)
        torch.cuda.synchronize()
        assert torch.equal(inplace, want), (w, h, "in place")
    # Holes in two bands only: the other bands may be skipped.
    w, h = 1832, 1920
    rgba, depth, mask = _frame(rng, h, w)
    keep = np.zeros((h, w), bool)
    keep[300:340] = True
    keep[1500:1510] = True
    mask[~keep] = 0
    a, d, m = _dev(torch, rgba, depth, mask)
    nb = -(-h // band)
    flags = [int(mask[b * band:(b + 1) * band].any()) for b in range(nb)]
    assert 0 < sum(flags) < nb
    want = net.fill_native(a[None], d[None], m[None])[0]
    got = a.clone()
    net.fill_bands(got, d, m, out=got, band=band, halo=halo, band_has_holes=flags)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
