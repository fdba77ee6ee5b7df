"""GPU parity of the binning with per-tile culling (gs_bin_sort_culled)
against the oracle's tile test, through the C ABI.

Bars: with the records the GPU projection chose (the oracle's floats, or the
other correct rounding where it flagged one), the culled keys, values and
ranges are bit-exact against the oracle's binning of its kept copies; the
image, final_T and n_contrib equal bit for bit those of the same frame
binned without culling (the test never drops a tile a pixel can reach);
n_eval against the oracle's culled lists on sampled pixels; on the 4M-splat
scene, where the lists are too large to bin on the host, per-tile counts,
index sums and sums of squares against the oracle, plus sampled tiles list
for list.
"""
from dataclasses import replace
import math

import numpy as np
import pytest
import torch

from oracle import binning, core as ocore
from paper_2603_18707_amd import render, scenes
from tests import helpers as H
from tests.test_gpu_forward import _check_pixels, _check_projection, _np

pytestmark = pytest.mark.gpu


def _frames(scene, cam, kind, order, radius, params=None, capacity=None, kern=None):
    """The same frame binned with and without culling (one projection)."""
    print(f"[gpu] cull n={scene.n} {cam.width}x{cam.height} {kind}{order}/{radius}", flush=True)
    params = params or H.gpu_params()
    kern = kern or H.gpu_kernel(kind, order, radius)
    ds = render.to_device(scene)
    r0 = render.Rasterizer(kern, params, reuse_buffers=False)
    r1 = render.Rasterizer(kern, params, reuse_buffers=False, tile_cull=True)
    if capacity is not None:
        r1.capacity = capacity
    proj = r0.preprocess(ds, cam)
    b0 = r0.bin_sort_fit(proj, cam)
    b1 = r1.bin_sort_fit(proj, cam)
    f0 = r0.rasterize(proj, b0, cam, want_eval=True)
    f1 = r1.rasterize(proj, b1, cam, want_eval=True)
    torch.cuda.synchronize()
    return dict(proj=proj, binned=b1, **f1), dict(proj=proj, binned=b0, **f0)


def _same_image(g, g0):
    for k in ("image", "final_T", "n_contrib"):
        assert torch.equal(g[k], g0[k]), k
    assert bool((g["n_eval"] <= g0["n_eval"]).all())
    assert int(g["binned"]["num_keys"].item()) < int(g0["binned"]["num_keys"].item())


def _check_culled_binning(g, rec, cfg, gx, gy):
    b = g["binned"]
    K = int(b["num_keys"].item())
    assert int(b["overflow"].item()) == 0
    mask, nnear = ocore.cull_copy_mask(rec, replace(cfg, tile_cull=1))
    assert nnear == 0
    keys, vals, ranges = binning.bin_and_sort_fast(rec["rect"], rec["depth32"], gx, gy, copy_mask=mask)
    assert K == keys.shape[0]
    assert np.array_equal(_np(b["keys"])[:K].view(np.uint64), keys), "keys"
    assert np.array_equal(_np(b["vals"])[:K].view(np.uint32), vals), "vals"
    assert np.array_equal(_np(b["ranges"]).view(np.uint32), ranges), "ranges"
    return K, mask.size


@pytest.mark.parametrize("kind,order,radius,rect_mode", [
    ("exp", 1, "sigma3", 0), ("exp", 1, "exp_opacity", 1), ("poly", 1, "opacity", 0), ("poly", 1, "opacity", 1),
    ("poly", 2, "universal", 1), ("poly", 3, "opacity", 0), ("exp", 1, "sigma3", 1), ("exp", 1, "exp_opacity", 0),
    ("poly", 1, "sigma3", 1), ("poly", 1, "universal", 0), ("poly", 2, "opacity", 0), ("poly", 3, "universal", 1)])
def test_tiny_culled_full_frame(kind, order, radius, rect_mode):
    scene, cam = scenes.workload_tiny()
    scene.scales *= 2.0  # larger footprints: more tiles to drop
    cfg = H.oracle_cfg(kind, order, radius, rect_mode=rect_mode)
    o = ocore.project(scene, cam, cfg)
    g, g0 = _frames(scene, cam, kind, order, radius, params=H.gpu_params(rect_mode=rect_mode))
    exempt = (o["flags"] & ocore.SPLAT_EDGE_NEAR) != 0
    rec = _check_projection(g["proj"], o, exempt)
    if not exempt.any():  # else a rectangle may differ by a tile: no list to compare
        K, Kbox = _check_culled_binning(g, rec, cfg, 8, 8)
        assert K < Kbox
    _same_image(g, g0)
    pix = ocore.all_pixels(128, 128)
    ores = ocore.render_pixels(rec, replace(cfg, tile_cull=1), pix)
    nflag, err = _check_pixels(g, ores, pix, H.edge_flagged_tiles(o, 8, 8))
    assert not (ores["flags"] & ocore.PIX_CULL_NEAR).any()
    assert nflag <= H.flag_limit(kind, order, pix.shape[0])


def _records_frames(rec, cam, kind, order, radius):
    """Hand-made projected records binned with and without culling, then blended."""
    kern, params = H.gpu_kernel(kind, order, radius), H.gpu_params()
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()
    co = np.concatenate([rec["conic"], rec["opac"][:, None]], axis=1)
    proj = dict(n=rec["opac"].shape[0], means2d=dev(rec["means2d"], np.float32), conic_opacity=dev(co, np.float32),
                rgb=dev(rec["rgb"], np.float32), depth=dev(rec["depth32"], np.float32),
                rect=dev(rec["rect"], np.int32), tiles=dev(binning.tile_count(rec["rect"]), np.int32))
    out = []
    for cull in (True, False):
        r = render.Rasterizer(kern, params, reuse_buffers=False, tile_cull=cull)
        b = r.bin_sort_fit(proj, cam)
        out.append(dict(binned=b, **r.rasterize(proj, b, cam, want_eval=True)))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("kind,order,radius", [("poly", 1, "opacity"), ("exp", 1, "sigma3"), ("poly", 3, "opacity")])
def test_long_thin_footprints_culled(kind, order, radius):
    """Footprints 150-250 px long and about a pixel wide at many angles, each
    rectangle the whole grid: the blend's float evaluation is at its least
    accurate along their axis, and no pixel may change."""
    W, Hh = 320, 256
    cam = scenes.tiny_camera(W, Hh)
    rec = scenes.thin_footprint_records(W, Hh, n=40, seed=9)
    g, g0 = _records_frames(rec, cam, kind, order, radius)
    cfg = H.oracle_cfg(kind, order, radius)
    K, Kbox = _check_culled_binning(g, rec, cfg, 20, 16)
    print(f"K={K} box={Kbox}")
    assert K < 0.5 * Kbox
    _same_image(g, g0)


@pytest.mark.parametrize("kind,order,radius,rect_mode", [("poly", 1, "opacity", 1), ("exp", 1, "sigma3", 0),
                                                         ("poly", 1, "opacity", 0)])
def test_scene_scale_culled(kind, order, radius, rect_mode):
    """1M splats at 1080p: culled lists bit-exact, the image unchanged by
    culling, sampled pixels (n_eval included) against the oracle."""
    scene, cam = scenes.workload_scene()
    cfg = H.oracle_cfg(kind, order, radius, rect_mode=rect_mode)
    o = ocore.project(scene, cam, cfg)
    g, g0 = _frames(scene, cam, kind, order, radius, params=H.gpu_params(rect_mode=rect_mode))
    exempt = (o["flags"] & ocore.SPLAT_EDGE_NEAR) != 0
    assert exempt.sum() <= 4
    rec = _check_projection(g["proj"], o, exempt)
    _same_image(g, g0)
    if not exempt.any():
        K, Kbox = _check_culled_binning(g, rec, cfg, 120, 68)
        print(f"K={K} box copies={Kbox} kept={K / Kbox:.3f}")
    pix = scenes.sample_pixels(1920, 1080, 4096, seed=23)
    ores = ocore.render_pixels(rec, replace(cfg, tile_cull=1), pix)
    nflag, err = _check_pixels(g, ores, pix, H.edge_flagged_tiles(o, 120, 68))
    assert nflag <= H.flag_limit(kind, order, pix.shape[0])


def test_presort_route_and_overflow_culled():
    """A capacity of 2048 copies per tile or more takes the depth-first route;
    it must give the same lists. A capacity below the kept copies overflows
    with num_keys = the kept count."""
    scene, cam = scenes.workload_tiny()
    scene.scales *= 2.0
    kern, params = H.gpu_kernel("poly", 1, "opacity"), H.gpu_params(rect_mode=1)
    r = render.Rasterizer(kern, params, reuse_buffers=False, tile_cull=True)
    proj = r.preprocess(render.to_device(scene), cam)
    a = r.bin_sort_fit(proj, cam)
    K = int(a["num_keys"].item())
    big = r.bin_sort(proj, cam, capacity=2048 * 64 + 5)
    torch.cuda.synchronize()
    assert int(big["overflow"].item()) == 0 and int(big["num_keys"].item()) == K
    assert torch.equal(big["keys"][:K], a["keys"][:K]) and torch.equal(big["vals"][:K], a["vals"][:K])
    assert torch.equal(big["ranges"], a["ranges"])
    small = r.bin_sort(proj, cam, capacity=K - 1)
    torch.cuda.synchronize()
    assert int(small["overflow"].item()) == 1 and int(small["num_keys"].item()) == K
    assert not bool(small["ranges"].any())
    exact = r.bin_sort(proj, cam, capacity=K)
    torch.cuda.synchronize()
    assert int(exact["overflow"].item()) == 0 and torch.equal(exact["ranges"], a["ranges"])


def test_empty_and_all_culled_culled():
    cam = scenes.tiny_camera(64, 48)
    g, _ = _frames(scenes.tiny_scene(0, seed=1), cam, "poly", 1, "opacity")
    assert int(g["binned"]["num_keys"].item()) == 0 and np.all(_np(g["final_T"]) == 1.0)
    behind = scenes.tiny_scene(100, seed=2)
    behind.means3d[:, 2] = -behind.means3d[:, 2]
    g, _ = _frames(behind, cam, "exp", 1, "sigma3")
    assert int(g["binned"]["num_keys"].item()) == 0 and np.all(_np(g["image"]) == 0.0)
    # every splat below the opacity cut-off: rectangles may exist, no copy is kept
    faint = scenes.tiny_scene(200, seed=3)
    faint.opacities[:] = -12.0  # sigmoid ~ 6e-6 < eps
    g, g0 = _frames(faint, cam, "exp", 1, "sigma3")
    assert int(g["binned"]["num_keys"].item()) == 0 and int(g0["binned"]["num_keys"].item()) > 0
    assert torch.equal(g["image"], g0["image"])


def test_heavy_scene_culled():
    """4M heavy-tailed splats at 1080p, ellipse-box rectangles: per-tile kept
    counts, index sums and sums of squares against the oracle, sampled tiles
    list for list, the image unchanged by culling, sampled pixels."""
    scene, _ = scenes.workload_heavy()
    cam = scenes.orbit_camera(1920, 1080, 2.0 * math.pi * 3 / 8)
    cfg = H.oracle_cfg("poly", 1, "opacity", rect_mode=1)
    o = ocore.project(scene, cam, cfg)
    g, g0 = _frames(scene, cam, "poly", 1, "opacity", params=H.gpu_params(rect_mode=1))
    exempt = (o["flags"] & ocore.SPLAT_EDGE_NEAR) != 0
    assert not exempt.any()
    rec = _check_projection(g["proj"], o, exempt)
    _same_image(g, g0)
    gw, gh = 120, 68
    culled = replace(cfg, tile_cull=1)
    hist, near = ocore.cull_histogram(rec, culled, gw, gh)
    assert near.sum() == 0
    b = g["binned"]
    K = int(b["num_keys"].item())
    assert int(b["overflow"].item()) == 0 and K == int(hist.sum())
    ranges = _np(b["ranges"]).view(np.uint32).astype(np.int64)
    assert np.array_equal(ranges[:, 1] - ranges[:, 0], hist), "kept copies per tile"
    # index sums and sums of squares per tile (int64 on the device, exact)
    dev = b["vals"].device
    v = b["vals"][:K].long()
    tile_of = torch.repeat_interleave(torch.arange(gw * gh, device=dev), torch.from_numpy(hist).to(dev))
    s1 = torch.zeros(gw * gh, dtype=torch.int64, device=dev).index_add_(0, tile_of, v)
    s2 = torch.zeros(gw * gh, dtype=torch.int64, device=dev).index_add_(0, tile_of, v * v)
    # the oracle's sums from its per-copy decisions
    mask, nnear = ocore.cull_copy_mask(rec, culled)
    r = rec["rect"].astype(np.int64)
    cnt = np.maximum(r[:, 2] - r[:, 0] + 1, 0) * np.maximum(r[:, 3] - r[:, 1] + 1, 0)
    idx = np.repeat(np.arange(r.shape[0], dtype=np.int64), cnt)
    j = np.arange(idx.shape[0], dtype=np.int64) - (np.cumsum(cnt) - cnt)[idx]
    w = (r[:, 2] - r[:, 0] + 1)[idx]
    tid = (r[idx, 1] + j // w) * gw + r[idx, 0] + j % w
    idx, tid = idx[mask], tid[mask]
    del j, w
    o1 = np.bincount(tid, weights=None, minlength=gw * gh)
    assert np.array_equal(o1, hist)
    e1 = np.zeros(gw * gh, np.int64)
    e2 = np.zeros(gw * gh, np.int64)
    np.add.at(e1, tid, idx)
    np.add.at(e2, tid, idx * idx)
    assert np.array_equal(_np(s1), e1) and np.array_equal(_np(s2), e2), "kept splats per tile"
    rng = np.random.default_rng(5)
    for tid1 in [int(hist.argmax())] + [int(x) for x in rng.choice(gw * gh, size=5, replace=False)]:
        keep, nr = ocore.cull_tile_members(rec, culled, tid1 % gw, tid1 // gw)
        kb, vv = binning.tile_list(rec["rect"], rec["depth32"], tid1 % gw, tid1 // gw, keep=keep)
        lo, hi = ranges[tid1]
        assert np.array_equal(_np(b["vals"][lo:hi]).view(np.uint32), vv), f"tile {tid1}"
    pix = scenes.sample_pixels(1920, 1080, 1024, seed=34)
    ores = ocore.render_pixels(rec, culled, pix)
    nflag, err = _check_pixels(g, ores, pix, H.edge_flagged_tiles(o, gw, gh))
    print(f"K={K} box={int(cnt.sum())} kept={K / cnt.sum():.3f} flagged={nflag} max_err={err:.3g}")
    assert nflag <= H.flag_limit("poly", 1, pix.shape[0])


@pytest.mark.parametrize("radius", ["opacity", "universal"])
def test_order2_tile_range_fit(radius):
    """App. A's order-2 fit over every value a tile-culled renderer evaluates
    (gs_kernel_order2_tile_range): full frame against the oracle with the same
    coefficients, culled and unculled images equal."""
    from paper_2603_18707_amd import _lib
    rm = {"opacity": _lib.RADIUS_POLY_OPACITY, "universal": _lib.RADIUS_POLY_UNIVERSAL}[radius]
    kern = _lib.gs_kernel_order2_tile_range(rm)
    scene, cam = scenes.workload_tiny()
    scene.scales *= 2.0
    cfg = replace(H.oracle_cfg("poly", 2, radius, rect_mode=1), coeffs=tuple(kern.coeffs))
    o = ocore.project(scene, cam, cfg)
    g, g0 = _frames(scene, cam, "poly", 2, radius, params=H.gpu_params(rect_mode=1), kern=kern)
    exempt = (o["flags"] & ocore.SPLAT_EDGE_NEAR) != 0
    rec = _check_projection(g["proj"], o, exempt)
    if not exempt.any():
        _check_culled_binning(g, rec, cfg, 8, 8)
    _same_image(g, g0)
    pix = ocore.all_pixels(128, 128)
    ores = ocore.render_pixels(rec, replace(cfg, tile_cull=1), pix)
    nflag, err = _check_pixels(g, ores, pix, H.edge_flagged_tiles(o, 8, 8))
    assert nflag <= H.flag_limit("poly", 2, pix.shape[0])


@pytest.mark.parametrize("size", [(37, 23), (1, 1), (17, 200), (300, 40)])
def test_ragged_image_sizes_culled(size):
    """Partial tiles at the right and bottom edges (the test uses the whole
    tile's pixel-centre rectangle, inside the image or not) and splats far
    larger than the image."""
    W, Hh = size
    cam = scenes.tiny_camera(W, Hh)
    scene, _ = scenes.workload_tiny()
    scene.scales *= 4.0
    cfg = H.oracle_cfg("exp", 1, "sigma3", rect_mode=1)
    o = ocore.project(scene, cam, cfg)
    g, g0 = _frames(scene, cam, "exp", 1, "sigma3", params=H.gpu_params(rect_mode=1))
    exempt = (o["flags"] & ocore.SPLAT_EDGE_NEAR) != 0
    rec = _check_projection(g["proj"], o, exempt)
    gx, gy = (W + 15) // 16, (Hh + 15) // 16
    if not exempt.any():
        _check_culled_binning(g, rec, cfg, gx, gy)
    for k in ("image", "final_T", "n_contrib"):
        assert torch.equal(g[k], g0[k]), k
    pix = ocore.all_pixels(W, Hh)
    ores = ocore.render_pixels(rec, replace(cfg, tile_cull=1), pix)
    nflag, err = _check_pixels(g, ores, pix, H.edge_flagged_tiles(o, gx, gy))
    assert nflag <= H.flag_limit("exp", 1, pix.shape[0])


def test_saved_runs_fallback():
    """Workgroups whose rectangles hold more rows than their share of the
    space for saved runs recompute the runs in the emission kernel: faint
    splats (no pixel reaches eps) with whole-grid rectangles add 64 empty rows
    each beside small visible splats, so the kept copies, and with them the
    key capacity, stay small."""
    W = Hh = 1024
    cam = scenes.tiny_camera(W, Hh)
    rng = np.random.default_rng(17)
    n = 4096
    faint = np.arange(n) % 2 == 1
    m2 = rng.uniform(8, W - 8, size=(n, 2))
    tx, ty = (m2[:, 0] // 16).astype(np.int32), (m2[:, 1] // 16).astype(np.int32)
    rect = np.stack([tx, ty, tx, ty], 1).astype(np.int32)
    rect[faint] = (0, 0, 63, 63)
    rec = dict(means2d=m2, conic=np.tile([0.25, 0.0, 0.25], (n, 1)), opac=np.where(faint, 1e-3, 0.5),
               rgb=rng.uniform(0, 1, (n, 3)), depth32=rng.permutation(np.arange(1, n + 1)).astype(np.float32),
               rect=rect, flags=np.zeros(n, np.uint8))
    for k in ("means2d", "conic", "opac", "rgb"):
        rec[k] = rec[k].astype(np.float32).astype(np.float64)
    g, g0 = _records_frames(rec, cam, "exp", 1, "sigma3")
    K, Kbox = _check_culled_binning(g, rec, H.oracle_cfg("exp", 1, "sigma3"), 64, 64)
    assert 0 < K <= n // 2 and Kbox > 64 * K
    for k in ("image", "final_T", "n_contrib"):
        assert torch.equal(g[k], g0[k]), k


def test_conic_not_positive_definite_gets_no_copy():
    """Records whose conic is indefinite, singular or NaN, which the blend
    never includes, get no copy at all from the culled binning; the image is
    the unculled one."""
    W, Hh = 320, 256
    cam = scenes.tiny_camera(W, Hh)
    rec = scenes.thin_footprint_records(W, Hh)
    rec["conic"] = rec["conic"].copy()
    rec["conic"][2] = (1.0, 2.0, 1.0)        # indefinite
    rec["conic"][5] = (0.5, 0.0, 0.0)        # c = 0
    rec["conic"][8] = (np.nan, 0.0, 1.0)
    g, g0 = _records_frames(rec, cam, "poly", 1, "opacity")
    K, Kbox = _check_culled_binning(g, rec, H.oracle_cfg("poly", 1, "opacity"), 20, 16)
    b = g["binned"]
    vals = _np(b["vals"])[:K].view(np.uint32)
    assert not np.isin(vals, [2, 5, 8]).any()
    for k in ("image", "final_T", "n_contrib"):
        assert torch.equal(g[k], g0[k]), k


@pytest.mark.parametrize("scale", [1.0, 8.0])
def test_auto_culling_choice(scale):
    """tile_cull="auto" culls when the rectangles hold at least
    AUTO_CULL_TILES_PER_SPLAT tiles per visible splat; either way the frame is
    the unculled one."""
    scene, cam = scenes.workload_tiny()
    scene.scales *= scale
    kern, params = H.gpu_kernel("poly", 1, "opacity"), H.gpu_params()
    ds = render.to_device(scene)
    ra = render.Rasterizer(kern, params, reuse_buffers=False, tile_cull="auto")
    r0 = render.Rasterizer(kern, params, reuse_buffers=False)
    fa, f0 = ra.render(ds, cam), r0.render(ds, cam)
    torch.cuda.synchronize()
    tiles = _np(fa["proj"]["tiles"]).astype(np.int64)
    want = tiles.sum() >= render.AUTO_CULL_TILES_PER_SPLAT * (tiles > 0).sum()
    print(f"scale {scale}: {tiles.sum() / max(1, (tiles > 0).sum()):.2f} tiles per splat, culling {ra.culling}")
    assert ra.culling == want and ra.culling == (scale > 1.0)
    for k in ("image", "final_T", "n_contrib"):
        assert torch.equal(fa[k], f0[k]), k
    Ka, K0 = int(fa["binned"]["num_keys"].item()), int(f0["binned"]["num_keys"].item())
    assert (Ka < K0) == ra.culling
    with pytest.raises(ValueError):
        render.Rasterizer(kern, params, tile_cull="always")


def test_culled_without_tile_order():
    """tile_order = NULL (row-major dispatch of the per-tile sort): the same
    keys, values and ranges."""
    from paper_2603_18707_amd import _lib as L
    scene, cam = scenes.workload_tiny()
    scene.scales *= 2.0
    kern, params = H.gpu_kernel("exp", 1, "sigma3"), H.gpu_params(rect_mode=1)
    r = render.Rasterizer(kern, params, reuse_buffers=False, tile_cull=True)
    proj = r.preprocess(render.to_device(scene), cam)
    a = r.bin_sort_fit(proj, cam)
    K, cap = int(a["num_keys"].item()), a["capacity"]
    dev = a["keys"].device
    gw, gh = render.grid_of(cam)
    ws_bytes = L.gs_bin_sort_workspace(proj["n"], cap, gw * gh)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    keys = torch.full((cap,), -1, dtype=torch.int64, device=dev)
    vals = torch.full((cap,), -1, dtype=torch.int32, device=dev)
    ranges = torch.full((gw * gh, 2), -1, dtype=torch.int32, device=dev)
    nk = torch.zeros(1, dtype=torch.int64, device=dev)
    ov = torch.zeros(1, dtype=torch.int32, device=dev)
    L.gs_bin_sort_culled(kern, params, proj["n"], proj["depth"], proj["rect"], proj["tiles"], proj["means2d"],
                         proj["conic_opacity"], gw, gh, cap, ws, ws_bytes, keys, vals, ranges, None, nk, ov)
    torch.cuda.synchronize()
    assert int(ov.item()) == 0 and int(nk.item()) == K
    assert torch.equal(keys[:K], a["keys"][:K]) and torch.equal(vals[:K], a["vals"][:K])
    assert torch.equal(ranges, a["ranges"])


def test_runs_longer_than_a_digit_cycle():
    """Long horizontal footprints on a wide grid (128 x 4 tiles: two 5-bit tile
    digits), so kept runs cover the lowest digit's 32 values more than once
    (the emission counts a run's lowest digits as whole cycles plus a range of
    bins, which may wrap): keys equal to the oracle's culled lists, images
    equal to the unculled ones."""
    W, Hh = 2048, 64
    cam = scenes.tiny_camera(W, Hh)
    rng = np.random.default_rng(23)
    n = 300
    sx, sy = rng.uniform(150, 500, n), rng.uniform(0.8, 3.0, n)
    m2 = np.stack([rng.uniform(0, W, n), rng.uniform(0, Hh, n)], 1)
    rec = dict(means2d=m2, conic=np.stack([1 / sx**2, np.zeros(n), 1 / sy**2], 1), opac=rng.uniform(0.3, 0.99, n),
               rgb=rng.uniform(0, 1, (n, 3)), depth32=rng.permutation(np.arange(1, n + 1)).astype(np.float32),
               rect=np.tile(np.array([0, 0, W // 16 - 1, Hh // 16 - 1], np.int32), (n, 1)),
               flags=np.zeros(n, np.uint8))
    for k in ("means2d", "conic", "opac", "rgb"):
        rec[k] = rec[k].astype(np.float32).astype(np.float64)
    g, g0 = _records_frames(rec, cam, "poly", 1, "opacity")
    K, Kbox = _check_culled_binning(g, rec, H.oracle_cfg("poly", 1, "opacity"), W // 16, Hh // 16)
    print(f"K={K} box={Kbox}")
    assert 0 < K < Kbox
    for k in ("image", "final_T", "n_contrib"):
        assert torch.equal(g[k], g0[k]), k
