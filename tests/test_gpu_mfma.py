"""GPU parity of the matrix-core blend (gs_rasterize_fwd_mfma: the quadric of
a block of pixels against a batch of splats as an MFMA product, Sec. 5.1)
against the FP64 oracle, through the C ABI.

Its quadric rounds differently from the vector blend's: each splat's
coefficients expand t = x_e - Q about the centre of an 8x8 pixel block in
double and round once, and the product accumulates six terms of up to a few
hundred where t is near 0, so t is within ~1.5e-5 of the FP64 value there
(measured on long, thin footprints, tests/test_quadric_forms.py). Inclusion
decisions within that distance of the threshold may go either way, so the
oracle's "too close to call" band on alpha is widened to MFMA_ALPHA_BAND, the
kernel's slope at the threshold times that error, with a factor 3 of
headroom. Everything else is the vector blend's bar: unflagged pixels within
2e-4, flagged ones within the oracle's reach, blended counts equal.
"""
from dataclasses import replace

import numpy as np
import pytest
import torch

from oracle import binning, core as ocore
from paper_2603_18707_amd import render, scenes
from tests import helpers as H
from tests.test_gpu_forward import KERNELS, _check_pixels, _check_projection, _np

pytestmark = pytest.mark.gpu

# |d alpha / d t| at the threshold (o' = 1) x 1.5e-5 x 3
MFMA_ALPHA_BAND = {("exp", 1): 1.5e-7, ("poly", 1): 1e-5, ("poly", 2): 1.2e-5, ("poly", 3): 2.5e-5}
# flagged share allowed: the vector blend's limit scaled by the band ratio
MFMA_FLAG_RATE = {k: H.FLAG_RATE[k] * 5.0 for k in H.FLAG_RATE}


def _cfg(kind, order, radius, **kw):
    key = (kind, order if kind == "poly" else 1)
    return replace(H.oracle_cfg(kind, order, radius, **kw), alpha_band=MFMA_ALPHA_BAND[key])


def _flag_limit(kind, order, npix):
    return max(2.0, MFMA_FLAG_RATE[(kind, order if kind == "poly" else 1)] * npix)


def _frames(scene, cam, kind, order, radius, params=None):
    """The same frame through the vector blend and the matrix-core blend."""
    print(f"[gpu] mfma render n={scene.n} {cam.width}x{cam.height} {kind}{order}/{radius}", flush=True)
    r = render.Rasterizer(H.gpu_kernel(kind, order, radius), params or H.gpu_params())
    ds = render.to_device(scene)
    out = r.render(ds, cam, want_eval=True)
    vec = {k: _np(out[k]).copy() for k in ("image", "final_T", "n_contrib", "last_contrib", "n_eval")}
    r.mfma = True
    m = r.rasterize(out["proj"], out["binned"], cam, want_eval=True)
    torch.cuda.synchronize()
    return dict(proj=out["proj"], binned=out["binned"], **m), vec


@pytest.mark.parametrize("kind,order,radius", KERNELS)
def test_tiny_full_frame_mfma(kind, order, radius):
    scene, cam = scenes.workload_tiny()
    cfg = _cfg(kind, order, radius)
    o = ocore.project(scene, cam, cfg)
    g, vec = _frames(scene, cam, kind, order, radius)
    rec = _check_projection(g["proj"], o, (o["flags"] & ocore.SPLAT_EDGE_NEAR) != 0)
    pix = ocore.all_pixels(128, 128)
    ores = ocore.render_pixels(rec, cfg, pix)
    nflag, err = _check_pixels(g, ores, pix, H.edge_flagged_tiles(o, 8, 8))
    print(f"flagged={nflag} max_err={err:.3g}")
    assert nflag <= _flag_limit(kind, order, pix.shape[0])
    # against the vector blend: the same blended counts wherever the oracle
    # flags nothing, colours within float rounding of each other
    good = ores["flags"] == 0
    d = np.abs(_np(g["image"]) - vec["image"]).max(axis=0).ravel()
    assert d[good].max() <= 2e-5, d[good].max()
    assert np.array_equal(_np(g["n_contrib"]).ravel()[good], vec["n_contrib"].ravel()[good])


@pytest.mark.parametrize("kind,order,radius", [("poly", 1, "opacity"), ("exp", 1, "sigma3"), ("poly", 3, "opacity")])
def test_dense_tiles_and_termination_mfma(kind, order, radius):
    """Doubled scales: long lists (many 32-splat steps per wave) and pixels
    that stop in either half of a step, including the replayed case."""
    scene, cam = scenes.workload_tiny()
    scene.scales *= 2.0
    cfg = _cfg(kind, order, radius)
    o = ocore.project(scene, cam, cfg)
    g, vec = _frames(scene, cam, kind, order, radius)
    rec = _check_projection(g["proj"], o, (o["flags"] & ocore.SPLAT_EDGE_NEAR) != 0)
    pix = ocore.all_pixels(128, 128)
    ores = ocore.render_pixels(rec, cfg, pix)
    nflag, err = _check_pixels(g, ores, pix, H.edge_flagged_tiles(o, 8, 8))
    ends = np.array([o["tiles"].sum()])  # more than any list: a pixel whose n_eval is below its list stopped
    stopped = int((_np(g["final_T"]).ravel() < 2e-4).sum())
    print(f"flagged={nflag} max_err={err:.3g} stopped={stopped}")
    assert nflag <= _flag_limit(kind, order, pix.shape[0])
    assert stopped > 100 and ends[0] > 0  # pixels that terminated early


def _records_frame_mfma(rec, cam, kind, order, radius):
    r = render.Rasterizer(H.gpu_kernel(kind, order, radius), H.gpu_params(), mfma=True)
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()
    co = np.concatenate([rec["conic"], rec["opac"][:, None]], axis=1)
    proj = dict(n=rec["opac"].shape[0], means2d=dev(rec["means2d"], np.float32), conic_opacity=dev(co, np.float32),
                rgb=dev(rec["rgb"], np.float32), depth=dev(rec["depth32"], np.float32),
                rect=dev(rec["rect"], np.int32), tiles=dev(binning.tile_count(rec["rect"]), np.int32))
    b = r.bin_sort_fit(proj, cam)
    out = r.rasterize(proj, b, cam, want_eval=True)
    torch.cuda.synchronize()
    return {k: _np(v).copy() for k, v in out.items() if v is not None}


@pytest.mark.parametrize("kind,order,radius", [("poly", 1, "opacity"), ("exp", 1, "sigma3"), ("poly", 3, "opacity")])
def test_long_thin_footprints_mfma(kind, order, radius):
    """Every pixel within 2e-4 of the oracle for footprints whose expanded
    quadric cancels by five orders of magnitude along their axis: the
    block-centred expansion in double keeps the product's terms small."""
    W, Hh = 320, 256
    cam = scenes.tiny_camera(W, Hh)
    rec = scenes.thin_footprint_records(W, Hh)
    g = _records_frame_mfma(rec, cam, kind, order, radius)
    cfg = _cfg(kind, order, radius)
    pix = ocore.all_pixels(W, Hh)
    ores = ocore.render_pixels(rec, cfg, pix)
    good = ores["flags"] == 0
    err = np.abs(g["image"].reshape(3, -1).T - ores["color"]).max(axis=1)
    print(f"flagged={int((~good).sum())} max_err={err[good].max():.3g}")
    assert (~good).sum() <= _flag_limit(kind, order, pix.shape[0])
    assert err[good].max() <= 2e-4
    assert np.all(err[~good] <= ores["reach"][~good, 0] + 2e-4)
    assert np.array_equal(g["n_contrib"].ravel()[good], ores["n_contrib"][good])


@pytest.mark.parametrize("size", [(37, 61), (200, 90), (301, 157)])
def test_ragged_image_sizes_mfma(size):
    W, Hh = size
    scene, _ = scenes.workload_tiny()
    cam = scenes.tiny_camera(W, Hh)
    cfg = _cfg("poly", 1, "opacity")
    o = ocore.project(scene, cam, cfg)
    g, vec = _frames(scene, cam, "poly", 1, "opacity")
    gx, gy = (W + 15) // 16, (Hh + 15) // 16
    rec = _check_projection(g["proj"], o, (o["flags"] & ocore.SPLAT_EDGE_NEAR) != 0)
    pix = ocore.all_pixels(W, Hh)
    ores = ocore.render_pixels(rec, cfg, pix)
    nflag, _ = _check_pixels(g, ores, pix, H.edge_flagged_tiles(o, gx, gy))
    assert nflag <= _flag_limit("poly", 1, pix.shape[0])


@pytest.fixture(scope="module")
def scene_1m():
    return scenes.workload_scene()


@pytest.mark.parametrize("kind,order,radius", [("poly", 1, "opacity"), ("exp", 1, "sigma3"), ("poly", 2, "opacity"),
                                               ("poly", 3, "universal")])
def test_scene_scale_sampled_mfma(scene_1m, kind, order, radius):
    """1M splats, SH degree 3, 1920x1080: 4096 sampled pixels against the oracle."""
    scene, cam = scene_1m
    cfg = _cfg(kind, order, radius)
    o = ocore.project(scene, cam, cfg)
    g, vec = _frames(scene, cam, kind, order, radius)
    exempt = (o["flags"] & ocore.SPLAT_EDGE_NEAR) != 0
    rec = _check_projection(g["proj"], o, exempt)
    pix = scenes.sample_pixels(1920, 1080, 4096, seed=21)
    ores = ocore.render_pixels(rec, cfg, pix)
    nflag, err = _check_pixels(g, ores, pix, H.edge_flagged_tiles(o, 120, 68))
    print(f"flagged={nflag} max_err={err:.3g}")
    assert nflag <= _flag_limit(kind, order, pix.shape[0])
    d = np.abs(_np(g["image"]) - vec["image"]).max()
    print(f"max |mfma - vector| over the frame {d:.3g}")


def test_rejects_culled_lists():
    with pytest.raises(ValueError):
        render.Rasterizer(H.gpu_kernel("poly", 1, "opacity"), tile_cull=True, mfma=True)
