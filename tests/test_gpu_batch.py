"""Batched multi-view rendering (gs_render_batched) on the GPU.

Against the FP64 oracle: every pixel of every view of a small ragged batch
and sampled pixels of six views of the full 96-view workload (colour, T and
blended counts at the forward's bar), and each view's key count against the
oracle's tile count.

The batched frame must also equal per-view gs_rasterize_fwd frames bit for bit
(same per-tile lists, same blend code), including views of an empty scene and
ragged resolutions; a captured HIP graph must reproduce the eager result on
every replay, with eager work and synchronisations between replays. At the
batched workload's full size (6 scenes, 100k-2M splats, 96 views) sampled
views are compared bit for bit as well.
"""
import numpy as np
import pytest
import torch

from oracle import core as ocore
from paper_2603_18707_amd import batch, render, scenes
from tests import helpers as H
from tests.test_gpu_forward import _check_pixels

pytestmark = pytest.mark.gpu


def _per_view(dev_scenes, views, kernel_args, params_kw=None):
    outs = []
    for si, cam in views:
        r = render.Rasterizer(H.gpu_kernel(*kernel_args), H.gpu_params(**(params_kw or {})))
        f = r.render(dev_scenes[si], cam)
        outs.append({k: f[k].detach().cpu().numpy().copy() for k in ("image", "final_T", "n_contrib", "last_contrib")})
    return outs


def _small_batch():
    sc = [scenes.tiny_scene(2000, seed=21, sh_degree=3), scenes.tiny_scene(0, seed=22, sh_degree=3),
          scenes.tiny_scene(4500, seed=23, sh_degree=3)]
    sc[2].scales *= 2.5
    cams = [scenes.tiny_camera(128, 128), scenes.tiny_camera(37, 61), scenes.pinhole(200, 90, 70.0),
            scenes.tiny_camera(16, 16), scenes.pinhole(301, 157, 50.0)]
    views = [(0, cams[0]), (2, cams[1]), (1, cams[2]), (2, cams[2]), (0, cams[3]), (2, cams[4]), (0, cams[4])]
    return sc, views


def _compare(br, ref):
    for i, r in enumerate(ref):
        o = br.view_outputs(i)
        for k in r:
            got = o[k].cpu().numpy()
            assert np.array_equal(got, r[k]), (i, k, np.abs(got.astype(np.float64) - r[k]).max())


@pytest.mark.parametrize("kind,order,radius", [("poly", 1, "opacity"), ("exp", 1, "sigma3"), ("poly", 3, "universal")])
@pytest.mark.parametrize("threads,wgs", [(256, 0), (64, 7), (128, 3000)])
def test_batched_equals_per_view(kind, order, radius, threads, wgs):
    sc, views = _small_batch()
    dev = [render.to_device(s) for s in sc]
    print(f"[gpu] batch {kind}{order}/{radius} threads={threads} wgs={wgs}", flush=True)
    ref = _per_view(dev, views, (kind, order, radius))
    br = batch.BatchRenderer(dev, views, H.gpu_kernel(kind, order, radius), H.gpu_params(blend_threads=threads))
    br.workgroups = wgs
    br.render_fit()
    torch.cuda.synchronize()
    _compare(br, ref)


def test_graph_replay_matches_eager():
    sc, views = _small_batch()
    dev = [render.to_device(s) for s in sc]
    br = batch.BatchRenderer(dev, views, H.gpu_kernel("poly", 1, "opacity"), H.gpu_params())
    br.render_fit()
    torch.cuda.synchronize()
    ref = [{k: v.cpu().numpy().copy() for k, v in br.view_outputs(i).items()} for i in range(len(views))]
    K = int(br.num_keys.item())
    br.capture()
    for rep in range(3):
        br.images.fill_(-1.0)           # eager work between replays
        br.final_T.zero_()
        torch.cuda.synchronize()
        br.replay()
        torch.cuda.synchronize()
        assert int(br.num_keys.item()) == K and int(br.overflow.item()) == 0
        _compare(br, ref)


def test_batch_overflow_reported():
    sc, views = _small_batch()
    dev = [render.to_device(s) for s in sc]
    br = batch.BatchRenderer(dev, views, H.gpu_kernel("poly", 1, "opacity"), H.gpu_params())
    br.capacity = 50
    br._layout()
    br.render()
    torch.cuda.synchronize()
    assert int(br.overflow.item()) == 1 and int(br.num_keys.item()) > 50


def test_device_view_table_differing_from_the_host_one():
    """The kernels read the view table from device memory. An entry there that
    differs from the validated host copy must never reach memory outside the
    batch's arrays: here view 2 (the empty scene on the host) names the
    4500-splat scene on the device, so the device layout runs out of pair
    slots at view 5 (the host sized them for its own table) and drops it (it
    renders nothing), while every other view renders its device entry."""
    import ctypes
    from paper_2603_18707_amd import _lib as L
    sc, views = _small_batch()
    dev = [render.to_device(s) for s in sc]
    kern = ("poly", 1, "opacity")
    br = batch.BatchRenderer(dev, views, H.gpu_kernel(*kern), H.gpu_params())
    br.capacity = 4 * br.render_fit() + 4096
    br._layout()
    table = (L.GsView * len(views))()
    ctypes.memmove(table, br.c_views, ctypes.sizeof(table))
    table[2].scene = 2
    raw = bytes(ctypes.string_at(ctypes.addressof(table), ctypes.sizeof(table)))
    br.views_dev.copy_(torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(br.device))
    for t in (br.images, br.final_T):
        t.fill_(-7.0)
    for t in (br.n_contrib, br.last_contrib):
        t.fill_(-7)
    br.render()
    torch.cuda.synchronize()
    assert int(br.overflow.item()) == 0
    rendered = [(i, (2, views[i][1]) if i == 2 else views[i]) for i in (0, 1, 2, 3, 4, 6)]
    ref = _per_view(dev, [v for _, v in rendered], kern)
    for (i, _), r in zip(rendered, ref):
        o = br.view_outputs(i)
        for k in r:
            assert np.array_equal(o[k].cpu().numpy(), r[k]), (i, k)
    o = br.view_outputs(5)  # dropped: untouched
    assert bool((o["image"] == -7.0).all()) and bool((o["final_T"] == -7.0).all())
    assert bool((o["n_contrib"] == -7).all()) and bool((o["last_contrib"] == -7).all())


def test_full_size_batched_workload_sampled_views():
    """6 scenes (100k..2M splats, SH3), 96 views at 640x360..1920x1080."""
    sc, views = scenes.workload_batched()
    dev = [render.to_device(s) for s in sc]
    br = batch.BatchRenderer(dev, views, H.gpu_kernel("poly", 1, "opacity"), H.gpu_params())
    K = br.render_fit()
    torch.cuda.synchronize()
    print(f"[gpu] full batch: pairs={br.pairs} K={K} grid={br.grid_w}x{br.grid_h}", flush=True)
    pick = [0, 17, 40, 63, 95]
    ref = _per_view(dev, [views[i] for i in pick], ("poly", 1, "opacity"))
    for j, i in enumerate(pick):
        o = br.view_outputs(i)
        for k in ref[j]:
            assert np.array_equal(o[k].cpu().numpy(), ref[j][k]), (i, k)


@pytest.mark.parametrize("kind,order,radius", [("poly", 1, "opacity"), ("exp", 1, "sigma3")])
def test_batched_equals_per_view_ellipse_box(kind, order, radius):
    """Ellipse-box tile rectangles in the batched path: bit-identical to the
    per-view frames in the same mode."""
    sc, views = _small_batch()
    dev = [render.to_device(s) for s in sc]
    print(f"[gpu] batch {kind}{order}/{radius} ellipse box", flush=True)
    ref = _per_view(dev, views, (kind, order, radius), {"rect_mode": 1})
    br = batch.BatchRenderer(dev, views, H.gpu_kernel(kind, order, radius), H.gpu_params(rect_mode=1))
    br.render_fit()
    torch.cuda.synchronize()
    _compare(br, ref)


# --- against the FP64 oracle ---------------------------------------------------

def _oracle_view(scene, cam, cfg, pixels, dev_scene, kind, order, radius, params_kw=None):
    """The oracle's projection and compositing of one view at `pixels`, with
    the records the GPU projection holds (gs_preprocess runs the batch's
    projection code; the certified choice between correct roundings is
    taken from it, see helpers.records_chosen_by)."""
    o = ocore.project(scene, cam, cfg)
    exempt = (o["flags"] & ocore.SPLAT_EDGE_NEAR) != 0
    assert not exempt.any()
    if scene.n:
        r = render.Rasterizer(H.gpu_kernel(kind, order, radius), H.gpu_params(**(params_kw or {})))
        g = r.preprocess(dev_scene, cam)
        torch.cuda.synchronize()
        assert np.array_equal(g["rect"].cpu().numpy(), o["rect"])
        rec, _ = H.records_chosen_by(o, g["means2d"].cpu().numpy(), g["conic_opacity"].cpu().numpy(),
                                     o["tiles"] > 0)
    else:
        rec = ocore.round_records(o)
    return o, ocore.render_pixels(rec, cfg, pixels)


@pytest.mark.parametrize("kind,order,radius,rect_mode", [("poly", 1, "opacity", 0), ("exp", 1, "sigma3", 0),
                                                         ("poly", 3, "universal", 1), ("exp", 1, "exp_opacity", 1)])
def test_small_batch_against_oracle(kind, order, radius, rect_mode):
    """Every pixel of every view of the ragged batch (an empty scene, partial
    tiles, 16x16 up to 301x157) against the oracle, and each view's key
    count against the oracle's tile count."""
    sc, views = _small_batch()
    dev = [render.to_device(s) for s in sc]
    print(f"[gpu] batch vs oracle {kind}{order}/{radius} rect {rect_mode}", flush=True)
    br = batch.BatchRenderer(dev, views, H.gpu_kernel(kind, order, radius), H.gpu_params(rect_mode=rect_mode))
    K = br.render_fit()
    torch.cuda.synchronize()
    vk = br.view_keys.cpu().numpy()
    assert int(vk.sum()) == K
    cfg = H.oracle_cfg(kind, order, radius, rect_mode=rect_mode)
    nflag_all = npix_all = 0
    for i, (si, cam) in enumerate(views):
        W, Hh = int(cam.width), int(cam.height)
        pix = ocore.all_pixels(W, Hh)
        o, ores = _oracle_view(sc[si], cam, cfg, pix, dev[si], kind, order, radius, {"rect_mode": rect_mode})
        assert int(vk[i]) == int(o["tiles"].sum()), (i, int(vk[i]), int(o["tiles"].sum()))
        gx, gy = (W + 15) // 16, (Hh + 15) // 16
        nflag, err = _check_pixels(br.view_outputs(i), ores, pix, H.edge_flagged_tiles(o, gx, gy))
        nflag_all, npix_all = nflag_all + nflag, npix_all + pix.shape[0]
    # counted over the batch: its 16x16 view of 2000 splats flags a few percent
    assert nflag_all <= H.flag_limit(kind, order, npix_all), nflag_all


def test_full_size_batched_workload_against_oracle():
    """The 96-view workload (6 scenes of 100k-2M splats): six views spread
    over every scene and resolution, 2048 sampled pixels each, and their key
    counts, against the oracle; the view key counts sum to K."""
    sc, views = scenes.workload_batched()
    dev = [render.to_device(s) for s in sc]
    br = batch.BatchRenderer(dev, views, H.gpu_kernel("poly", 1, "opacity"), H.gpu_params())
    K = br.render_fit()
    torch.cuda.synchronize()
    vk = br.view_keys.cpu().numpy()
    assert int(vk.sum()) == K
    cfg = H.oracle_cfg("poly", 1, "opacity")
    pick = [7, 17, 34, 48, 66, 83]  # one view of each scene, every resolution
    assert len({views[i][0] for i in pick}) == 6 and len({views[i][1].width for i in pick}) == 4
    for i in pick:
        si, cam = views[i]
        W, Hh = int(cam.width), int(cam.height)
        print(f"[gpu] batch view {i}: scene {si} ({sc[si].n} splats) {W}x{Hh}", flush=True)
        pix = scenes.sample_pixels(W, Hh, 2048, seed=60 + i)
        o, ores = _oracle_view(sc[si], cam, cfg, pix, dev[si], "poly", 1, "opacity")
        assert int(vk[i]) == int(o["tiles"].sum()), (i, int(vk[i]), int(o["tiles"].sum()))
        nflag, err = _check_pixels(br.view_outputs(i), ores, pix, H.edge_flagged_tiles(o, (W + 15) // 16,
                                                                                        (Hh + 15) // 16))
        assert nflag <= H.flag_limit("poly", 1, pix.shape[0]), (i, nflag)
        assert float(np.abs(ores["color"]).max()) > 0.1
