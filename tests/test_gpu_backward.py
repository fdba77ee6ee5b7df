"""GPU backward against the reference gradient, through the C ABI.

The reference gradient is exact reverse-mode through the FP64 torch
re-implementation (``oracle.grad``), itself pinned to FP64 central finite
differences of the C oracle (tests/test_oracle_grad.py). Sub-problem: 64
splats, 32x32, SH degree 3 (and the same with 4x larger splats, where splats
overlap and the transmittance recursion matters). Loss: sum of random weights
times the image, so dL/dimage is the weight image.

Bar (FP32 kernels with float atomics against FP64): cosine similarity of every
parameter group above 0.9999, and per entry |g - g_ref| <= 2e-3 |g_ref| +
2e-5 max |g_ref| of the group.
"""
import numpy as np
import pytest
import torch

from oracle import core as ocore, grad as ograd
from paper_2603_18707_amd import autograd, render, scenes
from tests import helpers as H

pytestmark = pytest.mark.gpu

CASES = [("poly", 1, "opacity", 1.0), ("poly", 1, "opacity", 4.0), ("exp", 1, "sigma3", 4.0),
         ("poly", 2, "opacity", 4.0), ("poly", 3, "opacity", 4.0), ("poly", 1, "universal", 4.0)]


def _scene(scale_mul):
    scene, cam = scenes.workload_fd()
    scene.scales *= scale_mul
    return scene, cam


def _compare(name, g, ref):
    g, ref = np.asarray(g, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    mx = np.abs(ref).max()
    if mx == 0:
        assert np.abs(g).max() == 0, name
        return
    cos = g @ ref / (np.linalg.norm(g) * np.linalg.norm(ref))
    assert cos > 0.9999, (name, cos)
    bad = np.abs(g - ref) > 2e-3 * np.abs(ref) + 2e-5 * mx
    assert not bad.any(), (name, np.nonzero(bad)[0][:5], g[bad][:5], ref[bad][:5])


@pytest.mark.parametrize("kind,order,radius,scale_mul,cull", [c + (False,) for c in CASES] +
                         [("poly", 1, "opacity", 4.0, True), ("exp", 1, "sigma3", 4.0, True)])
def test_scene_gradients_match_reference(kind, order, radius, scale_mul, cull):
    """cull: the frame is binned with per-tile culling (gs_bin_sort_culled);
    the backward walks the culled lists and must give the same gradients."""
    scene, cam = _scene(scale_mul)
    cfg = H.oracle_cfg(kind, order, radius)
    # pixels holding a decision within single-precision reach of a threshold get zero weight,
    # so whichever way the GPU takes that decision the loss does not see it
    ref = ocore.render_image(scene, cam, cfg, round_to=None)
    assert (ref["flags"] != 0).sum() <= 2
    w = np.random.default_rng(31).normal(size=(3, cam.height, cam.width)) * (ref["flags"] == 0)

    leaves = {k: torch.tensor(np.asarray(getattr(scene, k), np.float64), requires_grad=True)
              for k in ("means3d", "scales", "quats", "opacities", "sh")}
    img, _ = ograd.render(leaves["means3d"], leaves["scales"], leaves["quats"], leaves["opacities"], leaves["sh"],
                          scene.sh_degree, cam, cfg)
    (img * torch.as_tensor(w)).sum().backward()

    print(f"[gpu] backward {kind}{order}/{radius} x{scale_mul}", flush=True)
    dev = {k: torch.tensor(np.asarray(getattr(scene, k), np.float32), device="cuda", requires_grad=True)
           for k in ("means3d", "scales", "quats", "opacities", "sh")}
    kern, params = H.gpu_kernel(kind, order, radius), H.gpu_params()
    rast = render.Rasterizer(kern, params, reuse_buffers=False, tile_cull=True) if cull else None
    gimg = autograd.render(dev["means3d"], dev["scales"], dev["quats"], dev["opacities"], dev["sh"], scene.sh_degree,
                           cam, kern, params, rasterizer=rast)
    assert np.abs(gimg.detach().cpu().numpy() - ref["image"]).max() < 2e-4
    (gimg * torch.as_tensor(w, dtype=torch.float32, device="cuda")).sum().backward()
    torch.cuda.synchronize()
    for k in leaves:
        _compare(k, dev[k].grad.cpu().numpy(), leaves[k].grad.numpy())


@pytest.mark.parametrize("kind,order,radius,scale_mul", CASES[:4])
def test_record_gradients_match_reference(kind, order, radius, scale_mul):
    """Gradients of the 2D record (means2d, conic a/b/c, opacity o', rgb) from gs_rasterize_bwd."""
    scene, cam = _scene(scale_mul)
    cfg = H.oracle_cfg(kind, order, radius)
    t64 = {k: torch.tensor(np.asarray(getattr(scene, k), np.float64)) for k in
           ("means3d", "scales", "quats", "opacities", "sh")}
    proj = ograd.project(t64["means3d"], t64["scales"], t64["quats"], t64["opacities"], t64["sh"], scene.sh_degree,
                         cam, cfg)
    leaf = {k: proj[k].detach().clone().requires_grad_(True) for k in ("u", "v", "a", "b", "c", "opac", "rgb")}
    p2 = dict(proj, **leaf)
    img, _ = ograd.render(None, None, None, None, None, scene.sh_degree, cam, cfg, proj=p2)
    ref = ocore.render_image(scene, cam, cfg, round_to=None)
    w = np.random.default_rng(32).normal(size=(3, cam.height, cam.width)) * (ref["flags"] == 0)
    (img * torch.as_tensor(w)).sum().backward()

    r = render.Rasterizer(H.gpu_kernel(kind, order, radius), H.gpu_params(), reuse_buffers=False)
    frame = r.render(render.to_device(scene), cam)
    g2d = autograd.rasterize_backward(r, frame, cam, torch.as_tensor(w, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    gm = g2d["means2d"].cpu().numpy()
    gc = g2d["conic_opacity"].cpu().numpy()
    _compare("u", gm[:, 0], leaf["u"].grad.numpy())
    _compare("v", gm[:, 1], leaf["v"].grad.numpy())
    _compare("a", gc[:, 0], leaf["a"].grad.numpy())
    _compare("b", gc[:, 1], leaf["b"].grad.numpy())
    _compare("c", gc[:, 2], leaf["c"].grad.numpy())
    _compare("opacity", gc[:, 3], leaf["opac"].grad.numpy())
    _compare("rgb", g2d["rgb"].cpu().numpy(), leaf["rgb"].grad.numpy())


def test_backward_with_background_and_termination():
    """Dense opaque splats so pixels terminate early, with a non-zero background."""
    scene, cam = _scene(6.0)
    scene.opacities[:] = np.float32(0.97)
    bg = (0.3, 0.1, 0.7)
    cfg = H.oracle_cfg("poly", 1, "opacity", bg=bg)
    ref = ocore.render_image(scene, cam, cfg, round_to=None)
    leaves = {k: torch.tensor(np.asarray(getattr(scene, k), np.float64), requires_grad=True)
              for k in ("means3d", "scales", "quats", "opacities", "sh")}
    img, _ = ograd.render(*[leaves[k] for k in ("means3d", "scales", "quats", "opacities", "sh")], scene.sh_degree,
                          cam, cfg)
    w = np.random.default_rng(33).normal(size=(3, cam.height, cam.width)) * (ref["flags"] == 0)
    (img * torch.as_tensor(w)).sum().backward()
    dev = {k: torch.tensor(np.asarray(getattr(scene, k), np.float32), device="cuda", requires_grad=True)
           for k in ("means3d", "scales", "quats", "opacities", "sh")}
    gimg = autograd.render(*[dev[k] for k in ("means3d", "scales", "quats", "opacities", "sh")], scene.sh_degree,
                           cam, H.gpu_kernel("poly", 1, "opacity"), H.gpu_params(bg=bg))
    (gimg * torch.as_tensor(w, dtype=torch.float32, device="cuda")).sum().backward()
    torch.cuda.synchronize()
    assert (ref["T"] < 1.5e-4).sum() > 50  # many pixels end near t_min
    for k in leaves:
        _compare(k, dev[k].grad.cpu().numpy(), leaves[k].grad.numpy())


# --- long lists: the adjoint's walk over many 64-record stages ---------------

def _multistage_scene(opacity_logit_mean, n=1500, size=64, seed=77):
    """1,500 tiny-generator splats (SH degree 3) with doubled scales on a
    64x64 camera: the central tiles' lists hold 500-800 copies, so blend_bwd
    walks 8-13 stages of 64 records back to front. Opacity logits
    N(mean, 1): at mean -4 no pixel terminates and the transmittance and the
    colour behind are carried across every stage; at mean -1 several hundred
    pixels stop at list positions beyond the first stage."""
    scene = scenes.tiny_scene(n, seed=seed, sh_degree=3)
    scene.scales *= 2.0
    logit = np.random.default_rng(seed).normal(opacity_logit_mean, 1.0, n)
    scene.opacities[:] = (1.0 / (1.0 + np.exp(-logit))).astype(np.float32)
    return scene, scenes.tiny_camera(size, size)


def _list_lengths(proj, size, tile=16):
    """Unculled copies per tile, from the oracle's rectangles."""
    g = size // tile
    L = np.zeros((g, g), np.int64)
    for x0, y0, x1, y1 in proj["rect"]:
        if x1 >= x0 and y1 >= y0:
            L[y0:y1 + 1, x0:x1 + 1] += 1
    return np.kron(L, np.ones((tile, tile), np.int64))  # per pixel


MULTISTAGE = [("poly", 1, "opacity", -4.0, False), ("poly", 1, "opacity", -4.0, True),
              ("exp", 1, "sigma3", -4.0, False), ("exp", 1, "sigma3", -4.0, True),
              ("poly", 1, "opacity", -1.0, False), ("exp", 1, "sigma3", -1.0, False),
              ("poly", 1, "opacity", -1.0, True), ("poly", 2, "opacity", -1.0, False),
              ("poly", 3, "opacity", -1.0, False)]


@pytest.mark.parametrize("kind,order,radius,logit_mean,cull", MULTISTAGE)
def test_multistage_gradients_match_reference(kind, order, radius, logit_mean, cull):
    """Scene-parameter gradients through tiles whose lists span many 64-record
    stages, against the FP64 reverse-mode reference, at the bar above."""
    scene, cam = _multistage_scene(logit_mean)
    cfg = H.oracle_cfg(kind, order, radius)
    ref = ocore.render_image(scene, cam, cfg, round_to=None)
    L = _list_lengths(ref["proj"], cam.width)
    # the walk really crosses stage boundaries, with contributions on both sides
    assert L.max() >= 500 and (ref["last_contrib"] > 3 * 64).sum() >= 500, (L.max(), ref["last_contrib"].max())
    stopped = ref["n_eval"] < L
    if logit_mean > -2.0:
        assert (stopped & (ref["n_eval"] > 64)).sum() >= 150, int((stopped & (ref["n_eval"] > 64)).sum())
    else:
        assert not stopped.any()
    w = np.random.default_rng(34).normal(size=(3, cam.height, cam.width)) * (ref["flags"] == 0)

    leaves = {k: torch.tensor(np.asarray(getattr(scene, k), np.float64), requires_grad=True)
              for k in ("means3d", "scales", "quats", "opacities", "sh")}
    img, _ = ograd.render(*[leaves[k] for k in ("means3d", "scales", "quats", "opacities", "sh")], scene.sh_degree,
                          cam, cfg)
    (img * torch.as_tensor(w)).sum().backward()

    print(f"[gpu] multi-stage backward {kind}{order}/{radius} logit {logit_mean} cull {cull}", flush=True)
    dev = {k: torch.tensor(np.asarray(getattr(scene, k), np.float32), device="cuda", requires_grad=True)
           for k in ("means3d", "scales", "quats", "opacities", "sh")}
    kern, params = H.gpu_kernel(kind, order, radius), H.gpu_params()
    rast = render.Rasterizer(kern, params, reuse_buffers=False, tile_cull=cull)
    gimg = autograd.render(*[dev[k] for k in ("means3d", "scales", "quats", "opacities", "sh")], scene.sh_degree,
                           cam, kern, params, rasterizer=rast)
    good = ref["flags"] == 0
    assert np.abs(gimg.detach().cpu().numpy() - ref["image"]).max(axis=0)[good].max() < 2e-4
    (gimg * torch.as_tensor(w, dtype=torch.float32, device="cuda")).sum().backward()
    torch.cuda.synchronize()
    for k in leaves:
        _compare(k, dev[k].grad.cpu().numpy(), leaves[k].grad.numpy())


@pytest.mark.parametrize("kind,order,radius,logit_mean", [("poly", 1, "opacity", -4.0), ("exp", 1, "sigma3", -4.0),
                                                          ("poly", 1, "opacity", -1.0), ("exp", 1, "sigma3", -1.0)])
def test_multistage_record_gradients_match_reference(kind, order, radius, logit_mean):
    """gs_rasterize_bwd's 2D record gradients on the long lists."""
    scene, cam = _multistage_scene(logit_mean)
    cfg = H.oracle_cfg(kind, order, radius)
    t64 = {k: torch.tensor(np.asarray(getattr(scene, k), np.float64)) for k in
           ("means3d", "scales", "quats", "opacities", "sh")}
    proj = ograd.project(t64["means3d"], t64["scales"], t64["quats"], t64["opacities"], t64["sh"], scene.sh_degree,
                         cam, cfg)
    leaf = {k: proj[k].detach().clone().requires_grad_(True) for k in ("u", "v", "a", "b", "c", "opac", "rgb")}
    img, _ = ograd.render(None, None, None, None, None, scene.sh_degree, cam, cfg, proj=dict(proj, **leaf))
    ref = ocore.render_image(scene, cam, cfg, round_to=None)
    w = np.random.default_rng(35).normal(size=(3, cam.height, cam.width)) * (ref["flags"] == 0)
    (img * torch.as_tensor(w)).sum().backward()

    print(f"[gpu] multi-stage record backward {kind}{order}/{radius} logit {logit_mean}", flush=True)
    r = render.Rasterizer(H.gpu_kernel(kind, order, radius), H.gpu_params(), reuse_buffers=False)
    frame = r.render(render.to_device(scene), cam)
    g2d = autograd.rasterize_backward(r, frame, cam, torch.as_tensor(w, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    gm, gc = g2d["means2d"].cpu().numpy(), g2d["conic_opacity"].cpu().numpy()
    for name, g, k in (("u", gm[:, 0], "u"), ("v", gm[:, 1], "v"), ("a", gc[:, 0], "a"), ("b", gc[:, 1], "b"),
                       ("c", gc[:, 2], "c"), ("opacity", gc[:, 3], "opac")):
        _compare(name, g, leaf[k].grad.numpy())
    _compare("rgb", g2d["rgb"].cpu().numpy(), leaf["rgb"].grad.numpy())


def test_sync_free_frames_match_and_report_overflow():
    """Rasterizer.render(sync=False) (and autograd.render(sync=False)) bins
    with the fitted key capacity without reading the overflow flag back: the
    image and the gradients equal those of a fitted frame bit for bit, and a
    frame whose keys do not fit raises at check_overflow()."""
    scene, cam = _scene(4.0)
    kern, params = H.gpu_kernel("poly", 1, "opacity"), H.gpu_params()
    dev = {k: torch.tensor(np.asarray(getattr(scene, k), np.float32), device="cuda", requires_grad=True)
           for k in ("means3d", "scales", "quats", "opacities", "sh")}
    w = torch.as_tensor(np.random.default_rng(34).normal(size=(3, cam.height, cam.width)), dtype=torch.float32,
                        device="cuda")
    r = render.Rasterizer(kern, params, reuse_buffers=False)
    grads, imgs = [], []
    for sync in (True, False):
        for t in dev.values():
            t.grad = None
        img = autograd.render(*[dev[k] for k in ("means3d", "scales", "quats", "opacities", "sh")],
                              scene.sh_degree, cam, kern, params, rasterizer=r, sync=sync)
        (img * w).sum().backward()
        torch.cuda.synchronize()
        imgs.append(img.detach().cpu().numpy())
        grads.append({k: t.grad.cpu().numpy() for k, t in dev.items()})
    assert r.check_overflow() == 0
    assert np.array_equal(imgs[0], imgs[1])
    # float atomics add the partial gradients in any order: equal up to rounding
    for k in dev:
        np.testing.assert_allclose(grads[1][k], grads[0][k], rtol=1e-5, atol=1e-6 * np.abs(grads[0][k]).max())
    r.capacity = 16  # far fewer than the frame's keys
    r.render(render.to_device(scene), cam, sync=False)
    torch.cuda.synchronize()
    with pytest.raises(RuntimeError, match="overflowed"):
        r.check_overflow()
    assert r.check_overflow() == 0  # cleared by the check
