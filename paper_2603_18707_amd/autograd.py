"""Differentiable rendering over the hand-written backward kernels.

``render(scene_tensors..., cam, kernel)`` returns the image [3, H, W]; its
backward runs gs_rasterize_bwd (per-pixel adjoint of blending, transmittance
recomputed back to front) then gs_preprocess_bwd (adjoint of the projection)
and returns gradients for means3d, scales, quats, opacities and sh. The
gradients of the 2D record (means2d, conic, opacity, rgb) are available from
``rasterize_backward``. Every step runs in libgs; torch only holds memory.
"""
import torch

from . import _lib as L
from .render import DeviceScene, Rasterizer


def rasterize_backward(r: Rasterizer, frame: dict, cam, dL_dimage: torch.Tensor) -> dict:
    """Gradients of the 2D record: means2d [n,2], conic_opacity [n,4], rgb [n,3]."""
    proj, b = frame["proj"], frame["binned"]
    n = proj["n"]
    dev = dL_dimage.device
    out = dict(means2d=torch.empty((n, 2), dtype=torch.float32, device=dev),
               conic_opacity=torch.empty((n, 4), dtype=torch.float32, device=dev),
               rgb=torch.empty((n, 3), dtype=torch.float32, device=dev))
    L.gs_rasterize_bwd(L.make_camera(cam), r.kernel, r.params, n, proj["means2d"], proj["conic_opacity"], proj["rgb"],
                       b["vals"], b["ranges"], b.get("tile_order"), frame["final_T"], frame["last_contrib"],
                       dL_dimage.contiguous(),
                       out["means2d"], out["conic_opacity"], out["rgb"])
    return out


def preprocess_backward(r: Rasterizer, scene: DeviceScene, frame: dict, cam, g2d: dict) -> dict:
    n = scene.n
    dev = scene.means3d.device
    out = dict(means3d=torch.empty((n, 3), dtype=torch.float32, device=dev),
               scales=torch.empty((n, 3), dtype=torch.float32, device=dev),
               quats=torch.empty((n, 4), dtype=torch.float32, device=dev),
               opacities=torch.empty((n,), dtype=torch.float32, device=dev),
               sh=torch.empty_like(scene.sh))
    L.gs_preprocess_bwd(L.make_camera(cam), r.kernel, r.params, n, scene.means3d, scene.scales, scene.quats,
                        scene.opacities, scene.sh, scene.sh_degree, frame["proj"]["tiles"], g2d["means2d"],
                        g2d["conic_opacity"], g2d["rgb"], out["means3d"], out["scales"], out["quats"],
                        out["opacities"], out["sh"])
    return out


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means3d, scales, quats, opacities, sh, sh_degree, cam, r, sync):
        scene = DeviceScene(means3d.detach().contiguous(), scales.detach().contiguous(), quats.detach().contiguous(),
                            opacities.detach().contiguous(), sh.detach().contiguous(), int(sh_degree))
        frame = r.render(scene, cam, sync=sync)
        ctx.scene, ctx.frame, ctx.cam, ctx.r = scene, frame, cam, r
        return frame["image"]

    @staticmethod
    def backward(ctx, dL_dimage):
        g2d = rasterize_backward(ctx.r, ctx.frame, ctx.cam, dL_dimage)
        g3d = preprocess_backward(ctx.r, ctx.scene, ctx.frame, ctx.cam, g2d)
        return g3d["means3d"], g3d["scales"], g3d["quats"], g3d["opacities"], g3d["sh"], None, None, None, None


def render(means3d, scales, quats, opacities, sh, sh_degree: int, cam, kernel: L.GsKernel,
           params: L.GsParams = None, rasterizer: Rasterizer = None, sync: bool = True) -> torch.Tensor:
    """Differentiable image [3, H, W] of the scene (activated parameters).
    Passing the same ``rasterizer`` (built with reuse_buffers=False) across
    steps keeps its fitted key capacity; with sync=False the forward enqueues
    without reading the overflow flag back (see Rasterizer.render), and the
    caller checks rasterizer.check_overflow() once it has synchronised."""
    r = rasterizer if rasterizer is not None else Rasterizer(kernel, params, device=means3d.device,
                                                             reuse_buffers=False)
    return _Render.apply(means3d, scales, quats, opacities, sh, sh_degree, cam, r, sync)
