"""Frame-level driver over the C ABI: buffers, key capacity and the three stages.

PyTorch supplies device memory and the stream; every stage is one of libgs's
HIP entry points (gs_preprocess -> gs_bin_sort, or gs_bin_sort_culled with
per-tile culling -> gs_rasterize_fwd).
"""
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

TILE = 16
# tile_cull="auto" bins with per-tile culling when the splats' rectangles hold
# at least this many tiles per visible splat: culling costs a per-splat FP64
# set-up and pays back in proportion to the rectangle tiles it drops
# (measured: 1.6 tiles per splat, 11% slower frames; 13 and more, 2-4x faster)
AUTO_CULL_TILES_PER_SPLAT = 4.0


@dataclass
class DeviceScene:
    means3d: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    opacities: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means3d.shape[0])


def to_device(scene, device="cuda") -> DeviceScene:
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(device)
    return DeviceScene(f(scene.means3d), f(scene.scales), f(scene.quats), f(scene.opacities), f(scene.sh),
                       int(scene.sh_degree))


def kernel_spec(kind: str, order: int = 1, radius: str = "opacity", coeffs=None) -> L.GsKernel:
    """kind 'exp' or 'poly'; radius 'sigma3', 'universal', 'opacity' (polynomial
    root at eps / o') or 'exp_opacity' (exp's own opacity bound)."""
    k = {"exp": L.KERNEL_EXP, "poly": L.KERNEL_POLY}[kind]
    r = {"sigma3": L.RADIUS_SIGMA3, "universal": L.RADIUS_POLY_UNIVERSAL, "opacity": L.RADIUS_POLY_OPACITY,
         "exp_opacity": L.RADIUS_EXP_OPACITY}[radius]
    return L.make_kernel(k, order, r, coeffs)


def grid_of(cam):
    return (int(cam.width) + TILE - 1) // TILE, (int(cam.height) + TILE - 1) // TILE


class Rasterizer:
    """Renders frames of one kernel configuration; keeps its buffers and the
    key capacity between frames (the capacity grows when a frame overflows)."""

    def __init__(self, kernel: L.GsKernel, params: L.GsParams = None, device="cuda", capacity: int = 0,
                 reuse_buffers: bool = True, tile_cull=False, mfma: bool = False):
        self.kernel = kernel
        # True: blend with gs_rasterize_fwd_mfma (the quadric on the matrix
        # cores); needs lists from gs_bin_sort, so it excludes tile culling
        if mfma and tile_cull:
            raise ValueError("the matrix-core blend takes lists binned without per-tile culling")
        self.mfma = bool(mfma)
        # True: bin with gs_bin_sort_culled (copies only for reachable tiles); "auto": decided in
        # bin_sort_fit from the frame's rectangle tiles per visible splat
        if isinstance(tile_cull, str) and tile_cull != "auto":
            raise ValueError(f"tile_cull must be True, False or 'auto', not {tile_cull!r}")
        self.tile_cull = tile_cull if tile_cull == "auto" else bool(tile_cull)
        self.culling = self.tile_cull is True  # the choice bin_sort follows
        self.params = params if params is not None else L.gs_params_default()
        self.device = torch.device(device)
        self.capacity = int(capacity)
        self.reuse = reuse_buffers  # False: every frame gets fresh outputs (autograd keeps them)
        self._bufs = {}
        self._overflow_acc = None  # overflow flags of the frames binned without a readback (render(sync=False))

    # -- buffers ---------------------------------------------------------
    def _buf(self, name, shape, dtype):
        t = self._bufs.get(name)
        numel = int(np.prod(shape))
        if not self.reuse and name != "ws":
            t = None
        if t is None or t.numel() < numel or t.dtype != dtype:
            t = torch.empty(max(numel, 1), dtype=dtype, device=self.device)
            self._bufs[name] = t
        return t[:numel].view(*shape) if len(shape) else t[:1]

    # -- stages ----------------------------------------------------------
    def preprocess(self, scene: DeviceScene, cam, stream=None) -> dict:
        n = scene.n
        out = dict(means2d=self._buf("means2d", (n, 2), torch.float32),
                   conic_opacity=self._buf("conic_opacity", (n, 4), torch.float32),
                   rgb=self._buf("rgb", (n, 3), torch.float32),
                   depth=self._buf("depth", (n,), torch.float32),
                   rect=self._buf("rect", (n, 4), torch.int32),
                   tiles=self._buf("tiles", (n,), torch.int32))
        L.gs_preprocess(L.make_camera(cam), self.kernel, self.params, n, scene.means3d, scene.scales, scene.quats,
                        scene.opacities, scene.sh, scene.sh_degree, out["means2d"], out["conic_opacity"],
                        out["rgb"], out["depth"], out["rect"], out["tiles"], stream)
        out["n"] = n
        return out

    def bin_sort(self, proj: dict, cam, capacity: int = None, stream=None) -> dict:
        n = proj["n"]
        gw, gh = grid_of(cam)
        cap = self.capacity if capacity is None else int(capacity)
        ws_bytes = L.gs_bin_sort_workspace(n, cap, gw * gh)
        ws = self._buf("ws", ((ws_bytes + 255) // 256 * 256,), torch.uint8)
        out = dict(keys=self._buf("keys", (max(cap, 1),), torch.int64),
                   vals=self._buf("vals", (max(cap, 1),), torch.int32),
                   ranges=self._buf("ranges", (gw * gh, 2), torch.int32),
                   tile_order=self._buf("tile_order", (gw * gh,), torch.int32),
                   num_keys=self._buf("num_keys", (1,), torch.int64),
                   overflow=self._buf("overflow", (1,), torch.int32))
        if self.culling:
            L.gs_bin_sort_culled(self.kernel, self.params, n, proj["depth"], proj["rect"], proj["tiles"],
                                 proj["means2d"], proj["conic_opacity"], gw, gh, cap, ws, ws.numel(), out["keys"],
                                 out["vals"], out["ranges"], out["tile_order"], out["num_keys"], out["overflow"], stream)
        else:
            L.gs_bin_sort(n, proj["depth"], proj["rect"], proj["tiles"], gw, gh, cap, ws, ws.numel(), out["keys"],
                          out["vals"], out["ranges"], out["tile_order"], out["num_keys"], out["overflow"], stream)
        out["capacity"] = cap
        return out

    def bin_sort_fit(self, proj: dict, cam, stream=None) -> dict:
        """bin_sort, growing the capacity and retrying when the keys overflow
        (reads device scalars back: use outside timed or captured regions).
        With tile_cull="auto" it also decides whether to cull, for this frame
        and the bin_sort calls that follow."""
        if self.tile_cull == "auto":
            tiles = proj["tiles"][: proj["n"]]
            visible = int((tiles > 0).sum().item())
            copies = int(tiles.to(torch.int64).sum().item())
            self.culling = visible > 0 and copies >= AUTO_CULL_TILES_PER_SPLAT * visible
        b = self.bin_sort(proj, cam, stream=stream)
        flag = int(b["overflow"].item())
        if flag & 1:
            K = int(b["num_keys"].item())
            self.capacity = int(K * 1.125) + 1024
            b = self.bin_sort(proj, cam, stream=stream)
            flag = int(b["overflow"].item())
        if flag:
            raise RuntimeError(f"gs_bin_sort reported overflow flags {flag}")
        return b

    def rasterize(self, proj: dict, binned: dict, cam, want_eval: bool = False, stream=None,
                  want_tested: bool = False) -> dict:
        """gs_rasterize_fwd (gs_rasterize_fwd_mfma for a matrix-core
        rasterizer); with want_tested, the vector blend's counting build
        gs_rasterize_fwd_count (adds n_tested, the evaluations performed)."""
        W, H = int(cam.width), int(cam.height)
        out = dict(image=self._buf("image", (3, H, W), torch.float32),
                   final_T=self._buf("final_T", (H, W), torch.float32),
                   n_contrib=self._buf("n_contrib", (H, W), torch.int32),
                   last_contrib=self._buf("last_contrib", (H, W), torch.int32),
                   n_eval=self._buf("n_eval", (H, W), torch.int32) if want_eval else None)
        args = (L.make_camera(cam), self.kernel, self.params, proj["n"], proj["means2d"], proj["conic_opacity"],
                proj["rgb"], binned["vals"], binned["ranges"], binned.get("tile_order"), out["image"],
                out["final_T"], out["n_contrib"], out["last_contrib"], out["n_eval"])
        if want_tested:
            out["n_tested"] = self._buf("n_tested", (H, W), torch.int32)
            L.gs_rasterize_fwd_count(*args, out["n_tested"], stream)
        elif self.mfma:
            L.gs_rasterize_fwd_mfma(*args, stream)
        else:
            L.gs_rasterize_fwd(*args, stream)
        return out

    def render(self, scene: DeviceScene, cam, want_eval: bool = False, stream=None, sync: bool = True) -> dict:
        """One frame. sync=False bins with the current key capacity (fitted by an
        earlier frame) without reading the overflow flag back, so the frame
        enqueues with no host round trip; the flag is OR-ed into a device
        accumulator that check_overflow() reads (a frame that overflowed has
        no keys and must be redone with a larger capacity)."""
        proj = self.preprocess(scene, cam, stream)
        if sync:
            binned = self.bin_sort_fit(proj, cam, stream)
        else:
            binned = self.bin_sort(proj, cam, stream=stream)
            if self._overflow_acc is None:
                self._overflow_acc = torch.zeros(1, dtype=torch.int32, device=self.device)
            self._overflow_acc.bitwise_or_(binned["overflow"])
        img = self.rasterize(proj, binned, cam, want_eval, stream)
        return dict(proj=proj, binned=binned, **img)

    def check_overflow(self) -> int:
        """Reads (and clears) the overflow flags of the frames rendered with
        sync=False since the last check; raises when any frame overflowed."""
        if self._overflow_acc is None:
            return 0
        flag = int(self._overflow_acc.item())
        self._overflow_acc.zero_()
        if flag:
            raise RuntimeError(f"a frame rendered with sync=False overflowed (flags {flag}); "
                               f"render it again with sync=True to fit the key capacity")
        return flag
