"""Batched multi-view renderer over gs_render_batched, with graph capture.

A ``BatchRenderer`` holds the scenes (device tensors), the views (host and
device copies of the gs_view table), the output buffers and the workspace.
``render()`` enqueues the whole batch (projection of every (scene, view) pair,
one shared binning and sort, one persistent blend); ``capture()`` records that
sequence once in a HIP graph (torch.cuda.CUDAGraph is HIP's graph API on
ROCm) and ``replay()`` re-runs it with no per-kernel launch cost. The key
capacity and the persistent grid size come from an eager run and the
autotuner; they must be fixed before capture.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L
from .render import DeviceScene


class BatchRenderer:
    def __init__(self, scenes, views, kernel: L.GsKernel, params: L.GsParams = None, device="cuda"):
        """scenes: list of DeviceScene; views: list of (scene index, camera)."""
        self.device = torch.device(device)
        self.kernel = kernel
        self.params = params if params is not None else L.gs_params_default()
        self.scenes = scenes
        self.c_scenes = (L.GsScene * len(scenes))()
        for i, s in enumerate(scenes):
            self.c_scenes[i].n = s.n
            self.c_scenes[i].means3d, self.c_scenes[i].scales = s.means3d.data_ptr(), s.scales.data_ptr()
            self.c_scenes[i].quats, self.c_scenes[i].opacities = s.quats.data_ptr(), s.opacities.data_ptr()
            self.c_scenes[i].sh, self.c_scenes[i].sh_degree, self.c_scenes[i].reserved = s.sh.data_ptr(), s.sh_degree, 0
        self.c_views = (L.GsView * len(views))()
        self.sizes = []
        img_off = pix_off = 0
        for i, (si, cam) in enumerate(views):
            v = self.c_views[i]
            v.cam = L.make_camera(cam)
            v.scene, v.reserved = int(si), 0
            v.image_offset, v.pixel_offset = img_off, pix_off
            W, H = int(cam.width), int(cam.height)
            self.sizes.append((W, H, img_off, pix_off))
            img_off += 3 * W * H
            pix_off += W * H
        raw = bytes(ctypes.string_at(ctypes.addressof(self.c_views), ctypes.sizeof(self.c_views)))
        self.views_dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(self.device)
        self.images = torch.zeros(img_off, dtype=torch.float32, device=self.device)
        self.final_T = torch.zeros(pix_off, dtype=torch.float32, device=self.device)
        self.n_contrib = torch.zeros(pix_off, dtype=torch.int32, device=self.device)
        self.last_contrib = torch.zeros(pix_off, dtype=torch.int32, device=self.device)
        self.num_keys = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.view_keys = torch.zeros(len(views), dtype=torch.int64, device=self.device)  # keys of each view
        self.capacity = 0
        self.workgroups = 0
        self.ws = None
        self.graph = None
        self._layout()

    def _layout(self):
        self.pairs, self.grid_w, self.grid_h, ws_bytes = L.gs_batch_layout(self.c_scenes, self.c_views, self.capacity)
        if self.ws is None or self.ws.numel() < ws_bytes:
            self.ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self.ws_bytes = ws_bytes

    def render(self, stream=None):
        L.gs_render_batched(self.kernel, self.params, self.c_scenes, self.c_views, self.views_dev, self.capacity,
                            self.workgroups, self.ws, self.ws_bytes, self.images, self.images.numel(), self.final_T,
                            self.n_contrib, self.last_contrib, self.final_T.numel(), self.num_keys, self.overflow,
                            stream, view_keys=self.view_keys)

    def render_fit(self):
        """Eager render that grows the key capacity until nothing overflows."""
        self.render()
        flag = int(self.overflow.item())
        if flag & 1:
            self.capacity = int(int(self.num_keys.item()) * 1.05) + 4096
            self._layout()
            self.render()
            flag = int(self.overflow.item())
        if flag:
            raise RuntimeError(f"gs_render_batched reported overflow flags {flag}")
        return int(self.num_keys.item())

    def capture(self):
        """Records one batch in a HIP graph (capacity, workgroups and buffers fixed)."""
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.render()  # warm the exact launch sequence once outside capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.render()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def view_outputs(self, i):
        W, H, io, po = self.sizes[i]
        return dict(image=self.images[io:io + 3 * W * H].view(3, H, W),
                    final_T=self.final_T[po:po + W * H].view(H, W),
                    n_contrib=self.n_contrib[po:po + W * H].view(H, W),
                    last_contrib=self.last_contrib[po:po + W * H].view(H, W))


def tune_batch(br: BatchRenderer, threads=(64, 128, 256), workgroups=(1024, 2048, 4096), stages=(1, 2),
               reps: int = 3) -> dict:
    """Times every (threads per tile, persistent workgroups, records staged
    per thread) triple on the batch (eager launches) and keeps the fastest;
    returns {(threads, wgs, stage): ms}."""
    stream = torch.cuda.current_stream()
    res = {}
    for nt in threads:
        for wg in workgroups:
            for sb in stages:
                br.params.blend_threads, br.workgroups, br.params.blend_stage = int(nt), int(wg), int(sb)
                br.render()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                for _ in range(reps):
                    br.render()
                b.record(stream)
                torch.cuda.synchronize()
                res[(int(nt), int(wg), int(sb))] = a.elapsed_time(b) / reps
    best = min(res, key=res.get)
    br.params.blend_threads, br.workgroups, br.params.blend_stage = best
    return res
