"""Launch-shape autotuner.

The blend's launch shape (threads per 16x16 tile: 64, 128 or 256, i.e. 4, 2 or
1 pixels per thread, each wave shading a 16x16, 8x16 or 8x8 block; and the LDS
batch, 1 or 2 records staged per thread) trades per-pixel arithmetic, LDS
traffic and barriers against the parallelism available to a tile with a long
splat list; the best choice depends on the splat-size distribution and
resolution. ``tune_blend`` times
every candidate on the frame at hand with HIP events and keeps the fastest;
results are cached per (device, resolution, kernel, splat-count bucket) in
memory and, when ``cache_path`` is given, in a JSON file. Outputs do not depend
on the choice (tests check that).
"""
import json
import math
import os

import torch

from . import _lib as L

BLEND_THREADS = (64, 128, 256)
BLEND_STAGES = (1, 2)  # records each thread stages per batch (the LDS batch is threads x stage)
_cache = {}


def _key(cam, kernel, n):
    dev = torch.cuda.get_device_name(torch.cuda.current_device()) if torch.cuda.is_available() else "cpu"
    return f"{dev}|{int(cam.width)}x{int(cam.height)}|k{kernel.kind}o{kernel.order}r{kernel.radius_mode}|n2^{int(math.log2(max(n, 1)))}"


def _load(cache_path):
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            _cache.update(json.load(f))


def _save(cache_path):
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(_cache, f, indent=1, sort_keys=True)


def tune_blend(r, proj, binned, cam, candidates=BLEND_THREADS, stages=BLEND_STAGES, reps: int = 5,
               cache_path: str = None) -> dict:
    """Times gs_rasterize_fwd for every candidate launch shape (threads per
    tile x records staged per thread); sets the winner on r.params
    (blend_threads, blend_stage) and returns {"threads x stage": ms}."""
    _load(cache_path)
    key = _key(cam, r.kernel, proj["n"])
    if key in _cache:
        r.params.blend_threads, r.params.blend_stage = (int(v) for v in _cache[key]["best"])
        return _cache[key]["ms"]
    stream = torch.cuda.current_stream()
    times = {}
    for nt in candidates:
        for sb in stages:
            r.params.blend_threads, r.params.blend_stage = int(nt), int(sb)
            r.rasterize(proj, binned, cam)  # warm
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                r.rasterize(proj, binned, cam)
            b.record(stream)
            torch.cuda.synchronize()
            times[(int(nt), int(sb))] = a.elapsed_time(b) / reps
    best = min(times, key=times.get)
    r.params.blend_threads, r.params.blend_stage = best
    _cache[key] = {"best": list(best), "ms": {f"{k[0]}x{k[1]}": v for k, v in times.items()}}
    _save(cache_path)
    return _cache[key]["ms"]
