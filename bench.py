"""Throughput of the polynomial-kernel splatting path on one MI355X.

Workload: 1,000,000 splats (64 anisotropic clusters in a 20-unit box, log-scales
N(-4.5, 1), opacity logits N(0, 2), SH degree 3), one 1920x1080 camera at
distance 30 with a 60 degree field of view. A step is one full frame:
gs_preprocess -> gs_bin_sort -> gs_rasterize_fwd, inputs resident in HBM.

Headline: poly order 1 with the opacity-dependent radius (Eq. 4); the same
frame with the exponential kernel and 3-sigma culling is timed on the same GPU
for comparison. `value` is whole-job throughput: K frames launched back to
back with only a synchronised event pair around them; the medians of frames
timed with events between the stages are reported beside it. The same JSON
line carries the kernel x culling sweep of the frame (the analogue of the
paper's Table 3 and Table 4), the heavy-tailed 4M-splat scene over 8 orbit
poses, the batched multi-view frame and a training step, each with per-stage
times, and the FP64 oracle timed on the host cores.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
       python bench.py --only poly2/opacity[/culled]   (one frame configuration, for profiling)
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s and splat-pixel evals/s, poly-1 vs exp kernel, 1M splats 1080p, err≤2e-4"

# Algorithmic VALU lane-operations of the blend per evaluated (pixel, splat)
# pair, one op per add, multiply, FMA, min/max, compare or exponential: 14
# shared (dx, dy: 2; the quadric with FMAs: 5; the eps test: 1; T': 1; the
# t_min test: 1; w = alpha T: 1; the colour: 3) plus the kernel's own (poly-1:
# the clamp, o' c_1 folded into the quadric: 1; exp: the exponent's add, the
# exponential and the clamp: 3; poly-2: two Horner steps and the cut: 3;
# poly-3: three Horner steps: 3). The headline roofline uses this count with
# every evaluated pair charged the blend; the exponential, a quarter-rate
# transcendental, costs 3 issue slots more (TRANS_SLOTS).
OPS_8D = {"poly1": 15, "exp": 17, "poly2": 17, "poly3": 17}
TRANS_SLOTS = {"exp": 3}
# A refined count charges the blend only to blended pairs: per evaluated pair
# dx, dy (2), the quadric (5), the kernel (poly-1: 1 FMA; exp: add + exp = 2;
# poly-2: 3; poly-3: 4), the clamp (1) and the eps test (1); per blended pair
# 1 - alpha and T' (2), the t_min test (1), alpha T (1), colour FMAs (3).
# Evaluated pairs are those the kernel performs (gs_rasterize_fwd_count's
# n_tested: list entries a wave does not skip by its box test, up to each
# pixel's termination); the per-pixel list entries without the box test are
# reported beside them as list_entries.
OPS_EVAL = {"poly1": 10, "exp": 11, "poly2": 12, "poly3": 13}
OPS_BLEND = 7
# MI355X vector ALU issue peak without packed FP32: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz = 39.3e12 lane-ops/s (the 157.3 TFLOP/s FP32 figure counts
# packed FMA as 4 flops; the library is compiled with packed FP32 disabled).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK = 8e12  # bytes/s


def tile_passes(ntiles):
    """Stable tile-digit passes of the binning (8 bits or fewer each)."""
    bits = max(1, int(ntiles - 1).bit_length())
    return (bits + 7) // 8


def stage_bytes(n, sh_degree, K, ntiles, npix):
    """Algorithmic HBM bytes per frame stage.
    preprocess: per splat the inputs (means 12, scales 12, quats 16, opacity
      4, SH 12 per coefficient) and the record (means2d 8, conic+opacity 16,
      rgb 12, depth 4, rect 16, tiles 4);
    bin_sort: per splat depth, rect and tiles read (24); per copy the emitted
      key parts (12), each tile pass reading and writing them (24), the ranges
      pass (4) and the per-tile depth sort (8 read, 12 written);
    blend: per copy the splat index and its record (4 + 36), per pixel the
      outputs (image 12, T 4, n_contrib 4, last_contrib 4)."""
    pre = n * (44 + 12 * (sh_degree + 1) ** 2 + 60)
    srt = 24 * n + K * (12 + 24 * tile_passes(ntiles) + 4 + 20)
    bl = K * 40 + npix * 24
    return {"preprocess": pre, "bin_sort": srt, "blend": bl}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--only", default=None, metavar="KERNEL/RADIUS[/culled|/mfma]",
                    help="time one frame configuration, e.g. poly2/opacity, exp/sigma3/culled or poly1/opacity/mfma "
                         "(the matrix-core blend) (for profiling); "
                         "kernels exp|poly1|poly2|poly3, radii sigma3|universal|opacity|exp_opacity")
    ap.add_argument("--no-sweep", action="store_true", help="skip the kernel x culling sweep")
    ap.add_argument("--blend-threads", type=int, default=0, help="64|128|256; 0 = autotune")
    ap.add_argument("--rect", default="box", choices=("box", "square"),
                    help="tile rectangles of the headline frames: the ellipse's bounding box or the bounding square")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched multi-view measurement")
    ap.add_argument("--no-train", action="store_true", help="skip the forward+backward step measurement")
    ap.add_argument("--no-heavy", action="store_true", help="skip the 4M-splat heavy-tailed scene")
    ap.add_argument("--heavy-only", default=None, metavar="ROW",
                    help="time only the heavy-tailed scene, all rows ('all') or one row such as "
                         "'4k_tile_culled' (for profiling; prints its own JSON object)")
    ap.add_argument("--train-only", action="store_true", help="time only the training step (for profiling)")
    ap.add_argument("--batched-only", action="store_true", help="time only the batched frame (for profiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 256 MiB device-to-device copy (calibrates HBM byte counters)")
    return ap.parse_args()


BLEND_SOURCES = ("rasterize.hip", "blend_common.h")


def kernel_source_hash():
    """Hash of the sources that define the forward blend kernel; the committed
    HBM counter summary is used only while it matches."""
    h = hashlib.sha1()
    for name in BLEND_SOURCES:
        with open(os.path.join(ROOT, "paper_2603_18707_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


RECT_MODES = {"square": 0, "box": 1}
RECT_NAMES = {"square": "bounding-square tile rectangles", "box": "ellipse-box tile rectangles"}


def time_config(torch, render, scene, cam, kind, order, radius, steps, warmup, threads=0, rect="box", cull=False,
                count=True, mfma=False):
    """Times `steps` frames with HIP events on the launch stream around each
    frame and each stage; frame and stage times are medians over the frames
    (the mean of the whole loop is kept beside them). threads = 0 lets the
    autotuner pick the blend launch shape during warm-up; cull bins with
    per-tile culling (gs_bin_sort_culled); count adds an untimed frame of the
    counting blend (evaluations performed); mfma blends with the matrix-core
    blend (gs_rasterize_fwd_mfma; the counting frame stays the vector one's)."""
    from paper_2603_18707_amd import autotune
    r = render.Rasterizer(render.kernel_spec(kind, order, radius), tile_cull=cull)
    r.params.rect_mode = RECT_MODES[rect]
    stream = torch.cuda.current_stream()
    # warm-up frames also size the key capacity (host readback happens here only)
    for _ in range(max(warmup, 1)):
        out = r.render(scene, cam)
    torch.cuda.synchronize()
    K = int(out["binned"]["num_keys"].item())
    r.capacity = int(K * 1.05) + 4096
    b0 = r.bin_sort(out["proj"], cam)  # re-size buffers for the final capacity outside the timed loop
    torch.cuda.synchronize()
    tuned = None
    if threads or mfma:
        r.params.blend_threads = threads or 256
    else:
        tuned = autotune.tune_blend(r, out["proj"], b0, cam)
    r.mfma = mfma
    torch.cuda.synchronize()

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for s in range(steps):
        e = ev[s]
        e[0].record(stream)
        proj = r.preprocess(scene, cam)
        e[1].record(stream)
        b = r.bin_sort(proj, cam)
        e[2].record(stream)
        r.rasterize(proj, b, cam)
        e[3].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    assert int(b["overflow"].item()) == 0
    total_ms = start.elapsed_time(stop)
    st = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3])] for e in ev])
    frame = np.array([e[0].elapsed_time(e[3]) for e in ev])
    # the same frames back to back with no event between them: whole-job
    # throughput (an event recorded between stages costs the stream a few us)
    start.record(stream)
    for s in range(steps):
        proj = r.preprocess(scene, cam)
        b = r.bin_sort(proj, cam)
        r.rasterize(proj, b, cam)
    stop.record(stream)
    torch.cuda.synchronize()
    clean_ms = start.elapsed_time(stop) / steps
    res = dict(ms=float(np.median(frame)), ms_mean=total_ms / steps, ms_min=float(frame.min()),
               ms_max=float(frame.max()), ms_clean=clean_ms, stage_ms=np.median(st, axis=0).tolist(),
               blend_ms=float(np.median(st[:, 2])),
               K=int(b["num_keys"].item()), E=None, E_list=None, B=None, image=None, rast=r,
               threads=int(r.params.blend_threads), stage=int(r.params.blend_stage), tuned=tuned)
    if count:
        r.mfma = False
        # untimed frame of the counting build: E = kernel evaluations performed,
        # E_list = list entries a per-pixel walk without the box test would evaluate
        full = r.rasterize(proj, b, cam, want_eval=True, want_tested=True)
        torch.cuda.synchronize()
        res.update(E=int(full["n_tested"].sum().item()), E_list=int(full["n_eval"].sum().item()),
                   B=int(full["n_contrib"].sum().item()), image=full["image"].clone())
    return res


def summary(t, W, H):
    """JSON row of a timed frame configuration."""
    ms = t["ms"]
    row = {"ms_per_step": round(ms, 4), "ms_mean": round(t["ms_mean"], 4), "ms_back_to_back": round(t["ms_clean"], 4),
           "Mpix_per_s": round(W * H / (ms * 1e-3) / 1e6, 2), "keys": t["K"],
           "stage_ms": {"preprocess": round(t["stage_ms"][0], 4), "bin_sort": round(t["stage_ms"][1], 4),
                        "blend": round(t["stage_ms"][2], 4)},
           "blend_threads": t["threads"], "blend_stage": t["stage"]}
    if t["E"] is not None:
        row.update(evals=t["E"], list_entries=t["E_list"], blended=t["B"],
                   splat_pixel_evals_per_s=round(t["E"] / (ms * 1e-3), 1))
    return row


SWEEP_KERNELS = (("exp", "exp", 1), ("poly1", "poly", 1), ("poly2", "poly", 2), ("poly3", "poly", 3))
SWEEP_RADII = ("sigma3", "universal", "opacity", "exp_opacity")
# The paper's ablation (Table 3) in this build's terms: S = StopThePop's
# unaltered culling, whose bound is exp's opacity-aware extent (exp_opacity
# rectangles); 0 = the polynomial's root (universal radius); 1 = the
# polynomial's opacity-aware radius at 1/255.
TABLE3 = (("g/S", "exp/exp_opacity"), ("f1/S", "poly1/exp_opacity"), ("f1/0", "poly1/universal"),
          ("f1/1", "poly1/opacity"), ("f'2/S", "poly2/exp_opacity"), ("f'2/1", "poly2/opacity"),
          ("f3/S", "poly3/exp_opacity"), ("f3/1", "poly3/opacity"))


def time_sweep(torch, render, scene, cam, steps, warmup, rect, done):
    """Every kernel x radius combination of the 1M-splat frame, binned plainly
    and with per-tile culling; `done` holds rows already timed, keyed
    (kernel/radius, culled)."""
    W, H = cam.width, cam.height
    out = {"rect": RECT_NAMES[rect]}
    for cull in (False, True):
        sec = {}
        for kname, kind, order in SWEEP_KERNELS:
            for radius in SWEEP_RADII:
                key = f"{kname}/{radius}"
                row = done.get((key, cull))
                if row is None:
                    t = time_config(torch, render, scene, cam, kind, order, radius, steps, warmup, 0, rect, cull)
                    row = summary(t, W, H)
                    del t
                    print(f"[bench] sweep {key}{' culled' if cull else ''}: {row['ms_per_step']:.4f} ms K={row['keys']} "
                          f"E={row['evals']}", file=sys.stderr, flush=True)
                sec[key] = row
        base = sec["exp/sigma3"]["ms_per_step"]
        for row in sec.values():
            row["speedup_vs_exp_sigma3"] = round(base / row["ms_per_step"], 4)
        gs = sec["exp/exp_opacity"]["ms_per_step"]
        sec["table3_analogue"] = {lbl: {"config": key, "ms_per_step": sec[key]["ms_per_step"],
                                        "change_vs_g_S_pct": round(100.0 * (sec[key]["ms_per_step"] / gs - 1.0), 1)}
                                  for lbl, key in TABLE3}
        out["tile_culled" if cull else "plain"] = sec
    return out


def time_batched(torch, render, scenes, steps, rect):
    """96 views of 6 scenes (100k-2M splats): per-view sequential frames against
    one batched frame (eager, then replayed from a captured HIP graph)."""
    from paper_2603_18707_amd import _lib, batch
    sc_np, views = scenes.workload_batched()
    dev = [render.to_device(s) for s in sc_np]
    kern = render.kernel_spec("poly", 1, "opacity")
    params = _lib.gs_params_default()
    params.rect_mode = RECT_MODES[rect]
    stream = torch.cuda.current_stream()
    npix = sum(int(c.width) * int(c.height) for _, c in views)

    # per-view sequential launches (capacity fitted once per view, outside the timing)
    rs = []
    for si, cam in views:
        r = render.Rasterizer(kern)
        r.params.rect_mode = RECT_MODES[rect]
        f = r.render(dev[si], cam)
        r.capacity = int(int(f["binned"]["num_keys"].item()) * 1.05) + 4096
        rs.append(r)
    for (si, cam), r in zip(views, rs):
        pr = r.preprocess(dev[si], cam)
        r.rasterize(pr, r.bin_sort(pr, cam), cam)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        for (si, cam), r in zip(views, rs):
            pr = r.preprocess(dev[si], cam)
            r.rasterize(pr, r.bin_sort(pr, cam), cam)
    b.record(stream)
    torch.cuda.synchronize()
    seq_ms = a.elapsed_time(b) / steps
    del rs

    br = batch.BatchRenderer(dev, views, kern, params)
    K = br.render_fit()
    br.capacity = int(K * 1.05) + 4096
    br._layout()
    tuned = batch.tune_batch(br)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(steps):
        br.render()
    b.record(stream)
    torch.cuda.synchronize()
    eager_ms = a.elapsed_time(b) / steps
    br.capture()
    br.replay()
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(steps):
        br.replay()
    b.record(stream)
    torch.cuda.synchronize()
    graph_ms = a.elapsed_time(b) / steps
    assert int(br.overflow.item()) == 0
    return {"workload": "6 scenes (100k-2M splats, SH3), 96 views 640x360..1920x1080, poly-1/opacity, "
                        + RECT_NAMES[rect],
            "pixels": npix, "keys": K, "pairs": br.pairs,
            "per_view_sequential_ms": round(seq_ms, 3), "batched_eager_ms": round(eager_ms, 3),
            "batched_graph_ms": round(graph_ms, 3),
            "Mpix_per_s_graph": round(npix / (graph_ms * 1e-3) / 1e6, 1),
            "speedup_graph_vs_sequential": round(seq_ms / graph_ms, 3),
            # blend and sort work grows with the copies, not the pixels: the
            # low-resolution views hold more copies per pixel than the 1080p frame
            "keys_per_pixel": round(K / npix, 4), "Gkeys_per_s_graph": round(K / (graph_ms * 1e-3) / 1e9, 3),
            "tuned": {"blend_threads": int(br.params.blend_threads), "workgroups": int(br.workgroups),
                      "blend_stage": int(br.params.blend_stage),
                      "candidates_ms": {f"{k[0]}x{k[1]}x{k[2]}": round(v, 3) for k, v in tuned.items()}}}


def time_heavy(torch, render, scenes, steps, rect, only=None):
    """The 4M-splat heavy-tailed scene (Student-t log-scales) from all 8 orbit
    poses at 1920x1080 and 3840x2160: poly-1/opacity against exp/3 sigma in the
    headline's rectangle mode, binned plainly and with per-tile culling; per
    pose the frame times, and their mean and range. At 4K, pose 1 also in the
    other rectangle mode."""
    import math
    sc, _ = scenes.workload_heavy()
    dev = render.to_device(sc)
    out = {"workload": "4M splats (Student-t log-scales, SH3), 8 orbit poses at 1920x1080 and 3840x2160, "
                       + RECT_NAMES[rect]}
    other = "square" if rect == "box" else "box"
    kernels = (("poly1", "poly", 1, "opacity"), ("exp", "exp", 1, "sigma3"))

    def frame(w, h, view, mode, cull):
        cam = scenes.orbit_camera(w, h, 2.0 * math.pi * view / 8)
        row = {}
        for name, kind, order, radius in kernels:
            t = time_config(torch, render, dev, cam, kind, order, radius, steps, 1, 0, mode, cull, count=False)
            row[name] = {"ms_per_step": round(t["ms"], 3), "keys": t["K"],
                         "stage_ms": [round(x, 3) for x in t["stage_ms"]]}
            del t
            torch.cuda.empty_cache()
        row["speedup_poly1_vs_exp"] = round(row["exp"]["ms_per_step"] / row["poly1"]["ms_per_step"], 4)
        print(f"[bench] heavy {w}x{h} pose {view} {mode}{' tile-culled' if cull else ''}: "
              f"poly1 {row['poly1']['ms_per_step']} ms, exp {row['exp']['ms_per_step']} ms", file=sys.stderr,
              flush=True)
        return row

    for label, (w, h) in (("1080p", (1920, 1080)), ("4k", (3840, 2160))):
        for cull in (False, True):
            key = f"{label}{'_tile_culled' if cull else ''}"
            if only not in (None, "all", key):
                continue
            poses = [frame(w, h, v, rect, cull) for v in range(8)]
            agg = {}
            for name in ("poly1", "exp"):
                ms = np.array([p[name]["ms_per_step"] for p in poses])
                agg[name] = {"ms_mean": round(float(ms.mean()), 3), "ms_min": round(float(ms.min()), 3),
                             "ms_max": round(float(ms.max()), 3),
                             "Mpix_per_s_mean": round(w * h / (ms.mean() * 1e-3) / 1e6, 1)}
            sp = np.array([p["speedup_poly1_vs_exp"] for p in poses])
            out[key] = {"poses": poses, "summary": agg,
                        "speedup_poly1_vs_exp": {"mean": round(float(sp.mean()), 4), "min": round(float(sp.min()), 4),
                                                 "max": round(float(sp.max()), 4),
                                                 "of_mean_times": round(agg["exp"]["ms_mean"] / agg["poly1"]["ms_mean"],
                                                                        4)}}
    if only in (None, "all", "4k_pose1_" + other):
        out["4k_pose1_" + ("ellipse_box" if other == "box" else "square")] = frame(3840, 2160, 1, other, False)
    return out


def time_train_step(torch, render, scenes, steps):
    """One optimisation step's forward + hand-written backward: 500k splats,
    4 views at 1280x720, poly-1/opacity, L1 loss against targets rendered
    from a perturbed copy of the scene."""
    from paper_2603_18707_amd import autograd
    sc, tgt, cams = scenes.workload_train()
    kern = render.kernel_spec("poly", 1, "opacity")
    dt = render.to_device(tgt)
    targets = []
    for cam in cams:
        r = render.Rasterizer(kern)
        targets.append(r.render(dt, cam)["image"].clone())
    dev = render.to_device(sc)
    leaves = [t.clone().requires_grad_(True) for t in (dev.means3d, dev.scales, dev.quats, dev.opacities, dev.sh)]

    rs = [render.Rasterizer(kern, reuse_buffers=False) for _ in cams]

    def step(sync):
        loss = 0.0
        for cam, tg, r in zip(cams, targets, rs):
            img = autograd.render(*leaves, sc.sh_degree, cam, kern, rasterizer=r, sync=sync)
            loss = loss + (img - tg).abs().mean()
        loss.backward()
        return loss

    # warm-up: one step fits every view's key capacity, more run the timed
    # path (bin with it, overflow flags read back once after the loop) until
    # the allocator's pool and the clocks have settled
    step(True)
    for _ in range(8):
        step(False)
    torch.cuda.synchronize()
    for r in rs:
        r.check_overflow()
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        for t in leaves:
            t.grad = None
        loss = step(False)
    b.record(stream)
    torch.cuda.synchronize()
    for r in rs:
        r.check_overflow()
    ms = a.elapsed_time(b) / steps
    g = torch.cat([t.grad.reshape(-1) for t in leaves])
    assert torch.isfinite(g).all()

    # stage breakdown of the same step, launched directly: per view the
    # forward frame, the blend adjoint and the projection adjoint
    scene = render.DeviceScene(*[t.detach() for t in leaves], sc.sh_degree)
    frames = [r.render(scene, cam) for cam, r in zip(cams, rs)]
    dls = [torch.sign(f["image"] - tg) / tg.numel() for f, tg in zip(frames, targets)]
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for s in range(steps):
        e = ev[s]
        e[0].record(stream)
        frames = [r.render(scene, cam, sync=False) for cam, r in zip(cams, rs)]
        e[1].record(stream)
        g2 = [autograd.rasterize_backward(r, f, cam, dl) for cam, r, f, dl in zip(cams, rs, frames, dls)]
        e[2].record(stream)
        for cam, r, f, g in zip(cams, rs, frames, g2):
            autograd.preprocess_backward(r, scene, f, cam, g)
        e[3].record(stream)
    torch.cuda.synchronize()
    for r in rs:
        r.check_overflow()
    st = np.median(np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3])]
                             for e in ev]), axis=0)
    walked = sum(int(f["last_contrib"].to(torch.int64).sum().item()) for f in frames)
    n = scene.n
    # projection adjoint bytes per splat and view: the scene read (236 at SH3),
    # the 2D gradients read (36), the scene gradients written (236), tiles (4)
    pb = 4 * n * (2 * (44 + 12 * (sc.sh_degree + 1) ** 2) + 36 + 4)
    return {"workload": "500k splats (SH3), 4 views 1280x720, poly-1/opacity, L1 loss, forward + backward",
            "ms_per_step": round(ms, 3), "views_per_s": round(4 / (ms * 1e-3), 1), "loss": float(loss),
            "stage_ms_4_views": {"forward_frames": round(float(st[0]), 3), "blend_adjoint": round(float(st[1]), 3),
                                 "projection_adjoint": round(float(st[2]), 3)},
            "blend_adjoint_pairs": walked,
            "blend_adjoint_pairs_per_s": round(walked / (float(st[1]) * 1e-3), 1),
            "projection_adjoint_hbm": {"bytes": pb, "frac": round(pb / (float(st[2]) * 1e-3) / HBM_PEAK, 4)}}


def cpu_baseline(scene_np, cam, gpu_image, target_s, rect_mode):
    """The FP64 oracle on a bounded pixel sample of the same frame (poly-1, opacity radius)."""
    from oracle import core as ocore

    c = (0.773, -0.773 / 4.386)
    cfg = ocore.Cfg(kind=ocore.KERNEL_POLY, order=1, radius_mode=ocore.RADIUS_POLY_OPACITY, coeffs=c,
                    alpha_band=2e-6, rect_mode=rect_mode).float_params()
    t0 = time.perf_counter()
    proj = ocore.project(scene_np, cam, cfg)
    rec = ocore.round_records(proj)
    order = ocore.depth_order(proj["depth32"])
    t_setup = time.perf_counter() - t0
    W, H = int(cam.width), int(cam.height)
    from paper_2603_18707_amd import scenes
    probe = scenes.sample_pixels(W, H, 256, seed=77)
    t0 = time.perf_counter()
    ocore.render_pixels(rec, cfg, probe, order)
    per_px = (time.perf_counter() - t0) / probe.shape[0]
    m = int(min(W * H, max(256, (target_s - t_setup) / max(per_px, 1e-9))))
    pix = scenes.sample_pixels(W, H, m, seed=78)
    t0 = time.perf_counter()
    res = ocore.render_pixels(rec, cfg, pix, order)
    t_px = time.perf_counter() - t0
    full_s = t_setup + t_px * (W * H) / m
    g = gpu_image[:, pix[:, 1], pix[:, 0]].T
    good = res["flags"] == 0
    err = float(np.abs(g - res["color"]).max(axis=1)[good].max())
    return dict(value=W * H / full_s / 1e6, unit="Mpix/s", cores=ocore.num_threads(), kind="oracle",
                sample=f"{m} of {W * H} pixels of the poly-1/opacity frame after a full FP64 projection of "
                       f"all splats; full-frame time extrapolated {full_s:.1f} s",
                seconds=round(t_setup + t_px, 2)), err, int((~good).sum()), m


def parse_only(spec):
    parts = spec.split("/")
    names = {k[0]: k for k in SWEEP_KERNELS}
    if len(parts) not in (2, 3) or parts[0] not in names or parts[1] not in SWEEP_RADII or \
            (len(parts) == 3 and parts[2] not in ("culled", "mfma")):
        raise SystemExit(f"--only {spec!r}: expected KERNEL/RADIUS[/culled|/mfma]")
    _, kind, order = names[parts[0]]
    extra = parts[2] if len(parts) == 3 else ""
    return parts[0], kind, order, parts[1], extra == "culled", extra == "mfma"


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2603_18707_amd import _lib, render, scenes

    _lib.lib()
    torch.cuda.set_device(0)
    print(f"[bench] {_lib.gs_version()} on {torch.cuda.get_device_name(0)}", file=sys.stderr, flush=True)
    if a.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.heavy_only:
        print(json.dumps({"heavy": time_heavy(torch, render, scenes, max(3, a.steps // 10), a.rect, a.heavy_only)}),
              flush=True)
        return
    if a.train_only:
        print(json.dumps({"train_step": time_train_step(torch, render, scenes, max(10, a.steps // 3))}), flush=True)
        return
    if a.batched_only:
        print(json.dumps({"batched": time_batched(torch, render, scenes, max(2, a.steps // 10), a.rect)}), flush=True)
        return
    scene_np, cam = scenes.workload_scene()
    scene = render.to_device(scene_np)
    W, H = cam.width, cam.height
    if a.only:
        name, kind, order, radius, cull, mfma = parse_only(a.only)
        t = time_config(torch, render, scene, cam, kind, order, radius, a.steps, a.warmup, a.blend_threads, a.rect,
                        cull, mfma=mfma)
        print(json.dumps({"only": a.only, "rect": RECT_NAMES[a.rect], **summary(t, W, H)}), flush=True)
        return
    kernels = [("poly1", "poly", 1, "opacity"), ("exp", "exp", 1, "sigma3")]
    res = {}
    for name, kind, order, radius in kernels:
        res[name] = time_config(torch, render, scene, cam, kind, order, radius, a.steps, a.warmup, a.blend_threads,
                                a.rect)
        r = res[name]
        print(f"[bench] {name} ({a.rect}): {r['ms']:.4f} ms/frame median, {r['ms_mean']:.4f} mean (pre "
              f"{r['stage_ms'][0]:.4f}, sort {r['stage_ms'][1]:.4f}, blend {r['stage_ms'][2]:.4f}) K={r['K']} "
              f"E={r['E']} threads={r['threads']} tuned={r['tuned']}", file=sys.stderr, flush=True)

    head = res["poly1"]
    # whole-job throughput: K frames back to back, bracketed by synchronisation
    ms = head["ms_clean"]
    mpix = W * H / (ms * 1e-3) / 1e6
    evals = head["E"] / (ms * 1e-3)
    blend_s = head["blend_ms"] * 1e-3
    achieved = head["E"] * OPS_8D["poly1"] / blend_s / 1e12
    refined = (head["E"] * OPS_EVAL["poly1"] + head["B"] * OPS_BLEND) / blend_s / 1e12
    ntiles = ((W + 15) // 16) * ((H + 15) // 16)
    sb = stage_bytes(scene.n, scene.sh_degree, head["K"], ntiles, W * H)
    stage_roof = {}
    for i, stg in enumerate(("preprocess", "bin_sort", "blend")):
        gbs = sb[stg] / (head["stage_ms"][i] * 1e-3)
        stage_roof[stg] = {"bound": "alu" if stg == "blend" else "hbm", "algorithmic_bytes": sb[stg],
                           "GB_per_s": round(gbs / 1e9, 1), "hbm_frac": round(gbs / HBM_PEAK, 4)}
    stage_roof["blend"].update(ops=head["E"] * OPS_8D["poly1"], alu_frac=round(achieved / VALU_PEAK_TOPS, 4))

    traffic = None
    prof = os.path.join(ROOT, "profiles", "blend_poly1_scene1m_1080p_counters.json")
    if os.path.exists(prof):
        with open(prof) as f:
            pc = json.load(f)
        if pc.get("kernel_source_sha1") == kernel_source_hash() and pc.get("rect") == a.rect:
            traffic = pc.get("hbm_bytes_per_launch")

    hrow = summary(head, W, H)
    out = {
        "metric": METRIC, "value": round(mpix, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "1M splats (64 clusters, SH3), 1920x1080, poly-1 kernel, opacity-dependent radius, "
                               + RECT_NAMES[a.rect],
                   "splats": scene.n, "width": W, "height": H, "kernel": "poly1", "radius": "opacity",
                   "rect": RECT_NAMES[a.rect], "blend_threads": head["threads"], "blend_stage": head["stage"],
                   "blend_tuning_ms": head["tuned"]},
        "ms_per_step_median": round(head["ms"], 4),
        "ms_per_step_range": [round(head["ms_min"], 4), round(head["ms_max"], 4)],
        "ms_per_step_mean_with_stage_events": round(head["ms_mean"], 4),
        "splat_pixel_evals_per_s": round(evals, 1),
        "keys": head["K"], "evals": head["E"], "list_entries": head["E_list"], "blended": head["B"],
        "scheduled_pairs_bound": head["K"] * 256,
        "stage_ms": hrow["stage_ms"],
        "roofline": {"bound": "alu", "kernel": "blend_fwd<poly1>", "achieved": round(achieved, 3),
                     "peak": round(VALU_PEAK_TOPS, 2), "unit": "Tops/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                     "traffic": traffic, "ops_per_eval": OPS_8D["poly1"],
                     "refined": {"achieved": round(refined, 3), "frac": round(refined / VALU_PEAK_TOPS, 4),
                                 "ops": f"{OPS_EVAL['poly1']} per evaluated pair + {OPS_BLEND} per blended pair"}},
        "stage_roofline": stage_roof,
    }
    e = res["exp"]
    out["exp_sigma3"] = summary(e, W, H)
    out["exp_sigma3"]["roofline_frac"] = round(
        e["E"] * (OPS_8D["exp"] + TRANS_SLOTS["exp"]) / (e["blend_ms"] * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4)
    out["speedup_vs_exp_sigma3"] = round(e["ms_clean"] / ms, 4)
    out["speedup_vs_exp_sigma3_medians"] = round(e["ms"] / head["ms"], 4)
    done = {("poly1/opacity", False): hrow, ("exp/sigma3", False): out["exp_sigma3"]}

    # the same frames with the quadric on the matrix cores (gs_rasterize_fwd_mfma)
    mf = {"blend": "gs_rasterize_fwd_mfma (v_mfma_f32_32x32x2_f32 quadric, 256 threads per tile)"}
    for name, kind, order, radius in kernels:
        t = time_config(torch, render, scene, cam, kind, order, radius, a.steps, a.warmup, 256, a.rect, mfma=True,
                        count=False)
        mf[name] = summary(t, W, H)
        mf[name]["blend_vs_vector_blend"] = round(t["blend_ms"] / res[name]["blend_ms"], 3)
        print(f"[bench] {name} (mfma blend): {t['ms']:.4f} ms/frame, blend {t['blend_ms']:.4f}", file=sys.stderr,
              flush=True)
    out["mfma_blend"] = mf

    other = "square" if a.rect == "box" else "box"
    alt = {"rect": RECT_NAMES[other]}
    for name, kind, order, radius in kernels:
        t = time_config(torch, render, scene, cam, kind, order, radius, a.steps, a.warmup, a.blend_threads, other)
        alt[name] = summary(t, W, H)
        print(f"[bench] {name} ({other}): {t['ms']:.4f} ms/frame K={t['K']}", file=sys.stderr, flush=True)
    alt["speedup_poly1_vs_exp"] = round(alt["exp"]["ms_per_step"] / alt["poly1"]["ms_per_step"], 4)
    out["other_rect"] = alt
    if not a.no_sweep:
        print("[bench] kernel x culling sweep ...", file=sys.stderr, flush=True)
        out["sweep"] = time_sweep(torch, render, scene, cam, a.steps, a.warmup, a.rect, done)
        tc = out["sweep"]["tile_culled"]
        out["tile_culled"] = {"rect": RECT_NAMES[a.rect], "binning": "gs_bin_sort_culled",
                              "poly1": tc["poly1/opacity"], "exp": tc["exp/sigma3"],
                              "speedup_poly1_vs_exp": round(tc["exp/sigma3"]["ms_per_step"] /
                                                            tc["poly1/opacity"]["ms_per_step"], 4)}
    if not a.no_batched:
        print("[bench] batched multi-view ...", file=sys.stderr, flush=True)
        out["batched"] = time_batched(torch, render, scenes, max(2, a.steps // 10), a.rect)
        out["batched"]["Gkeys_per_s_single_1m_frame"] = round(head["K"] / (ms * 1e-3) / 1e9, 3)
        print(f"[bench] batched: {out['batched']}", file=sys.stderr, flush=True)
    if not a.no_heavy:
        print("[bench] heavy scene ...", file=sys.stderr, flush=True)
        out["heavy"] = time_heavy(torch, render, scenes, max(3, a.steps // 10), a.rect)
    if not a.no_train:
        print("[bench] training step ...", file=sys.stderr, flush=True)
        out["train_step"] = time_train_step(torch, render, scenes, max(10, a.steps // 3))
        print(f"[bench] train: {out['train_step']}", file=sys.stderr, flush=True)
    if not a.no_cpu:
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        # the oracle is compared with the frame the counting build rendered
        # (identical outputs to the timed blend)
        cb, err, nflag, m = cpu_baseline(scene_np, cam, head["image"].cpu().numpy(), a.cpu_seconds, RECT_MODES[a.rect])
        out["cpu_baseline"] = cb
        out["max_abs_err_vs_oracle"] = err
        out["oracle_flagged_pixels"] = f"{nflag} of {m}"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
