"""Throughput of the polynomial-kernel splatting path on one MI355X.

Workload: 1,000,000 splats (64 anisotropic clusters in a 20-unit box, log-scales
N(-4.5, 1), opacity logits N(0, 2), SH degree 3), one 1920x1080 camera at
distance 30 with a 60 degree field of view. A step is one full frame:
gs_preprocess -> gs_bin_sort -> gs_rasterize_fwd, inputs resident in HBM.

Headline: poly order 1 with the opacity-dependent radius (Eq. 4); the same
frame with the exponential kernel and 3-sigma culling is timed on the same GPU
for comparison. Prints one JSON line (see the repository's benchmark contract).

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
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

# Algorithmic VALU lane-operations of the blend (one op per add, multiply,
# FMA, min/max, compare or exp), the count the kernel is measured against:
#   every evaluated (pixel, splat) pair: dx, dy (2), quadric a dx^2 + 2b dx dy
#   + c dy^2 (5), kernel (poly-1: 1 FMA; exp: add + exp = 2; poly-2: 3;
#   poly-3: 4), alpha clamp (1), eps test (1);
#   every blended pair in addition: 1 - alpha, T' (2), t_min test (1),
#   alpha T (1), colour FMAs (3).
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--only", default=None, help="time one configuration: poly1|exp")
    ap.add_argument("--blend-threads", type=int, default=0, help="64|128|256; 0 = autotune")
    ap.add_argument("--rect", default="box", choices=("box", "square"),
                    help="tile rectangles of the headline frames: the ellipse's bounding box or the bounding square")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched multi-view measurement")
    ap.add_argument("--no-train", action="store_true", help="skip the forward+backward step measurement")
    ap.add_argument("--no-heavy", action="store_true", help="skip the 4M-splat heavy-tailed scene")
    ap.add_argument("--heavy-only", default=None, metavar="ROW",
                    help="time only the heavy-tailed scene, all rows ('all') or one row such as "
                         "'4k_ellipse_box_tile_culled' (for profiling; prints its own JSON object)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 256 MiB device-to-device copy (calibrates HBM byte counters)")
    return ap.parse_args()


BLEND_SOURCES = ("rasterize.hip", "blend_common.h", "gs_internal.h")


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


def time_config(torch, render, scene, cam, kind, order, radius, steps, warmup, threads=0, rect="box", cull=False):
    """Times `steps` frames; per-stage HIP events inside the same timed loop.
    threads = 0 lets the autotuner pick the blend launch shape during warm-up;
    cull bins with per-tile culling (gs_bin_sort_culled)."""
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
    if threads:
        r.params.blend_threads = threads
    else:
        tuned = autotune.tune_blend(r, out["proj"], b0, cam)
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

    # untimed frame of the counting build: E = kernel evaluations performed,
    # E_list = list entries a per-pixel walk without the box test would evaluate
    full = r.rasterize(proj, b, cam, want_eval=True, want_tested=True)
    torch.cuda.synchronize()
    E = int(full["n_tested"].sum().item())
    E_list = int(full["n_eval"].sum().item())
    B = int(full["n_contrib"].sum().item())
    return dict(ms=total_ms / steps, stage_ms=st.mean(axis=0).tolist(), blend_ms=float(st[:, 2].mean()),
                K=int(b["num_keys"].item()), E=E, E_list=E_list, B=B, image=full["image"].clone(), rast=r,
                threads=int(r.params.blend_threads), tuned=tuned)


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
            "tuned": {"blend_threads": int(br.params.blend_threads), "workgroups": int(br.workgroups),
                      "candidates_ms": {f"{k[0]}x{k[1]}": round(v, 3) for k, v in tuned.items()}}}


def time_heavy(torch, render, scenes, steps, rect, only=None):
    """The 4M-splat heavy-tailed scene (Student-t log-scales), one orbit view at
    1920x1080 and one at 3840x2160: poly-1/opacity against exp/3 sigma, in the
    headline's rectangle mode, and at 4K also in the other one."""
    import math
    sc, _ = scenes.workload_heavy()
    dev = render.to_device(sc)
    out = {"workload": "4M splats (Student-t log-scales, SH3), orbit views 0 (1920x1080) and 1 (3840x2160)"}
    other = "square" if rect == "box" else "box"
    for label, (w, h, view), modes in (("1080p", (1920, 1080, 0), ((rect, False), (rect, True))),
                                       ("4k", (3840, 2160, 1), ((rect, False), (other, False), (rect, True)))):
        cam = scenes.orbit_camera(w, h, 2.0 * math.pi * view / 8)
        for mode, cull in modes:
            key = f"{label}_{'ellipse_box' if mode == 'box' else 'square'}{'_tile_culled' if cull else ''}"
            if only not in (None, "all", key):
                continue
            row = {}
            for name, kind, order, radius in (("poly1", "poly", 1, "opacity"), ("exp", "exp", 1, "sigma3")):
                t = time_config(torch, render, dev, cam, kind, order, radius, steps, 2, 0, mode, cull)
                row[name] = {"ms_per_step": round(t["ms"], 3), "Mpix_per_s": round(w * h / (t["ms"] * 1e-3) / 1e6, 1),
                             "keys": t["K"], "stage_ms": [round(x, 3) for x in t["stage_ms"]]}
                print(f"[bench] heavy {label} {mode}{' tile-culled' if cull else ''} {name}: {t['ms']:.3f} ms "
                      f"K={t['K']} stages={[round(x, 3) for x in t['stage_ms']]}", file=sys.stderr, flush=True)
                del t
                torch.cuda.empty_cache()
            row["speedup_poly1_vs_exp"] = round(row["exp"]["ms_per_step"] / row["poly1"]["ms_per_step"], 4)
            out[key] = row
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

    def step():
        loss = 0.0
        for cam, tg, r in zip(cams, targets, rs):
            img = autograd.render(*leaves, sc.sh_degree, cam, kern, rasterizer=r)
            loss = loss + (img - tg).abs().mean()
        loss.backward()
        return loss

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        for t in leaves:
            t.grad = None
        loss = step()
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    g = torch.cat([t.grad.reshape(-1) for t in leaves])
    assert torch.isfinite(g).all()
    return {"workload": "500k splats (SH3), 4 views 1280x720, poly-1/opacity, L1 loss, forward + backward",
            "ms_per_step": round(ms, 3), "views_per_s": round(4 / (ms * 1e-3), 1), "loss": float(loss)}


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
        print(json.dumps({"heavy": time_heavy(torch, render, scenes, a.steps, a.rect, a.heavy_only)}), flush=True)
        return
    scene_np, cam = scenes.workload_scene()
    scene = render.to_device(scene_np)
    W, H = cam.width, cam.height
    kernels = [("poly1", "poly", 1, "opacity"), ("exp", "exp", 1, "sigma3")]
    if a.only:
        kernels = [c for c in kernels if c[0] == a.only]
    res = {}
    for name, kind, order, radius in kernels:
        res[name] = time_config(torch, render, scene, cam, kind, order, radius, a.steps, a.warmup, a.blend_threads,
                                a.rect)
        r = res[name]
        print(f"[bench] {name} ({a.rect}): {r['ms']:.3f} ms/frame (pre {r['stage_ms'][0]:.3f}, sort {r['stage_ms'][1]:.3f},"
              f" blend {r['stage_ms'][2]:.3f}) K={r['K']} E={r['E']} threads={r['threads']} tuned={r['tuned']}",
              file=sys.stderr, flush=True)

    head = res[kernels[0][0]]
    ms = head["ms"]
    mpix = W * H / (ms * 1e-3) / 1e6
    evals = head["E"] / (ms * 1e-3)
    hname = kernels[0][0]
    ops = head["E"] * OPS_EVAL[hname] + head["B"] * OPS_BLEND
    achieved = ops / (head["blend_ms"] * 1e-3) / 1e12

    traffic = None
    prof = os.path.join(ROOT, "profiles", "blend_poly1_scene1m_1080p_counters.json")
    if os.path.exists(prof):
        with open(prof) as f:
            pc = json.load(f)
        if pc.get("kernel_source_sha1") == kernel_source_hash() and pc.get("rect") == a.rect:
            traffic = pc.get("hbm_bytes_per_launch")

    out = {
        "metric": METRIC, "value": round(mpix, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "1M splats (64 clusters, SH3), 1920x1080, poly-1 kernel, opacity-dependent radius, "
                               + RECT_NAMES[a.rect],
                   "splats": scene.n, "width": W, "height": H, "kernel": "poly1", "radius": "opacity",
                   "rect": RECT_NAMES[a.rect], "blend_threads": head["threads"]},
        "splat_pixel_evals_per_s": round(evals, 1),
        "keys": head["K"], "evals": head["E"], "list_entries": head["E_list"], "blended": head["B"],
        "scheduled_pairs_bound": head["K"] * 256,
        "stage_ms": {"preprocess": round(head["stage_ms"][0], 4), "bin_sort": round(head["stage_ms"][1], 4),
                     "blend": round(head["stage_ms"][2], 4)},
        "roofline": {"bound": "alu", "kernel": "blend_fwd<poly1>", "achieved": round(achieved, 3),
                     "peak": round(VALU_PEAK_TOPS, 2), "unit": "Tops/s",
                     "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": traffic},
    }
    if "exp" in res and hname != "exp":
        e = res["exp"]
        out["exp_sigma3"] = {"ms_per_step": round(e["ms"], 4), "blend_threads": e["threads"], "Mpix_per_s": round(W * H / (e["ms"] * 1e-3) / 1e6, 2),
                             "splat_pixel_evals_per_s": round(e["E"] / (e["ms"] * 1e-3), 1), "keys": e["K"],
                             "evals": e["E"], "list_entries": e["E_list"],
                             "stage_ms": {"preprocess": round(e["stage_ms"][0], 4),
                                          "bin_sort": round(e["stage_ms"][1], 4),
                                          "blend": round(e["stage_ms"][2], 4)}}
        out["speedup_vs_exp_sigma3"] = round(e["ms"] / ms, 4)
    if not a.only:
        other = "square" if a.rect == "box" else "box"
        alt = {"rect": RECT_NAMES[other]}
        for name, kind, order, radius in kernels:
            t = time_config(torch, render, scene, cam, kind, order, radius, a.steps, a.warmup, a.blend_threads, other)
            print(f"[bench] {name} ({other}): {t['ms']:.3f} ms/frame (pre {t['stage_ms'][0]:.3f}, sort "
                  f"{t['stage_ms'][1]:.3f}, blend {t['stage_ms'][2]:.3f}) K={t['K']} E={t['E']}", file=sys.stderr,
                  flush=True)
            alt[name] = {"ms_per_step": round(t["ms"], 4), "Mpix_per_s": round(W * H / (t["ms"] * 1e-3) / 1e6, 2),
                         "keys": t["K"], "evals": t["E"],
                         "stage_ms": {"preprocess": round(t["stage_ms"][0], 4), "bin_sort": round(t["stage_ms"][1], 4),
                                      "blend": round(t["stage_ms"][2], 4)}}
        if "exp" in alt and "poly1" in alt:
            alt["speedup_poly1_vs_exp"] = round(alt["exp"]["ms_per_step"] / alt["poly1"]["ms_per_step"], 4)
        out["other_rect"] = alt
        # the same frames binned with per-tile culling (identical images, shorter lists)
        tc = {"rect": RECT_NAMES[a.rect], "binning": "gs_bin_sort_culled"}
        for name, kind, order, radius in kernels:
            t = time_config(torch, render, scene, cam, kind, order, radius, a.steps, a.warmup, a.blend_threads, a.rect,
                            cull=True)
            print(f"[bench] {name} ({a.rect}, tile-culled): {t['ms']:.3f} ms/frame (pre {t['stage_ms'][0]:.3f}, sort "
                  f"{t['stage_ms'][1]:.3f}, blend {t['stage_ms'][2]:.3f}) K={t['K']} E={t['E']}", file=sys.stderr,
                  flush=True)
            tc[name] = {"ms_per_step": round(t["ms"], 4), "Mpix_per_s": round(W * H / (t["ms"] * 1e-3) / 1e6, 2),
                        "keys": t["K"], "evals": t["E"],
                        "stage_ms": {"preprocess": round(t["stage_ms"][0], 4), "bin_sort": round(t["stage_ms"][1], 4),
                                     "blend": round(t["stage_ms"][2], 4)}}
        if "exp" in tc and "poly1" in tc:
            tc["speedup_poly1_vs_exp"] = round(tc["exp"]["ms_per_step"] / tc["poly1"]["ms_per_step"], 4)
        out["tile_culled"] = tc
    if not a.no_batched and not a.only:
        print("[bench] batched multi-view ...", file=sys.stderr, flush=True)
        out["batched"] = time_batched(torch, render, scenes, max(2, a.steps // 10), a.rect)
        print(f"[bench] batched: {out['batched']}", file=sys.stderr, flush=True)
    if not a.no_heavy and not a.only:
        print("[bench] heavy scene ...", file=sys.stderr, flush=True)
        out["heavy"] = time_heavy(torch, render, scenes, max(3, a.steps // 5), a.rect)
    if not a.no_train and not a.only:
        print("[bench] training step ...", file=sys.stderr, flush=True)
        out["train_step"] = time_train_step(torch, render, scenes, max(3, a.steps // 10))
        print(f"[bench] train: {out['train_step']}", file=sys.stderr, flush=True)
    if not a.no_cpu and hname == "poly1":
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        cb, err, nflag, m = cpu_baseline(scene_np, cam, head["image"].cpu().numpy(), a.cpu_seconds, RECT_MODES[a.rect])
        out["cpu_baseline"] = cb
        out["max_abs_err_vs_oracle"] = err
        out["oracle_flagged_pixels"] = f"{nflag} of {m}"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
