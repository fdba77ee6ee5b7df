"""Pins of the reference's front-to-back compositing (Sec. 2, Eq. 1 and the
alpha blending it feeds) with hand-built splat records.

Closed forms: one splat gives alpha * rgb; two splats give the over operator;
white splats give exactly 1 - T; transmittance never increases; early
termination stops before the splat that would push T below T_min. A plain
Python per-pixel loop on a tiny scene must agree with the C reference.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

from oracle import core
from paper_2603_18707_amd import scenes

PAPER_F1 = (0.773, -0.773 / 4.386, 0.0, 0.0)


def _records(splats, tile_rect=(0, 0, 3, 3)):
    """splats: list of (u, v, (a, b, c), opac, rgb, depth)."""
    n = len(splats)
    rec = dict(means2d=np.array([s[0:2] for s in splats], np.float64).reshape(n, 2),
               conic=np.array([s[2] for s in splats], np.float64).reshape(n, 3),
               opac=np.array([s[3] for s in splats], np.float64),
               rgb=np.array([s[4] for s in splats], np.float64).reshape(n, 3),
               depth32=np.array([s[5] for s in splats], np.float32),
               rect=np.tile(np.array(tile_rect, np.int32), (n, 1)),
               flags=np.zeros(n, np.uint8))
    return rec


def test_single_splat_is_alpha_times_rgb():
    for cfg in (core.Cfg(kind=core.KERNEL_EXP), core.Cfg(kind=core.KERNEL_POLY, order=1, coeffs=PAPER_F1)):
        rec = _records([(10.5, 7.5, (0.2, 0.05, 0.1), 0.8, (0.3, 0.6, 0.9), 2.0)])
        px = np.array([[10, 7], [12, 7], [11, 9], [40, 40]], np.int32)
        r = core.render_pixels(rec, cfg, px)
        for j, (x, y) in enumerate(px):
            dx, dy = x + 0.5 - 10.5, y + 0.5 - 7.5
            Q = 0.2 * dx * dx + 2 * 0.05 * dx * dy + 0.1 * dy * dy
            k = math.exp(-Q / 2) if cfg.kind == core.KERNEL_EXP else max(PAPER_F1[0] + PAPER_F1[1] * Q, 0.0)
            a = min(0.99, 0.8 * k)
            if a < 1 / 255:
                a = 0.0
            assert r["color"][j] == pytest.approx(a * np.array([0.3, 0.6, 0.9]), abs=1e-15)
            assert r["T"][j] == pytest.approx(1 - a, abs=1e-15)


def test_two_splats_over_operator():
    cfg = core.Cfg(kind=core.KERNEL_POLY, order=1, coeffs=PAPER_F1)
    # the farther splat is listed first: order comes from depth, not position
    rec = _records([(5.5, 5.5, (0.1, 0.0, 0.1), 0.9, (0.0, 1.0, 0.0), 5.0),
                    (5.5, 5.5, (0.05, 0.0, 0.05), 0.6, (1.0, 0.0, 0.0), 1.0)])
    r = core.render_pixels(rec, cfg, np.array([[5, 5], [7, 4]], np.int32))
    for j, (x, y) in enumerate([(5, 5), (7, 4)]):
        d2 = (x + 0.5 - 5.5) ** 2 + (y + 0.5 - 5.5) ** 2
        a_front = 0.6 * (PAPER_F1[0] + PAPER_F1[1] * 0.05 * d2)
        a_back = 0.9 * (PAPER_F1[0] + PAPER_F1[1] * 0.1 * d2)
        ref = np.array([1.0, 0.0, 0.0]) * a_front + np.array([0.0, 1.0, 0.0]) * a_back * (1 - a_front)
        assert r["color"][j] == pytest.approx(ref, abs=1e-15)
        assert r["T"][j] == pytest.approx((1 - a_front) * (1 - a_back), abs=1e-15)
        assert r["n_contrib"][j] == 2


def _random_records(rng, n, size, white=False):
    sp = []
    for _ in range(n):
        s = rng.uniform(0.5, 4.0)
        a, c = 1 / (s * rng.uniform(0.5, 1.5)) ** 2, 1 / (s * rng.uniform(0.5, 1.5)) ** 2
        b = rng.uniform(-0.4, 0.4) * math.sqrt(a * c)
        rgb = (1.0, 1.0, 1.0) if white else tuple(rng.uniform(0, 1, 3))
        sp.append((rng.uniform(0, size), rng.uniform(0, size), (a, b, c), rng.uniform(0.05, 1.0), rgb,
                   rng.uniform(1, 10)))
    return _records(sp, (0, 0, (size - 1) // 16, (size - 1) // 16))


@pytest.mark.parametrize("kind", [core.KERNEL_EXP, core.KERNEL_POLY])
def test_white_splats_give_one_minus_T(kind):
    rng = np.random.default_rng(3)
    cfg = core.Cfg(kind=kind, order=1, coeffs=PAPER_F1)
    rec = _random_records(rng, 60, 32, white=True)
    r = core.render_pixels(rec, cfg, core.all_pixels(32, 32))
    assert np.allclose(r["color"], (1 - r["T"])[:, None], atol=1e-12)
    assert np.all(r["T"] > 0) and np.all(r["T"] <= 1)


def test_transmittance_never_increases():
    rng = np.random.default_rng(4)
    cfg = core.Cfg(kind=core.KERNEL_POLY, order=1, coeffs=PAPER_F1, t_min=0.0)
    rec = _random_records(rng, 40, 32)
    order = core.depth_order(rec["depth32"])
    prev = np.ones(32 * 32)
    for k in range(1, 41):
        sub = {key: (val[order[:k]] if isinstance(val, np.ndarray) else val) for key, val in rec.items()}
        T = core.render_pixels(sub, cfg, core.all_pixels(32, 32))["T"]
        assert np.all(T <= prev + 1e-15)
        prev = T


def test_early_termination_stops_before_the_splat():
    cfg = core.Cfg(kind=core.KERNEL_EXP, t_min=1e-4)
    # five opaque splats centred on the pixel: alpha = 0.95 each
    rec = _records([(3.5, 3.5, (0.01, 0.0, 0.01), 0.95, (0.1 * (i + 1),) * 3, float(i + 1)) for i in range(5)])
    r = core.render_pixels(rec, cfg, np.array([[3, 3]], np.int32))
    T, C = 1.0, 0.0
    for i in range(3):            # T after 3 splats: 1.25e-4; the 4th would give 6.25e-6
        C += 0.1 * (i + 1) * 0.95 * T
        T *= 0.05
    assert r["n_contrib"][0] == 3 and r["n_eval"][0] == 4 and r["last_contrib"][0] == 3
    assert r["T"][0] == pytest.approx(T, rel=1e-14)
    assert r["color"][0] == pytest.approx([C] * 3, rel=1e-14)


def test_background_and_rect_membership():
    cfg = core.Cfg(kind=core.KERNEL_EXP, bg=(0.2, 0.4, 0.6))
    rec = _records([(8.0, 8.0, (0.01, 0.0, 0.01), 0.5, (1, 1, 1), 1.0)], tile_rect=(0, 0, 0, 0))
    r = core.render_pixels(rec, cfg, np.array([[8, 8], [17, 8]], np.int32))
    # pixel in tile (1, 0) is outside the splat's rectangle: background only, nothing evaluated
    assert r["n_eval"][1] == 0 and r["color"][1] == pytest.approx([0.2, 0.4, 0.6])
    a = 0.5 * math.exp(-0.5 * 0.01 * 0.5)
    assert r["color"][0] == pytest.approx(a + (1 - a) * np.array([0.2, 0.4, 0.6]), abs=1e-15)


def _python_loop(rec, cfg, W, H):
    """Per-pixel loop written out directly from the compositing rule."""
    n = rec["opac"].shape[0]
    order = sorted(range(n), key=lambda i: (float(rec["depth32"][i]), i))
    out = np.zeros((H, W, 3))
    Tout = np.ones((H, W))
    c = list(cfg.coeffs)
    for y in range(H):
        for x in range(W):
            T, C = 1.0, np.zeros(3)
            for i in order:
                r = rec["rect"][i]
                if not (r[0] <= x // 16 <= r[2] and r[1] <= y // 16 <= r[3]):
                    continue
                dx, dy = x + 0.5 - rec["means2d"][i][0], y + 0.5 - rec["means2d"][i][1]
                a_, b_, c_ = rec["conic"][i]
                Q = a_ * dx * dx + 2 * b_ * dx * dy + c_ * dy * dy
                if cfg.kind == core.KERNEL_EXP:
                    k = math.exp(-Q / 2)
                else:
                    k = max(sum(c[j] * Q ** j for j in range(cfg.order + 1)), 0.0)
                    if cfg.order == 2 and Q >= core.first_root(c, 2, 0.0):
                        k = 0.0
                alpha = min(cfg.alpha_max, rec["opac"][i] * k)
                if alpha < cfg.eps:
                    continue
                Tn = T * (1 - alpha)
                if Tn < cfg.t_min:
                    break
                C += rec["rgb"][i] * alpha * T
                T = Tn
            out[y, x], Tout[y, x] = C, T
    return out, Tout


@pytest.mark.parametrize("kind,order", [(core.KERNEL_EXP, 1), (core.KERNEL_POLY, 1), (core.KERNEL_POLY, 2),
                                        (core.KERNEL_POLY, 3)])
def test_tiny_scene_matches_python_loop(golden_coeffs, kind, order):
    sc = scenes.tiny_scene(25, seed=11)
    sc.scales *= 3.0
    cam = scenes.tiny_camera(24, 20)
    coeffs = PAPER_F1 if order == 1 else tuple(golden_coeffs[f"fit{order}"]["c"])
    cfg = core.Cfg(kind=kind, order=order, coeffs=coeffs,
                   radius_mode=core.RADIUS_SIGMA3 if kind == core.KERNEL_EXP else core.RADIUS_POLY_OPACITY)
    full = core.render_image(sc, cam, cfg, round_to=None)
    ref, Tref = _python_loop(full["proj"], cfg, 24, 20)
    assert np.allclose(full["image"].transpose(1, 2, 0), ref, atol=1e-13)
    assert np.allclose(full["T"], Tref, atol=1e-13)
    assert full["image"].max() > 0.05  # the scene is not empty


@pytest.mark.parametrize("kind,order", [(core.KERNEL_EXP, 1), (core.KERNEL_POLY, 1), (core.KERNEL_POLY, 3)])
def test_reach_bounds_the_flagged_decisions(golden_coeffs, kind, order):
    """``reach`` bounds what the flagged decisions can change: moving eps
    and t_min anywhere inside their bands (which flips exactly decisions the
    flags mark, and no others) leaves unflagged pixels bit-identical and
    moves flagged ones by at most reach (colour and T). Wide bands make
    thousands of pixels flagged, with stops and skips flipped together."""
    scene = scenes.tiny_scene(1500, seed=41)
    scene.scales *= 2.0
    scene.opacities[:] = np.clip(scene.opacities * 1.6, 0.0, 0.99).astype(np.float32)
    cam = scenes.tiny_camera(64, 64)
    c = tuple(golden_coeffs["paper1"]["c"]) if order == 1 else tuple(golden_coeffs[f"fit{order}"]["c"])
    base = core.Cfg(kind=kind, order=order, radius_mode=core.RADIUS_SIGMA3, coeffs=c,
                    alpha_band=2e-3, t_band_rel=0.05)
    proj = core.round_records(core.project(scene, cam, base))
    pix = core.all_pixels(64, 64)
    ref = core.render_pixels(proj, base, pix)
    fl = ref["flags"] != 0
    assert fl.sum() > 300 and (~fl).sum() > 300
    assert ((ref["flags"] & core.PIX_T_NEAR) != 0).sum() > 20
    worst = 0.0
    for de in (-0.99, -0.5, 0.5, 0.99):
        for dt in (-0.99, 0.0, 0.99):
            cfg = replace(base, eps=base.eps + de * base.alpha_band, t_min=base.t_min * (1.0 + dt * base.t_band_rel))
            r = core.render_pixels(proj, cfg, pix)
            dc = np.abs(r["color"] - ref["color"]).max(axis=1)
            dT = np.abs(r["T"] - ref["T"])
            assert np.all(dc[~fl] == 0.0) and np.all(dT[~fl] == 0.0), (de, dt)
            assert np.all(dc[fl] <= ref["reach"][fl, 0] * (1 + 1e-12) + 1e-15), (de, dt, (dc - ref["reach"][:, 0]).max())
            assert np.all(dT[fl] <= ref["reach"][fl, 1] * (1 + 1e-12) + 1e-15), (de, dt)
            worst = max(worst, float((dc[fl] / np.maximum(ref["reach"][fl, 0], 1e-30)).max()))
    assert worst > 0.25  # the bound is reached to within a small factor somewhere
    assert np.all(ref["reach"][~fl] == 0.0)
