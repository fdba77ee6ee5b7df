"""Pins of the reference's tile rectangles in both modes: the bounding square
of radius r = k sqrt(lambda_max) (Sec. 2.1) and the axis-aligned box of the
ellipse Q = k^2.

The box must lie inside the square, must contain every point of the ellipse
(sampled on its boundary, from its own parametrisation), and, for radii that
bound where alpha >= eps (POLY_* and EXP_OPACITY), must leave every pixel of
the image unchanged while dropping copies.
"""
import math

import numpy as np
import pytest

from oracle import binning, core
from paper_2603_18707_amd import scenes
from tests import helpers as H


def _both(scene, cam, kind, order, radius):
    sq = core.project(scene, cam, H.oracle_cfg(kind, order, radius, rect_mode=core.RECT_SQUARE))
    bx = core.project(scene, cam, H.oracle_cfg(kind, order, radius, rect_mode=core.RECT_ELLIPSE_BOX))
    return sq, bx


@pytest.mark.parametrize("kind,order,radius", [("poly", 1, "opacity"), ("exp", 1, "sigma3"), ("poly", 2, "universal")])
def test_box_inside_square_and_holds_the_ellipse(kind, order, radius):
    scene, _ = scenes.workload_heavy(n=20_000)
    cam = scenes.orbit_camera(1920, 1080, 0.3)
    sq, bx = _both(scene, cam, kind, order, radius)
    live = bx["tiles"] > 0
    assert np.array_equal(sq["depth32"], bx["depth32"]) and np.array_equal(sq["conic"], bx["conic"])
    # inside the square
    r1, r2 = sq["rect"][live], bx["rect"][live]
    assert np.all(r2[:, 0] >= r1[:, 0]) and np.all(r2[:, 1] >= r1[:, 1])
    assert np.all(r2[:, 2] <= r1[:, 2]) and np.all(r2[:, 3] <= r1[:, 3])
    assert bx["tiles"].sum() < 0.8 * sq["tiles"].sum()  # thin footprints: a large cut
    # every point of the ellipse Q = k^2 falls in a tile of the box (or outside the image)
    idx = np.nonzero(live)[0]
    a, b, c = bx["conic"][idx].T
    Sxx, Syy, Sxy = c / (a * c - b * b), a / (a * c - b * b), -b / (a * c - b * b)
    mid = 0.5 * (Sxx + Syy)
    lmax = mid + np.sqrt(np.maximum(mid * mid - (Sxx * Syy - Sxy * Sxy), 0.0))
    k = bx["radius"][idx] / math.sqrt(1.0) / np.sqrt(lmax) / (1.0 + 2.0 ** -20) * 0.999999  # just inside
    L = np.linalg.cholesky(np.stack([np.stack([Sxx, Sxy], -1), np.stack([Sxy, Syy], -1)], 1))
    th = np.linspace(0.0, 2.0 * math.pi, 64, endpoint=False)
    circ = np.stack([np.cos(th), np.sin(th)], 0)  # unit circle -> ellipse x^T S^-1 x = k^2
    pts = bx["means2d"][idx][:, :, None] + k[:, None, None] * np.einsum("nij,jm->nim", L, circ)
    tx, ty = np.floor(pts[:, 0] / 16), np.floor(pts[:, 1] / 16)
    r = bx["rect"][idx]
    onscreen = (tx >= 0) & (tx < 120) & (ty >= 0) & (ty < 68)
    inside = (tx >= r[:, 0, None]) & (tx <= r[:, 2, None]) & (ty >= r[:, 1, None]) & (ty <= r[:, 3, None])
    assert np.all(inside | ~onscreen)


@pytest.mark.parametrize("kind,order,radius", [("poly", 1, "opacity"), ("poly", 3, "universal"),
                                               ("exp", 1, "exp_opacity")])
def test_box_changes_no_pixel_for_alpha_bounding_radii(kind, order, radius):
    scene, cam = scenes.workload_tiny()
    scene.scales *= 2.0
    sq, bx = _both(scene, cam, kind, order, radius)
    cfg = H.oracle_cfg(kind, order, radius)
    pix = core.all_pixels(128, 128)
    a = core.render_pixels(core.round_records(sq), cfg, pix)
    b = core.render_pixels(core.round_records(bx), cfg, pix)
    assert np.array_equal(a["color"], b["color"]) and np.array_equal(a["n_contrib"], b["n_contrib"])
    assert np.all(b["n_eval"] <= a["n_eval"]) and b["n_eval"].sum() < a["n_eval"].sum()
    assert bx["tiles"].sum() < sq["tiles"].sum()
    kb, _, _ = binning.bin_and_sort(bx["rect"], bx["depth32"], 8, 8)
    assert kb.shape[0] == bx["tiles"].sum()


def test_square_mode_is_the_default():
    assert core.Cfg().rect_mode == core.RECT_SQUARE
