"""Pins of App. A's wider fitting range for the order-2 kernel.

App. A bounds the quadric values a renderer with exact per-tile culling ever
evaluates: a splat culled at its eps cut-off that barely touches a tile is
still evaluated across the whole tile, at most a tile diagonal away, so in
units of the smallest scale s_min the largest value is
x_max = (sqrt(2) p_t / s_min + sqrt(-2 ln eps))^2. Pinned here:
  - that bound by brute force over splats of every orientation with smallest
    scale s_min, culled by the per-tile test, and that the worst case comes
    close to it;
  - the library's order-2 fit over [0, x_max] against the oracle's
    independent fit of the same objective, its monotonicity over the whole
    range (no cut needed), and App. A's remark that with 16-px tiles it is
    practically the order-1 fit.
"""
import math

import numpy as np
import pytest

from oracle import coeffs, core

EPS = 1.0 / 255.0
T = 16


def _cov(s1, s2, th):
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    return R @ np.diag([s1 * s1, s2 * s2]) @ R.T


def test_x_max_bounds_the_evaluated_values():
    s_min = math.sqrt(0.3)
    xm = coeffs.x_max_extended(T, s_min)
    assert xm == pytest.approx((math.sqrt(2) * T / s_min + math.sqrt(2 * math.log(255))) ** 2, rel=1e-14)
    qc = -2.0 * math.log(EPS)  # the splat's cut-off (opacity 1)
    rng = np.random.default_rng(3)
    worst = 0.0
    for it in range(400):
        s1 = s_min * math.exp(rng.uniform(0.0, 2.0)) if it % 4 else s_min
        th = math.pi / 4 if it % 2 else rng.uniform(0, math.pi)
        inv = np.linalg.inv(_cov(s1, s_min, th))
        a, b, c = inv[0, 0], inv[0, 1], inv[1, 1]
        u, v = rng.uniform(60, 68), rng.uniform(60, 68)
        X = math.sqrt(qc * c / (a * c - b * b)) + T
        Y = math.sqrt(qc * a / (a * c - b * b)) + T
        for tx in range(int((u - X) // T), int((u + X) // T) + 1):
            for ty in range(int((v - Y) // T), int((v + Y) // T) + 1):
                x0, y0 = tx * T + 0.5 - u, ty * T + 0.5 - v
                if core.rect_min_q(a, b, c, x0, x0 + T - 1, y0, y0 + T - 1) > qc:
                    continue  # a tile the per-tile test drops
                px = np.arange(T) + x0
                py = np.arange(T) + y0
                X2, Y2 = np.meshgrid(px, py)
                worst = max(worst, float((a * X2 * X2 + 2 * b * X2 * Y2 + c * Y2 * Y2).max()))
    assert worst <= xm
    # pixel centres span 15 px of a 16-px tile: the bound is nearly reached
    assert worst >= 0.85 * xm


@pytest.fixture(scope="module")
def oracle_ext_fit():
    return coeffs.fit(2, coeffs.x_max_extended(T, math.sqrt(0.3)))


def _library_ext_f2():
    from paper_2603_18707_amd import _lib as L
    return list(L.gs_kernel_order2_tile_range(L.RADIUS_POLY_OPACITY).coeffs)


def test_library_fit_matches_the_oracle_fit(oracle_ext_fit):
    xm = coeffs.x_max_extended(T, math.sqrt(0.3))
    lib_c = _library_ext_f2()
    lo, ll = coeffs.l1_loss(oracle_ext_fit, 2, xm), coeffs.l1_loss(lib_c, 2, xm)
    # both reach the same flat optimum of the L1 objective
    assert abs(ll - lo) <= 2e-3 * lo
    assert np.allclose(lib_c[:3], oracle_ext_fit[:3], rtol=0.02, atol=1e-3)


def test_monotone_over_the_range_and_practically_first_order(oracle_ext_fit):
    xm = coeffs.x_max_extended(T, math.sqrt(0.3))
    x = np.linspace(0.0, xm, 400001)
    for c in (_library_ext_f2(), list(oracle_ext_fit)):
        f = np.maximum(c[0] + c[1] * x + c[2] * x * x, 0.0)
        assert np.all(np.diff(f) <= 0.0), "rises again inside [0, x_max]"
    # the standard order-2 fit turns positive again well inside the range (hence Eq. 6's cut)
    from paper_2603_18707_amd import _lib as L
    std = list(L.gs_kernel_default(L.KERNEL_POLY, 2, L.RADIUS_POLY_OPACITY).coeffs)
    fs = np.maximum(std[0] + std[1] * x + std[2] * x * x, 0.0)
    assert np.any(np.diff(fs) > 0.0)
    # App. A: with 16-px tiles the wide-range f2 is all but the order-1 fit
    f1 = coeffs.fit(1, xm)
    assert coeffs.l1_loss(oracle_ext_fit, 2, xm) == pytest.approx(coeffs.l1_loss(f1, 1, xm), rel=0.01)
    assert abs(oracle_ext_fit[2]) < 1e-3 and abs(oracle_ext_fit[1] - f1[1]) < 0.01
