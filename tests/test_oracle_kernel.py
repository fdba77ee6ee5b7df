"""Pins of the reference's kernel support and anti-aliasing to the paper.

Eq. 2 / Eq. 6 (the kernel is exactly zero from its first root on) and Sec. 3.4
(Eqs. 7-9: the v-dilation plus the sqrt(|S'| / |S' + vI|) opacity factor keeps
the integrated contribution of a splat for any kernel).
"""
import math

import numpy as np
import pytest

from oracle import coeffs, core
from paper_2603_18707_amd import scenes

EPS = 1.0 / 255.0


def _cfg(golden, name, kind=core.KERNEL_POLY, **kw):
    g = golden[name]
    return core.Cfg(kind=kind, order=g["order"], coeffs=tuple(g["c"]), **kw)


@pytest.mark.parametrize("name", ["paper1", "fit1", "fit2", "fit3"])
def test_zero_beyond_first_root(golden_coeffs, name):
    cfg = _cfg(golden_coeffs, name)
    x0 = golden_coeffs[name]["x0"]
    Q = np.concatenate([x0 + np.linspace(0.0, 60.0, 6001), [x0 * (1 + 1e-12)]])
    assert np.all(core.kernel_value(cfg, Q) == 0.0)
    Qin = np.linspace(0.0, x0 * (1 - 1e-9), 2001)
    assert np.all(core.kernel_value(cfg, Qin) > 0.0)


def test_f2_cut_removes_second_lobe(golden_coeffs):
    # beyond the second root the parabola is positive; Eq. 6 still gives 0
    cfg = _cfg(golden_coeffs, "fit2")
    c = golden_coeffs["fit2"]["c"]
    x1 = max(np.roots([c[2], c[1], c[0]]).real)
    assert core.poly(c, 2, x1 + 5.0) > 0
    assert core.kernel_value(cfg, np.array([x1 + 5.0]))[0] == 0.0


@pytest.mark.parametrize("name", ["paper1", "fit2", "fit3"])
@pytest.mark.parametrize("o", [1.0, 0.5, 0.1, 0.02])
def test_opacity_radius_bounds_contribution(golden_coeffs, name, o):
    # beyond the opacity-dependent radius t^2, o k(Q) < eps; just inside it is >= eps
    g = golden_coeffs[name]
    cfg = _cfg(golden_coeffs, name)
    xr = core.first_root(g["c"], g["order"], EPS / o)
    if xr < 0:
        assert o * g["c"][0] < EPS
        return
    Q = xr + np.linspace(1e-9, 40.0, 4001)
    assert np.all(o * core.kernel_value(cfg, Q) < EPS)
    assert o * core.kernel_value(cfg, np.array([xr * (1 - 1e-9)]))[0] >= EPS


def _grid_integral(f, half, h):
    x = np.arange(-half, half + h / 2, h)
    X, Y = np.meshgrid(x, x)
    return f(X, Y).sum() * h * h


@pytest.mark.parametrize("name", ["exp", "paper1", "fit2", "fit3"])
def test_kernel_mass_closed_form(golden_coeffs, name):
    # integral over R^2 of k(y^T y) = pi * integral_0^inf k(s) ds
    if name == "exp":
        cfg, closed = core.Cfg(kind=core.KERNEL_EXP), 2.0 * math.pi
    else:
        cfg = _cfg(golden_coeffs, name)
        g = golden_coeffs[name]
        c, x0 = g["c"], g["x0"]
        closed = math.pi * sum(c[i] * x0 ** (i + 1) / (i + 1) for i in range(g["order"] + 1))
        if name == "paper1":
            assert closed == pytest.approx(math.pi * c[0] ** 2 / (2 * abs(c[1])), rel=1e-12)
    kq = lambda Q: core.kernel_value(cfg, Q)
    num = _grid_integral(lambda X, Y: kq(X * X + Y * Y), 7.0, 0.02)
    assert num == pytest.approx(closed, rel=2e-3)


def _one_splat_scene(scale, quat, opacity=0.8):
    return scenes.Scene(np.array([[0.05, -0.03, 4.0]], np.float32), np.array([scale], np.float32),
                        np.array([quat], np.float32), np.array([opacity], np.float32),
                        np.zeros((1, 1, 3), np.float32), 0)


@pytest.mark.parametrize("name", ["exp", "paper1", "fit2", "fit3"])
@pytest.mark.parametrize("shape", [((0.02, 0.05, 0.01), (0.9, 0.1, -0.3, 0.2)),
                                   ((0.006, 0.004, 0.02), (0.2, 0.7, 0.1, -0.6))])
def test_antialiasing_preserves_mass(golden_coeffs, name, shape):
    # Sec. 3.4: o' k(Q_{S'+vI}) integrates to the same value as o k(Q_{S'})
    cfg = core.Cfg(kind=core.KERNEL_EXP) if name == "exp" else _cfg(golden_coeffs, name)
    cfg.radius_mode = core.RADIUS_SIGMA3
    cam = scenes.tiny_camera(128, 128)
    sc = _one_splat_scene(*shape)
    masses = []
    for v in (0.0, 0.3, 2.0):
        cfg.aa_v = v
        p = core.project(sc, cam, cfg)
        a, b, c = p["conic"][0]
        o = p["opac"][0]
        kq = lambda Q: core.kernel_value(cfg, Q)
        sig = 1.0 / math.sqrt(min(np.linalg.eigvalsh([[a, b], [b, c]])))
        h = min(0.02, sig / 40.0)
        masses.append(o * _grid_integral(lambda X, Y: kq(a * X * X + 2 * b * X * Y + c * Y * Y), 6.0 * sig, h))
    assert masses[1] == pytest.approx(masses[0], rel=3e-3)
    assert masses[2] == pytest.approx(masses[0], rel=3e-3)
