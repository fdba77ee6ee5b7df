"""Pins of the reference's kernel coefficients and radii to the paper.

Sec. 3.1 (printed f1 numbers), Sec. 3.2 Eqs. 3-5, Sec. 3.3 (shape of f2, f3)
and App. B (closed-form roots of f2, f3). None of these tests needs a GPU.
"""
import math

import numpy as np
import pytest

from oracle import coeffs, core

EPS = 1.0 / 255.0


def test_fit_range_is_two_ln_255():
    # Sec. 3.1: support of the truncated exponential is 0 <= x <= -2 ln(eps)
    assert coeffs.X_MAX == pytest.approx(2.0 * math.log(255.0), rel=1e-15)
    # 3DGS culls at 3.3 sigma: sqrt of that range
    assert round(math.sqrt(coeffs.X_MAX), 1) == 3.3


def test_paper_f1_printed_numbers():
    c = coeffs.PAPER_F1
    x0 = core.first_root(c, 1, 0.0)
    assert abs(x0 - 4.386) < 0.01                      # zero beyond x = 4.386
    assert abs(255.0 * math.exp(-0.5 * x0) - 28.45) < 0.1  # g culled at 28.45 / 255
    assert round(math.sqrt(x0), 1) == 2.1               # 2.1 sigma
    assert core.poly(c, 1, 0.0) < 1.0                   # peak opacity below one


def test_golden_fit1_near_printed_pair(golden_coeffs):
    c = golden_coeffs["fit1"]["c"]
    assert abs(c[0] - 0.773) < 0.005 and abs(c[1] + 0.176) < 0.005
    # the fitted pair is at least as good as the printed pair on the same objective
    assert coeffs.l1_loss(c, 1) <= coeffs.l1_loss(coeffs.PAPER_F1, 1) + 1e-12
    # and the two kernels differ little in the L1 sense: the optimum is flat
    assert coeffs.l1_loss(coeffs.PAPER_F1, 1) / coeffs.l1_loss(c, 1) - 1.0 < 1e-3


def test_fit1_rederives_golden(golden_coeffs):
    c = coeffs.fit(1)
    assert np.allclose(c, golden_coeffs["fit1"]["c"], atol=1e-6)


def test_fit_objective_prefers_fit_over_perturbations(golden_coeffs):
    # a local-optimality check of each stored fit: small perturbations of any
    # coefficient never lower the L1 objective
    for name in ("fit1", "fit2", "fit3"):
        g = golden_coeffs[name]
        c0 = np.array(g["c"])
        base = coeffs.l1_loss(c0, g["order"], m=40001)
        for i in range(g["order"] + 1):
            for s in (-1.0, 1.0):
                c = c0.copy()
                c[i] += s * 1e-3 * max(abs(c0[i]), 1e-3)
                assert coeffs.l1_loss(c, g["order"], m=40001) >= base - 1e-9


def test_higher_orders_better_fit(golden_coeffs):
    l = [golden_coeffs[f"fit{n}"]["l1"] for n in (1, 2, 3)]
    assert l[0] > l[1] > l[2]


def test_f2_parabola_turns_positive_again(golden_coeffs):
    # Sec. 3.3: the fitted quadratic is not monotone and rises above zero again
    c = golden_coeffs["fit2"]["c"]
    assert c[2] > 0
    roots = np.sort(np.roots([c[2], c[1], c[0]]).real)
    assert 0 < roots[0] < roots[1]
    assert roots[0] == pytest.approx(golden_coeffs["fit2"]["x0"], rel=1e-9)
    assert core.poly(c, 2, roots[1] + 1.0) > 0


def test_f3_monotone_single_real_root(golden_coeffs):
    # Sec. 3.3: the cubic fit is strictly monotone with a single real root
    c = golden_coeffs["fit3"]["c"]
    # p'(x) = c1 + 2 c2 x + 3 c3 x^2 has no real root
    assert (2 * c[2]) ** 2 - 4 * (3 * c[3]) * c[1] < 0
    r = np.roots([c[3], c[2], c[1], c[0]])
    real = r[np.abs(r.imag) < 1e-9].real
    assert real.shape[0] == 1 and real[0] > 0
    assert real[0] == pytest.approx(golden_coeffs["fit3"]["x0"], rel=1e-9)


def test_stored_roots_match_bisection(golden_coeffs):
    for g in golden_coeffs.values():
        assert core.first_root(g["c"], g["order"], 0.0) == pytest.approx(g["x0"], rel=1e-14)


# --- radii: Eq. 3, 4, 5 and App. B against bisection ----------------------

OPACITIES = (1.0, 0.9, 0.5, 0.1, 0.02, 0.01, 0.006)


def test_eq5_universal_f1():
    c = coeffs.PAPER_F1
    t_closed = math.sqrt(-c[0] / c[1])
    assert math.sqrt(core.first_root(c, 1, 0.0)) == pytest.approx(t_closed, rel=1e-13)


@pytest.mark.parametrize("o", OPACITIES)
def test_eq4_opacity_f1(o):
    c = coeffs.PAPER_F1
    xr = core.first_root(c, 1, EPS / o)
    if o * c[0] < EPS:
        assert xr < 0  # the whole splat is below eps: culled
        return
    t_closed = math.sqrt((EPS - o * c[0]) / (o * c[1]))
    assert math.sqrt(xr) == pytest.approx(t_closed, rel=1e-12)
    # the opacity bound is tighter than the universal one
    assert xr <= core.first_root(c, 1, 0.0)


@pytest.mark.parametrize("o", OPACITIES)
def test_eq3_exp_opacity(o):
    # t_g is the Mahalanobis radius where o exp(-x/2) reaches eps
    if o < EPS:
        return
    t = math.sqrt(2.0 * math.log(o / EPS))
    cfg = core.Cfg(kind=core.KERNEL_EXP)
    assert o * core.kernel_value(cfg, np.array([t * t]))[0] == pytest.approx(EPS, rel=1e-12)


@pytest.mark.parametrize("o", OPACITIES + (0.0,))
def test_appb_quadratic(golden_coeffs, o):
    c = golden_coeffs["fit2"]["c"]
    eps = EPS if o > 0 else 0.0          # eps = 0 gives the universal bound
    cc = c[0] - (eps / o if o > 0 else 0.0)
    xr = core.first_root(c, 2, eps / o if o > 0 else 0.0)
    if cc < 0:
        assert xr < 0
        return
    t_closed = (-c[1] - math.sqrt(c[1] ** 2 - 4.0 * cc * c[2])) / (2.0 * c[2])
    assert xr == pytest.approx(t_closed, rel=1e-11)


@pytest.mark.parametrize("o", OPACITIES + (0.0,))
def test_appb_cubic_cardano(golden_coeffs, o):
    c = golden_coeffs["fit3"]["c"]
    eps = EPS if o > 0 else 0.0
    cc = c[0] - (eps / o if o > 0 else 0.0)
    xr = core.first_root(c, 3, eps / o if o > 0 else 0.0)
    if cc < 0:
        assert xr < 0
        return
    d0 = c[2] ** 2 - 3.0 * c[3] * c[1]
    d1 = 2.0 * c[2] ** 3 - 9.0 * c[3] * c[2] * c[1] + 27.0 * c[3] ** 2 * cc
    s = math.sqrt(d1 * d1 - 4.0 * d0 ** 3)      # real: the cubic has one real root
    C = np.cbrt((d1 + s) / 2.0)
    t_closed = -(c[2] + C + d0 / C) / (3.0 * c[3])
    assert xr == pytest.approx(t_closed, rel=1e-9)


def test_higher_order_radii_between_f1_and_3sigma(golden_coeffs):
    # the universal radii grow with the order but stay below 3DGS's 3.3 sigma
    r = [math.sqrt(golden_coeffs[f"fit{n}"]["x0"]) for n in (1, 2, 3)]
    assert r[0] < r[1] < r[2] < math.sqrt(coeffs.X_MAX)
