"""Pin of the reference gradient: autograd through ``oracle.grad`` (FP64 torch)
against central finite differences of the independent C reference.

Sub-problem: 64 splats, 32x32, SH degree 3. A parameter is compared only when
every discrete decision (rectangles, alpha skips, termination) is identical at
theta - h and theta + h, so the image is smooth in between.
"""
import numpy as np
import pytest
import torch

from oracle import core, grad
from paper_2603_18707_amd import scenes

PAPER_F1 = (0.773, -0.773 / 4.386, 0.0, 0.0)


def _cfg(golden, kind, order):
    if kind == core.KERNEL_EXP:
        return core.Cfg(kind=kind, radius_mode=core.RADIUS_SIGMA3)
    c = PAPER_F1 if order == 1 else tuple(golden[f"fit{order}"]["c"])
    return core.Cfg(kind=kind, order=order, coeffs=c, radius_mode=core.RADIUS_POLY_OPACITY)


def _as64(sc):
    return {k: np.asarray(getattr(sc, k), np.float64).copy() for k in ("means3d", "scales", "quats", "opacities", "sh")}


class _S:
    def __init__(self, d, deg):
        self.__dict__.update(d)
        self.sh_degree = deg


def _loss_c(params, deg, cam, cfg, w):
    r = core.render_image(_S(params, deg), cam, cfg, round_to=None)
    sig = (r["n_contrib"].tobytes(), r["n_eval"].tobytes(), r["last_contrib"].tobytes(),
           r["proj"]["rect"].tobytes())
    return float((r["image"] * w).sum()), sig


@pytest.mark.parametrize("kind,order,scale_mul", [(core.KERNEL_POLY, 1, 1.0), (core.KERNEL_POLY, 1, 4.0),
                                                  (core.KERNEL_EXP, 1, 4.0), (core.KERNEL_POLY, 2, 4.0),
                                                  (core.KERNEL_POLY, 3, 4.0)])
def test_autograd_matches_finite_differences(golden_coeffs, kind, order, scale_mul):
    sc, cam = scenes.workload_fd()
    sc.scales *= scale_mul
    cfg = _cfg(golden_coeffs, kind, order)
    p0 = _as64(sc)
    w = np.random.default_rng(9).normal(size=(3, cam.height, cam.width))

    tens = {k: torch.tensor(v, requires_grad=True) for k, v in p0.items()}
    img, _ = grad.render(tens["means3d"], tens["scales"], tens["quats"], tens["opacities"], tens["sh"],
                         sc.sh_degree, cam, cfg)
    L = (img * torch.as_tensor(w)).sum()
    L.backward()
    base, sig0 = _loss_c(p0, sc.sh_degree, cam, cfg, w)
    assert float(L.detach()) == pytest.approx(base, rel=1e-12, abs=1e-12)

    proj = core.project(_S(p0, sc.sh_degree), cam, cfg)
    live = np.nonzero(proj["tiles"] > 0)[0]
    rng = np.random.default_rng(1)
    pick = rng.choice(live, size=min(10, live.shape[0]), replace=False)
    checked = skipped = 0
    gmax = max(float(t.grad.abs().max()) for t in tens.values())
    for key in ("means3d", "scales", "quats", "opacities", "sh"):
        g_ad = tens[key].grad.numpy()
        for i in pick:
            for idx in np.ndindex(p0[key].shape[1:]):
                full = (i,) + idx
                th = p0[key][full]
                h = 1e-6 * max(1.0, abs(th))
                pp = {k: v.copy() for k, v in p0.items()}
                pp[key][full] = th + h
                lp, sp = _loss_c(pp, sc.sh_degree, cam, cfg, w)
                pp[key][full] = th - h
                lm, sm = _loss_c(pp, sc.sh_degree, cam, cfg, w)
                if sp != sig0 or sm != sig0:
                    skipped += 1
                    continue
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g_ad[full]) <= 1e-7 * gmax + 1e-5 * abs(fd), (key, full, fd, g_ad[full])
                checked += 1
    assert checked > 200 and skipped < 0.05 * (checked + skipped)
