"""Test-side glue: matching configurations for the GPU library and the oracle.

The coefficients given to both sides come from the paper (order 1) or from the
oracle's own fit (orders 2, 3, stored in tests/golden/kernel_coeffs.json); the
GPU library receives them as explicit inputs.
"""
import json
import os

import numpy as np

from oracle import core as ocore

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
with open(os.path.join(ROOT, "tests", "golden", "kernel_coeffs.json")) as _f:
    GOLDEN = json.load(_f)["sets"]

RADIUS = {"sigma3": 0, "universal": 1, "opacity": 2, "exp_opacity": 3}

# Width of the "too close to call in single precision" band around alpha = eps,
# per kernel: the fp32 rounding of the blender's alpha (a few ulp of the terms
# that cancel in it: o c_0 ~ 1 for polynomials, the exponent ~ 10 for exp).
ALPHA_BAND = {("exp", 1): 5e-8, ("poly", 1): 2e-6, ("poly", 2): 3e-6, ("poly", 3): 6e-6}


def coeffs_for(order):
    return tuple(GOLDEN["paper1"]["c"]) if order == 1 else tuple(GOLDEN[f"fit{order}"]["c"])


def oracle_cfg(kind, order, radius, **kw):
    return ocore.Cfg(kind=0 if kind == "exp" else 1, order=order, radius_mode=RADIUS[radius],
                     coeffs=coeffs_for(order), alpha_band=ALPHA_BAND[(kind, order if kind == "poly" else 1)], **kw)


def gpu_kernel(kind, order, radius):
    from paper_2603_18707_amd import render
    return render.kernel_spec(kind, order, radius, coeffs=coeffs_for(order))


def gpu_params(**kw):
    from paper_2603_18707_amd import _lib
    p = _lib.gs_params_default()
    for k, v in kw.items():
        if k == "bg":
            for i in range(3):
                p.bg[i] = v[i]
        else:
            setattr(p, k, v)
    return p


def edge_flagged_tiles(proj, gx, gy):
    """Tiles next to an edge of a splat the oracle flagged (edge on a tile boundary)."""
    bad = np.zeros((gy, gx), bool)
    for i in np.nonzero(proj["flags"] & ocore.SPLAT_EDGE_NEAR)[0]:
        u, v = proj["means2d"][i]
        r = proj["radius"][i]
        x0, x1 = int(np.floor((u - r) / 16)) - 1, int(np.floor((u + r) / 16)) + 1
        y0, y1 = int(np.floor((v - r) / 16)) - 1, int(np.floor((v + r) / 16)) + 1
        bad[max(0, y0):max(0, min(gy, y1 + 1)), max(0, x0):max(0, min(gx, x1 + 1))] = True
    return bad
