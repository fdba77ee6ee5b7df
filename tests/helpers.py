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

# Allowed share of compared pixels that the oracle flags, per kernel: about
# twice the largest share measured on the test scenes with 1024 or more
# compared pixels (tiny frames at x1 and x2 scales, the 1M-splat frame, the
# 4M-splat heavy frames, the batched views). Dense scenes flag the most, and
# the cubic most of all: its alpha band is three times the linear one's (its
# Horner sum cancels terms up to ~4 near alpha = eps). Largest shares
# measured: exp 0.14%, poly-1 0.20%, poly-2 0.07%, poly-3 0.92% (the batch's
# 4500-splat scene at x2.5 scales; 0.46% of the 1M frame's samples).
# Flagged pixels are still checked, against the oracle's reach.
FLAG_RATE = {("exp", 1): 3e-3, ("poly", 1): 4e-3, ("poly", 2): 4e-3, ("poly", 3): 2e-2}


def flag_limit(kind, order, npix):
    return max(2.0, FLAG_RATE[(kind, order if kind == "poly" else 1)] * npix)


def coeffs_for(order):
    return tuple(GOLDEN["paper1"]["c"]) if order == 1 else tuple(GOLDEN[f"fit{order}"]["c"])


def oracle_cfg(kind, order, radius, **kw):
    """The oracle's configuration for a GPU comparison: the library takes its
    scalar parameters as float, so the oracle gets the same float values."""
    return ocore.Cfg(kind=0 if kind == "exp" else 1, order=order, radius_mode=RADIUS[radius],
                     coeffs=coeffs_for(order), alpha_band=ALPHA_BAND[(kind, order if kind == "poly" else 1)],
                     **kw).float_params()


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
    """Tiles next to an edge of a splat the oracle flagged (edge on a tile
    boundary): its rectangle (kept, clamped, for such splats) grown by one."""
    bad = np.zeros((gy, gx), bool)
    for i in np.nonzero(proj["flags"] & ocore.SPLAT_EDGE_NEAR)[0]:
        x0, y0, x1, y1 = (int(v) for v in proj["rect"][i])
        xa, xb = min(x0, x1) - 1, max(x0, x1) + 1
        ya, yb = min(y0, y1) - 1, max(y0, y1) + 1
        bad[max(0, ya):max(0, min(gy, yb + 1)), max(0, xa):max(0, min(gx, xb + 1))] = True
    return bad


def ulp_distance(a, b):
    """Floats between a and b (float32 arrays) plus one: 0 when equal."""
    ia = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    ib = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)  # order-preserving integer image of the floats
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    return np.abs(ia - ib)


# largest distance from the oracle's own float that an entry the oracle flags
# may take, in ulps of the entry (u, v, a, c, o') or of the conic's scale
# sqrt(a c) (b, which cancels when the footprint's axes lie near the image
# axes): the oracle's intervals span at most that many floats
# (test_bound_width_in_floats), thin footprints included
MAX_RECORD_ULPS = 2


def record_ulps(got, own, conic_scale):
    """Distance of record entries (columns u, v, a, b, c, o') from the
    oracle's floats in the units of MAX_RECORD_ULPS."""
    d = ulp_distance(got, own).astype(np.float64)
    db = np.abs(got[:, 3].astype(np.float64) - own[:, 3].astype(np.float64)) / np.spacing(
        np.asarray(conic_scale, np.float32)).astype(np.float64)
    d[:, 3] = db
    return d


def records_chosen_by(o, g_means2d, g_conic_opacity, live):
    """The float records the GPU projection chose among the correct ones.

    The oracle bounds the FP64 error of each record entry X (u, v, a, b, c,
    o') by E; any correct evaluation lies within 2 E of X, so its float lies
    between fl(X - 2 E) and fl(X + 2 E), rounding being monotone. Outside the
    entries the oracle flags as ambiguous that interval holds only the
    oracle's own float; inside, usually also one neighbour (the oracle's
    alternative), more where E is wide. Each entry of a live splat must lie
    in its interval, and within MAX_RECORD_ULPS ulps of the oracle's own
    float (b: of the conic's scale), else this fails. Returns the oracle's projection with
    the records set to those members of the oracle's intervals (held as
    float64) and the number of entries that are not the oracle's own float.
    """
    X = np.concatenate([o["means2d"], o["conic"], o["opac"][:, None]], axis=1)
    own = X.astype(np.float32)
    amb = ((o["rec_amb"][:, None].astype(np.int64) >> np.arange(6)) & 1).astype(bool)
    w = 2.0 * o["rec_err"]
    lo, hi = (X - w).astype(np.float32), (X + w).astype(np.float32)
    got = np.concatenate([g_means2d, g_conic_opacity[:, :3], g_conic_opacity[:, 3:4]], axis=1).astype(np.float32)
    same = got == own
    other = amb & (got >= lo) & (got <= hi) & ~same & live[:, None]
    bad = live[:, None] & ~(same | other)
    if bad.any():
        i, k = np.argwhere(bad)[0]
        raise AssertionError(f"{int(bad.sum())} record entries outside the oracle's interval of correct floats; "
                             f"first: splat {i} entry {'uvabco'[k]} gpu {got[i, k]!r} oracle {own[i, k]!r} "
                             f"interval [{lo[i, k]!r}, {hi[i, k]!r}] ambiguous {bool(amb[i, k])}")
    if other.any():
        d = record_ulps(got, own, np.sqrt(np.abs(X[:, 2] * X[:, 4])))[other]
        ulps = float(d.max())
        print(f"[proj] {int(other.sum())} record entries took another correct float, at most {ulps:.3g} ulp away")
        assert ulps <= MAX_RECORD_ULPS, f"a record entry {ulps} ulps from the oracle's float"
    chosen = np.where(other, got, own).astype(np.float64)
    rec = ocore.round_records(o)
    rec["means2d"], rec["conic"], rec["opac"] = chosen[:, 0:2].copy(), chosen[:, 2:5].copy(), chosen[:, 5].copy()
    return rec, int(other.sum())
