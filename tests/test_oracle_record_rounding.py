"""Pins of the reference's record-rounding analysis: the running FP64 error
bound E on each float record entry (u, v, a, b, c, o) and the ambiguity bits
and alternative roundings derived from it.

An extended-precision projection (numpy longdouble, a 64-bit significand on
x86) written here from the same formulas stands in for the exact record. The
oracle's FP64 record must lie within E of it; wherever the float of the
extended value differs from the float of the FP64 value, the entry must be
flagged ambiguous with the extended value's float as its alternative. Thin
footprints of a heavy-tailed scene supply cases with cancelling
determinants (condition up to ~1e6).
"""
import math

import numpy as np
import pytest

from oracle import core
from paper_2603_18707_amd import scenes
from tests import helpers as H

LD = np.longdouble


def _extended_records(scene, cam, sel, aa_v):
    """u, v, a, b, c, o of the splats sel in long double: world to camera,
    R(q) diag(s^2) R(q)^T, the clamped perspective Jacobian, J W Sigma W^T J^T,
    the anti-aliasing term and the inverse."""
    V = np.asarray(cam.viewmat, dtype=LD)
    R, t = V[:3, :3], V[:3, 3]
    m = scene.means3d[sel].astype(LD)
    tc = m @ R.T + t
    q = scene.quats[sel].astype(LD)
    q = q / np.sqrt((q * q).sum(axis=1, keepdims=True))
    w, x, y, z = q.T
    Rq = np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                   np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
                   np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], 1)
    s2 = scene.scales[sel].astype(LD) ** 2
    Sig = np.einsum("nik,nk,njk->nij", Rq, s2, Rq)
    fx, fy, cx, cy = LD(cam.fx), LD(cam.fy), LD(cam.cx), LD(cam.cy)
    tz = tc[:, 2]
    limx = LD(1.3) * (LD(cam.width) / (LD(2) * fx))
    limy = LD(1.3) * (LD(cam.height) / (LD(2) * fy))
    txz = np.clip(tc[:, 0] / tz, -limx, limx)
    tyz = np.clip(tc[:, 1] / tz, -limy, limy)
    zero = np.zeros_like(tz)
    J = np.stack([np.stack([fx / tz, zero, -fx * txz / tz], -1), np.stack([zero, fy / tz, -fy * tyz / tz], -1)], 1)
    TW = J @ R
    S2 = TW @ Sig @ np.swapaxes(TW, 1, 2)
    sxy = LD(0.5) * (S2[:, 0, 1] + S2[:, 1, 0])
    det0 = S2[:, 0, 0] * S2[:, 1, 1] - sxy * sxy
    A00, A11 = S2[:, 0, 0] + LD(aa_v), S2[:, 1, 1] + LD(aa_v)
    deta = A00 * A11 - sxy * sxy
    o = scene.opacities[sel].astype(LD) * np.sqrt(np.maximum(det0 / deta, LD(0)))
    u = fx * tc[:, 0] / tz + cx
    v = fy * tc[:, 1] / tz + cy
    return np.stack([u, v, A11 / deta, -sxy / deta, A00 / deta, o], 1)


@pytest.mark.parametrize("view", [0, 3])
def test_error_bound_and_ambiguity_against_extended_precision(view):
    scene, _ = scenes.workload_heavy(n=200_000)
    cam = scenes.orbit_camera(1920, 1080, 2.0 * math.pi * view / 8)
    cfg = H.oracle_cfg("poly", 1, "opacity")
    p = core.project(scene, cam, cfg)
    sel = np.nonzero(p["tiles"] > 0)[0]
    X = np.concatenate([p["means2d"], p["conic"], p["opac"][:, None]], 1)[sel]
    Xe = _extended_records(scene, cam, sel, aa_v=cfg.aa_v)
    E = p["rec_err"][sel]
    # the bound holds (the extended value's own error is ~2^-11 of FP64's)
    err = np.abs(X.astype(LD) - Xe).astype(np.float64)
    assert np.all(err <= E), f"bound exceeded {np.max(err / np.maximum(E, 1e-300)):.3g}x"
    # and is not vacuous: within a few thousand of the error actually made, on the conic
    hot = err[:, 2:5] > 1e-14 * np.abs(X[:, 2:5])
    assert np.median(E[:, 2:5][hot] / err[:, 2:5][hot]) < 5e3
    # every entry whose correct float differs from the FP64 value's float is flagged, with that float
    f64 = X.astype(np.float32)
    fex = Xe.astype(np.float64).astype(np.float32)
    amb = ((p["rec_amb"][sel][:, None].astype(np.int64) >> np.arange(6)) & 1).astype(bool)
    differ = f64 != fex
    assert np.all(amb[differ])
    assert np.all(p["rec_alt"][sel][differ].astype(np.float32) == fex[differ])
    # every entry whose exact value lies within E of a float rounding midpoint
    # (so that some evaluation within the bound rounds it either way) is flagged
    fe = Xe.astype(np.float64).astype(np.float32)
    up = np.nextafter(fe, np.float32(np.inf)).astype(LD)
    dn = np.nextafter(fe, np.float32(-np.inf)).astype(LD)
    mid_d = np.minimum(np.abs(Xe - (fe.astype(LD) + up) / 2), np.abs(Xe - (fe.astype(LD) + dn) / 2))
    near = mid_d.astype(np.float64) < E
    assert near.sum() > 20
    assert np.all(amb[near])
    # the alternative of an ambiguous entry is a neighbouring float; elsewhere the entry's own float
    alt = p["rec_alt"][sel].astype(np.float32)
    assert np.all(alt[~amb] == f64[~amb])
    gap = np.abs(alt[amb].astype(np.float64) - f64[amb].astype(np.float64))
    assert np.all(gap > 0) and np.all(gap <= np.abs(np.spacing(f64[amb])).astype(np.float64))
    # thin footprints make a small fraction of conic entries ambiguous; means almost never
    rate = amb.mean(axis=0)
    assert rate[2:5].max() < 0.01 and rate[0:2].max() < 1e-3


def test_ordinary_scene_is_rarely_ambiguous():
    scene, cam = scenes.workload_tiny()
    p = core.project(scene, cam, H.oracle_cfg("poly", 1, "opacity"))
    vis = p["tiles"] > 0
    amb = ((p["rec_amb"][vis][:, None].astype(np.int64) >> np.arange(6)) & 1).astype(bool)
    assert amb.mean() < 1e-3
    culled = p["tiles"] == 0
    assert np.all(p["rec_amb"][culled] == 0) and np.all(p["rec_err"][culled] == 0.0)


def test_records_chosen_by_accepts_only_the_oracles_roundings():
    """The test-side selector takes the oracle's floats, or for an ambiguous
    entry another float within its bound, and rejects anything else
    (planted on the CPU)."""
    scene, _ = scenes.workload_heavy(n=20_000)
    cam = scenes.orbit_camera(1920, 1080, 0.0)
    p = core.project(scene, cam, H.oracle_cfg("poly", 1, "opacity"))
    live = p["tiles"] > 0
    gm = p["means2d"].astype(np.float32)
    gco = np.concatenate([p["conic"], p["opac"][:, None]], 1).astype(np.float32)
    rec, nalt = H.records_chosen_by(p, gm, gco, live)
    assert nalt == 0 and np.array_equal(rec["conic"], p["conic"].astype(np.float32).astype(np.float64))
    amb = np.nonzero(live & ((p["rec_amb"] >> 2) & 1).astype(bool))[0]
    assert amb.size > 0
    i = amb[0]
    gco2 = gco.copy()
    gco2[i, 0] = np.float32(p["rec_alt"][i, 2])
    rec, nalt = H.records_chosen_by(p, gm, gco2, live)
    assert nalt == 1 and rec["conic"][i, 0] == p["rec_alt"][i, 2]
    # one ulp off on an entry that is not ambiguous
    j = np.nonzero(live & (p["rec_amb"] == 0))[0][0]
    gco3 = gco.copy()
    gco3[j, 2] = np.nextafter(gco3[j, 2], np.float32(np.inf))
    with pytest.raises(AssertionError):
        H.records_chosen_by(p, gm, gco3, live)
