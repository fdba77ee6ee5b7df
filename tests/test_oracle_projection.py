"""Pins of the reference projection: EWA, SH colour, depth and culling.

The projection is the 3DGS formulation the paper builds on (Sec. 2, Eq. 1):
EWA splatting with the Jacobian of the perspective map, real spherical
harmonics for colour. These checks use textbook facts, not the oracle's own
formulas: finite differences of the perspective map, Monte-Carlo projection
of a small 3D Gaussian, SciPy's quaternion rotation, and SH orthonormality.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import core
from paper_2603_18707_amd import scenes


def _scene1(mean, scale, quat, opacity=0.7, sh=None, deg=0):
    nb = (deg + 1) ** 2
    sh = np.zeros((1, nb, 3), np.float32) if sh is None else np.asarray(sh, np.float32).reshape(1, nb, 3)
    return scenes.Scene(np.array([mean], np.float32), np.array([scale], np.float32), np.array([quat], np.float32),
                        np.array([opacity], np.float32), sh, deg)


def _cov2d(p):
    a, b, c = p["conic"][0]
    return np.linalg.inv(np.array([[a, b], [b, c]]))


def _camera():
    return scenes.pinhole(320, 240, 55.0, scenes.look_at((1.0, -2.0, -6.0), (0.2, 0.1, 0.3)))


@pytest.mark.parametrize("seed", range(5))
def test_ewa_matches_finite_difference_jacobian(seed):
    rng = np.random.default_rng(seed)
    cam = _camera()
    mean = rng.uniform(-0.5, 0.5, 3) + np.array([0.2, 0.1, 0.3])
    scale = np.exp(rng.normal(-3, 0.5, 3))
    quat = rng.normal(size=4)
    sc = _scene1(mean, scale, quat)
    cfg = core.Cfg(kind=core.KERNEL_EXP, radius_mode=core.RADIUS_SIGMA3, aa_v=0.0)
    S2 = _cov2d(core.project(sc, cam, cfg))
    # covariance from scipy's rotation (scalar-last quaternion) and FD Jacobian
    m = sc.means3d[0].astype(np.float64)
    q = sc.quats[0].astype(np.float64)
    Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    Sig = Rq @ np.diag(sc.scales[0].astype(np.float64) ** 2) @ Rq.T
    V = cam.viewmat.astype(np.float64)

    def pix(x):
        t = V[:3, :3] @ x + V[:3, 3]
        return np.array([cam.fx * t[0] / t[2] + cam.cx, cam.fy * t[1] / t[2] + cam.cy])

    h = 1e-6
    J = np.stack([(pix(m + h * e) - pix(m - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
    ref = J @ Sig @ J.T
    assert np.allclose(S2, ref, rtol=1e-6, atol=1e-9 * np.abs(ref).max())


def test_ewa_monte_carlo_small_splat():
    rng = np.random.default_rng(7)
    cam = scenes.pinhole(640, 480, 60.0)
    mean = np.array([0.3, -0.2, 8.0])
    sc = _scene1(mean, (0.01, 0.03, 0.005), (0.8, 0.3, -0.4, 0.2))
    cfg = core.Cfg(kind=core.KERNEL_EXP, radius_mode=core.RADIUS_SIGMA3, aa_v=0.0)
    p = core.project(sc, cam, cfg)
    S2 = _cov2d(p)
    q = sc.quats[0].astype(np.float64)
    Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    Sig = Rq @ np.diag(sc.scales[0].astype(np.float64) ** 2) @ Rq.T
    X = rng.multivariate_normal(sc.means3d[0].astype(np.float64), Sig, size=400000)
    u = cam.fx * X[:, 0] / X[:, 2] + cam.cx
    v = cam.fy * X[:, 1] / X[:, 2] + cam.cy
    C = np.cov(np.stack([u, v]))
    assert np.allclose(C, S2, rtol=0.02, atol=0.02 * np.abs(S2).max())
    assert p["means2d"][0] == pytest.approx([u.mean(), v.mean()], abs=0.01)


def test_sh_orthonormal():
    # Gauss-Legendre in cos(theta) x uniform phi integrates degree <= 6 exactly
    xg, wg = np.polynomial.legendre.leggauss(16)
    nphi = 32
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (np.repeat(wg, nphi) * (2 * math.pi / nphi))
    Y = core.sh_basis(3, dirs)
    G = (Y * w[:, None]).T @ Y
    assert np.allclose(G, np.eye(16), atol=1e-12)


def test_sh_degree1_is_linear_in_direction():
    # band 1 spans the coordinate functions: each Y_1m is +-sqrt(3/4pi) times x, y or z
    d = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
    Y = core.sh_basis(1, d)[:, 1:]
    k = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(np.abs(Y), k * np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]]))


def test_sh_degree0_colour():
    cam = scenes.pinhole(64, 64, 60.0)
    dc = np.array([0.4, -1.2, 2.0])
    sc = _scene1((0.0, 0.0, 3.0), (0.05, 0.05, 0.05), (1, 0, 0, 0), sh=dc)
    p = core.project(sc, cam, core.Cfg(kind=core.KERNEL_EXP, radius_mode=core.RADIUS_SIGMA3))
    ref = np.maximum(dc / (2 * math.sqrt(math.pi)) + 0.5, 0.0)
    assert np.allclose(p["rgb"][0], ref, atol=1e-7)  # inputs are float32


def test_depth_near_cull_and_rect():
    cam = scenes.pinhole(64, 48, 60.0)
    pts = [(0.0, 0.0, 0.1), (0.0, 0.0, 0.2), (0.0, 0.0, 3.0), (40.0, 0.0, 3.0)]
    sc = scenes.Scene(np.array(pts, np.float32), np.full((4, 3), 0.05, np.float32),
                      np.tile(np.array([1, 0, 0, 0], np.float32), (4, 1)), np.full(4, 0.9, np.float32),
                      np.zeros((4, 1, 3), np.float32), 0)
    cfg = core.Cfg(kind=core.KERNEL_EXP, radius_mode=core.RADIUS_SIGMA3)
    p = core.project(sc, cam, cfg)
    assert p["depth32"].dtype == np.float32
    assert np.array_equal(p["depth32"], np.array([0.1, 0.2, 3.0, 3.0], np.float32))
    assert p["tiles"][0] == 0 and list(p["rect"][0]) == [0, 0, -1, -1]   # behind the near plane
    assert p["tiles"][1] > 0                                              # exactly at it: kept
    assert p["tiles"][2] > 0
    assert p["tiles"][3] == 0 and list(p["rect"][3]) == [0, 0, -1, -1]   # off screen
    # rectangle = tiles overlapped by the square of half-width r around the mean
    u, v = p["means2d"][2]
    r = p["radius"][2]
    assert list(p["rect"][2]) == [max(0, math.floor((u - r) / 16)), max(0, math.floor((v - r) / 16)),
                                  min(3, math.floor((u + r) / 16)), min(2, math.floor((v + r) / 16))]
    assert p["tiles"][2] == (p["rect"][2][2] - p["rect"][2][0] + 1) * (p["rect"][2][3] - p["rect"][2][1] + 1)


def test_radius_uses_largest_eigenvalue():
    cam = _camera()
    sc = _scene1((0.2, 0.1, 0.3), (0.02, 0.08, 0.01), (0.3, -0.5, 0.7, 0.1))
    for mode, k in ((core.RADIUS_SIGMA3, 3.0),):
        cfg = core.Cfg(kind=core.KERNEL_EXP, radius_mode=mode)
        p = core.project(sc, cam, cfg)
        lmax = np.linalg.eigvalsh(_cov2d(p)).max()
        assert p["radius"][0] == pytest.approx(k * math.sqrt(lmax) * cfg.radius_pad, rel=1e-12)


def test_sh_ordering_and_signs_against_complex_harmonics():
    """The basis against the textbook definition built from SciPy's complex
    spherical harmonics (Condon-Shortley phase included): band l, order
    m = -l..l, real Y_lm = sqrt(2) Im Y_l^|m| for m < 0, Y_l^0 for m = 0,
    sqrt(2) Re Y_l^m for m > 0. This fixes the ordering and every sign of the
    colour basis independently of the closed forms the reference writes."""
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(8)
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    polar, azim = np.arccos(d[:, 2]), np.arctan2(d[:, 1], d[:, 0])
    cols = []
    for l in range(4):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), polar, azim)
            cols.append(math.sqrt(2) * c.imag if m < 0 else (c.real if m == 0 else math.sqrt(2) * c.real))
    ref = np.stack(cols, 1)
    Y = core.sh_basis(3, d)
    assert np.allclose(Y, ref, atol=1e-12)
