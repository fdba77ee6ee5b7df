"""ctypes binding of the FP64 brute-force reference renderer (``oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Pins (tests/test_oracle_*.py, all run without a GPU):
  * kernel roots and radii: closed forms of Eq. 3, Eq. 4, Eq. 5 and App. B
    against the bisection used here; the printed f1 root 4.386, 28.45/255 and
    2.1 sigma / 3.3 sigma of Sec. 3.1;
  * kernel support: f_N is exactly zero from its first root on (Eq. 2, Eq. 6);
  * anti-aliasing: the integrated contribution of a splat is unchanged by the
    v-dilation plus opacity scaling for every kernel (Sec. 3.4, Eqs. 7-9);
  * EWA projection: Jacobian against finite differences of the perspective
    map, projected covariance against Monte-Carlo samples of a small splat;
  * spherical harmonics: orthonormality by quadrature on the sphere;
  * compositing: one splat gives alpha * rgb, two splats the over operator,
    white splats give 1 - T exactly, T is non-increasing, and a pure-Python
    per-pixel loop agrees on tiny scenes.
"""
import ctypes
import os
from dataclasses import dataclass, field, replace

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")

KERNEL_EXP, KERNEL_POLY = 0, 1
RECT_SQUARE, RECT_ELLIPSE_BOX = 0, 1
RADIUS_SIGMA3, RADIUS_POLY_UNIVERSAL, RADIUS_POLY_OPACITY, RADIUS_EXP_OPACITY = 0, 1, 2, 3

SPLAT_EDGE_NEAR, SPLAT_CULL_NEAR = 1, 2
PIX_ALPHA_NEAR, PIX_T_NEAR, PIX_EDGE_NEAR, PIX_CULL_NEAR = 1, 2, 4, 8


class _Cfg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("order", ctypes.c_int32), ("radius_mode", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("c", ctypes.c_double * 4), ("eps", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("t_min", ctypes.c_double), ("aa_v", ctypes.c_double),
                ("near_z", ctypes.c_double), ("radius_pad", ctypes.c_double), ("bg", ctypes.c_double * 3),
                ("alpha_band", ctypes.c_double), ("t_band_rel", ctypes.c_double), ("rect_mode", ctypes.c_int32),
                ("tile_cull", ctypes.c_int32)]


class _Cam(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


@dataclass
class Cfg:
    """Rendering configuration of the reference.

    Defaults follow the tiny-scene workload: eps = 1/255 (Sec. 3.1), alpha clamp
    0.99, early termination at T < 1e-4, 16x16 tiles, anti-aliasing variance
    0.3 px^2 (the paper does not give v), near plane 0.2, and a radius padded
    by 2^-20 so every rectangle is conservative.
    """
    kind: int = KERNEL_POLY
    order: int = 1
    radius_mode: int = RADIUS_POLY_OPACITY
    coeffs: tuple = (0.0, 0.0, 0.0, 0.0)
    eps: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    aa_v: float = 0.3
    near_z: float = 0.2
    radius_pad: float = 1.0 + 2.0 ** -20
    tile: int = 16
    bg: tuple = (0.0, 0.0, 0.0)
    # widths of the "too close to call in single precision" bands
    alpha_band: float = 2e-6
    t_band_rel: float = 1e-4
    # tile rectangle: 0 = bounding square of radius r (Sec. 2.1), 1 = the
    # ellipse Q = k^2's axis-aligned bounding box
    rect_mode: int = 0
    # 1: a splat is in a tile's list only when the tile passes the per-tile
    # test of the renderer's culled binning (orc_tile_keep)
    tile_cull: int = 0

    def float_params(self) -> "Cfg":
        """A copy whose scalar parameters (eps, alpha_max, t_min, aa_v, near_z,
        radius_pad, bg) are rounded to float: a renderer that takes them as
        float computes with those values, and so must the reference it is
        compared with (0.3 as a float is 0.3 + 1.2e-8, enough to move
        conic floats by an ulp)."""
        f = lambda x: float(np.float32(x))
        return replace(self, eps=f(self.eps), alpha_max=f(self.alpha_max), t_min=f(self.t_min), aa_v=f(self.aa_v),
                       near_z=f(self.near_z), radius_pad=f(self.radius_pad), bg=tuple(f(b) for b in self.bg))

    def _c(self) -> _Cfg:
        c = _Cfg()
        c.kind, c.order, c.radius_mode, c.tile = self.kind, self.order, self.radius_mode, self.tile
        cc = list(self.coeffs) + [0.0] * (4 - len(self.coeffs))
        for i in range(4):
            c.c[i] = float(cc[i])
        c.eps, c.alpha_max, c.t_min, c.aa_v = self.eps, self.alpha_max, self.t_min, self.aa_v
        c.near_z, c.radius_pad = self.near_z, self.radius_pad
        for i in range(3):
            c.bg[i] = float(self.bg[i])
        c.alpha_band, c.t_band_rel, c.rect_mode = self.alpha_band, self.t_band_rel, self.rect_mode
        c.tile_cull = int(self.tile_cull)
        return c


def _cam(cam) -> _Cam:
    """Accepts any camera object with viewmat (4x4 world->camera, row-major),
    fx, fy, cx, cy, width, height."""
    c = _Cam()
    vm = np.asarray(cam.viewmat, dtype=np.float64)
    for r in range(3):
        for k in range(3):
            c.R[3 * r + k] = vm[r, k]
        c.t[r] = vm[r, 3]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.orc_poly.restype = ctypes.c_double
        L.orc_poly.argtypes = [P, ctypes.c_int, ctypes.c_double]
        L.orc_first_root.restype = ctypes.c_double
        L.orc_first_root.argtypes = [P, ctypes.c_int, ctypes.c_double]
        L.orc_kernel.restype = ctypes.c_double
        L.orc_kernel.argtypes = [P, ctypes.c_double, ctypes.c_double]
        L.orc_kernel_many.restype = None
        L.orc_kernel_many.argtypes = [P, ctypes.c_int64, P, P]
        L.orc_sh_basis.restype = None
        L.orc_sh_basis.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
        L.orc_project.restype = None
        L.orc_project.argtypes = [P, P, ctypes.c_int64] + [P] * 5 + [ctypes.c_int32] + [P] * 13
        L.orc_depth_order.restype = None
        L.orc_depth_order.argtypes = [ctypes.c_int64, P, P]
        L.orc_render_pixels.restype = None
        L.orc_render_pixels.argtypes = [P, ctypes.c_int64, P, P, P, P, P, P, P, ctypes.c_int64] + [P] * 8
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_cull_cut.restype = ctypes.c_double
        L.orc_cull_cut.argtypes = [P] + [ctypes.c_double] * 4
        L.orc_rect_min_q.restype = ctypes.c_double
        L.orc_rect_min_q.argtypes = [ctypes.c_double] * 7
        L.orc_tile_keep.restype = ctypes.c_int
        L.orc_tile_keep.argtypes = [ctypes.c_double] * 6 + [ctypes.c_int] * 3 + [P]
        L.orc_cull_cuts.restype = None
        L.orc_cull_cuts.argtypes = [P, ctypes.c_int64, P, P, P]
        L.orc_cull_histogram.restype = None
        L.orc_cull_histogram.argtypes = [P, ctypes.c_int64, P, P, P, P, ctypes.c_int, ctypes.c_int, P, P]
        L.orc_cull_tile_members.restype = None
        L.orc_cull_copy_mask.restype = ctypes.c_int64
        L.orc_cull_copy_mask.argtypes = [P, ctypes.c_int64, P, P, P, P, P, P]
        L.orc_cull_tile_members.argtypes = [P, ctypes.c_int64, P, P, P, P, ctypes.c_int, ctypes.c_int, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def poly(coeffs, order, x) -> float:
    c = np.zeros(4, np.float64)
    c[: len(coeffs)] = coeffs
    return float(lib().orc_poly(_p(c), int(order), float(x)))


def first_root(coeffs, order, target=0.0) -> float:
    """Smallest x >= 0 with p(x) = target, by scan + bisection; -1 if none."""
    c = np.zeros(4, np.float64)
    c[: len(coeffs)] = coeffs
    return float(lib().orc_first_root(_p(c), int(order), float(target)))


def kernel_value(cfg: Cfg, Q) -> np.ndarray:
    """k(Q) for an array of quadric values (Eq. 2; Eq. 6 for order 2; exp otherwise)."""
    cc = cfg._c()
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    out = np.empty_like(Q)
    lib().orc_kernel_many(ctypes.byref(cc), int(Q.size), _p(Q), _p(out))
    return out


def sh_basis(deg: int, dirs: np.ndarray) -> np.ndarray:
    """Real SH basis values [m, (deg+1)^2] at unit directions dirs [m, 3]."""
    L = lib()
    dirs = np.asarray(dirs, dtype=np.float64)
    nb = (deg + 1) ** 2
    out = np.zeros((dirs.shape[0], 16), np.float64)
    for i in range(dirs.shape[0]):
        row = np.zeros(16, np.float64)
        L.orc_sh_basis(int(deg), float(dirs[i, 0]), float(dirs[i, 1]), float(dirs[i, 2]), _p(row))
        out[i] = row
    return out[:, :nb]


def project(scene, cam, cfg: Cfg) -> dict:
    """FP64 projection of every splat (see ``orc_project`` in oracle.c).

    ``scene`` needs means3d [n,3], scales [n,3], quats [n,4] (w,x,y,z),
    opacities [n], sh [n,(d+1)^2,3] and sh_degree; arrays are read as float64
    (float32 scenes convert exactly, finite differences may pass float64).
    Besides the record: rec_err [n,6], a running bound on the FP64 error of
    (u, v, a, b, c, o), and rec_amb [n], bit k set when entry k has a float
    rounding midpoint within twice that bound (two correct evaluations may
    round it one ulp apart), and rec_alt [n,6], the float on the other side
    of that midpoint (both are correct roundings).
    """
    L = lib()
    n = int(scene.means3d.shape[0])
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    m3, sc, qu, op, sh = (f64(scene.means3d), f64(scene.scales), f64(scene.quats),
                          f64(scene.opacities), f64(scene.sh))
    out = dict(means2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), opac=np.zeros(n), rgb=np.zeros((n, 3)),
               depth=np.zeros(n), depth32=np.zeros(n, np.float32), radius=np.zeros(n),
               rect=np.zeros((n, 4), np.int32), tiles=np.zeros(n, np.int64), flags=np.zeros(n, np.uint8),
               rec_amb=np.zeros(n, np.uint8), rec_err=np.zeros((n, 6)), rec_alt=np.zeros((n, 6)))
    cc, cm = cfg._c(), _cam(cam)
    L.orc_project(ctypes.byref(cc), ctypes.byref(cm), n, _p(m3), _p(sc), _p(qu), _p(op), _p(sh),
                  int(scene.sh_degree), _p(out["means2d"]), _p(out["conic"]), _p(out["opac"]),
                  _p(out["rgb"]), _p(out["depth"]), _p(out["depth32"]), _p(out["radius"]),
                  _p(out["rect"]), _p(out["tiles"]), _p(out["flags"]), _p(out["rec_amb"]), _p(out["rec_err"]),
                  _p(out["rec_alt"]))
    return out


def depth_order(depth32: np.ndarray) -> np.ndarray:
    """Compositing order: ascending float32 depth, ties by splat index."""
    d = np.ascontiguousarray(depth32, dtype=np.float32)
    o = np.zeros(d.shape[0], np.int64)
    lib().orc_depth_order(int(d.shape[0]), _p(d), _p(o))
    return o


def round_records(proj: dict, dtype=np.float32) -> dict:
    """The projected record as the rasterizer consumes it: the boundary between
    projection and blending carries single-precision means, conic, opacity
    and colour. Returns a copy with those fields rounded to ``dtype``."""
    r = dict(proj)
    for k in ("means2d", "conic", "opac", "rgb"):
        r[k] = proj[k].astype(dtype).astype(np.float64)
    return r


def all_pixels(width: int, height: int) -> np.ndarray:
    ys, xs = np.mgrid[0:height, 0:width]
    return np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)


def render_pixels(proj: dict, cfg: Cfg, pixels: np.ndarray, order: np.ndarray = None) -> dict:
    """Composites the given pixels ([m,2] integer x, y) front to back against
    every splat of ``proj`` in depth order. FP64 arithmetic throughout.
    Besides colour, T and the counts it returns the pixel flags and, for
    flagged pixels, ``reach`` [m, 2]: bounds on how far the colour and T can
    move when the flagged decisions go the other way (0 elsewhere)."""
    L = lib()
    n = int(proj["opac"].shape[0])
    if order is None:
        order = depth_order(proj["depth32"])
    c = lambda a, dt: np.ascontiguousarray(a, dtype=dt)
    m2, co, op, rgb = (c(proj["means2d"], np.float64), c(proj["conic"], np.float64),
                       c(proj["opac"], np.float64), c(proj["rgb"], np.float64))
    rect, fl = c(proj["rect"], np.int32), c(proj["flags"], np.uint8)
    order = c(order, np.int64)
    px = c(pixels, np.int32)
    m = int(px.shape[0])
    out = dict(color=np.zeros((m, 3)), T=np.zeros(m), n_contrib=np.zeros(m, np.int32),
               n_eval=np.zeros(m, np.int32), last_contrib=np.zeros(m, np.int32), flags=np.zeros(m, np.uint8),
               reach=np.zeros((m, 2), np.float64))
    cc = cfg._c()
    L.orc_render_pixels(ctypes.byref(cc), n, _p(order), _p(m2), _p(co), _p(op), _p(rgb), _p(rect), _p(fl),
                        m, _p(px), _p(out["color"]), _p(out["T"]), _p(out["n_contrib"]), _p(out["n_eval"]),
                        _p(out["last_contrib"]), _p(out["flags"]), _p(out["reach"]))
    return out


def rect_min_q(a, b, c, x0, x1, y0, y1) -> float:
    """Least a dx^2 + 2 b dx dy + c dy^2 over [x0, x1] x [y0, y1] (orc_rect_min_q)."""
    return float(lib().orc_rect_min_q(a, b, c, x0, x1, y0, y1))


def cull_cut(cfg: Cfg, o, a, b, c) -> float:
    """The per-tile test's bound on Q for one record (orc_cull_cut)."""
    return float(lib().orc_cull_cut(ctypes.byref(cfg._c()), o, a, b, c))


def tile_keep(cfg: Cfg, u, v, a, b, c, cut, tx, ty):
    """(keep, near) of the per-tile test for one splat and tile (orc_tile_keep)."""
    near = ctypes.c_int(0)
    k = lib().orc_tile_keep(u, v, a, b, c, cut, int(tx), int(ty), int(cfg.tile), ctypes.byref(near))
    return bool(k), bool(near.value)


def _cull_inputs(proj: dict, cfg: Cfg):
    c = lambda a, dt: np.ascontiguousarray(a, dtype=dt)
    m2, co, op = c(proj["means2d"], np.float64), c(proj["conic"], np.float64), c(proj["opac"], np.float64)
    n = int(op.shape[0])
    cut = np.zeros(n, np.float64)
    lib().orc_cull_cuts(ctypes.byref(cfg._c()), n, _p(co), _p(op), _p(cut))
    return n, m2, co, cut, c(proj["rect"], np.int32)


def cull_histogram(proj: dict, cfg: Cfg, grid_w: int, grid_h: int):
    """Kept copies per tile and near decisions per tile (int64 [grid_h * grid_w]
    each) with per-tile culling, over the records of ``proj``."""
    n, m2, co, cut, rect = _cull_inputs(proj, cfg)
    hist, near = np.zeros(grid_w * grid_h, np.int64), np.zeros(grid_w * grid_h, np.int64)
    lib().orc_cull_histogram(ctypes.byref(cfg._c()), n, _p(m2), _p(co), _p(cut), _p(rect), int(grid_w), int(grid_h),
                             _p(hist), _p(near))
    return hist, near


def cull_copy_mask(proj: dict, cfg: Cfg):
    """The test for every rectangle copy, in the order binning.bin_and_sort_fast
    lists copies before sorting (bool [sum of areas]), and the number of near
    decisions."""
    n, m2, co, cut, rect = _cull_inputs(proj, cfg)
    r = rect.astype(np.int64)
    cnt = np.maximum(r[:, 2] - r[:, 0] + 1, 0) * np.maximum(r[:, 3] - r[:, 1] + 1, 0)
    start = np.ascontiguousarray(np.cumsum(cnt) - cnt, np.int64)
    keep = np.zeros(int(cnt.sum()), np.uint8)
    nnear = lib().orc_cull_copy_mask(ctypes.byref(cfg._c()), n, _p(m2), _p(co), _p(cut), _p(rect), _p(start),
                                     _p(keep))
    return keep.astype(bool), int(nnear)


def cull_tile_members(proj: dict, cfg: Cfg, tx: int, ty: int):
    """Per splat: in tile (tx, ty)'s culled list (bool [n]), and whether that
    decision is near (bool [n])."""
    n, m2, co, cut, rect = _cull_inputs(proj, cfg)
    keep, near = np.zeros(n, np.uint8), np.zeros(n, np.uint8)
    lib().orc_cull_tile_members(ctypes.byref(cfg._c()), n, _p(m2), _p(co), _p(cut), _p(rect), int(tx), int(ty),
                                _p(keep), _p(near))
    return keep.astype(bool), near.astype(bool)


def render_image(scene, cam, cfg: Cfg, round_to=np.float32) -> dict:
    """Full frame: projection, fp32 record rounding (``round_to=None`` keeps
    FP64 records), depth order and every pixel. Returns image [3,H,W], T [H,W],
    n_contrib, n_eval, last_contrib, flags [H,W] and the projection."""
    proj = project(scene, cam, cfg)
    rec = round_records(proj, round_to) if round_to is not None else proj
    W, H = int(cam.width), int(cam.height)
    r = render_pixels(rec, cfg, all_pixels(W, H))
    return dict(image=r["color"].reshape(H, W, 3).transpose(2, 0, 1).copy(), T=r["T"].reshape(H, W),
                n_contrib=r["n_contrib"].reshape(H, W), n_eval=r["n_eval"].reshape(H, W),
                last_contrib=r["last_contrib"].reshape(H, W), flags=r["flags"].reshape(H, W), proj=proj)
