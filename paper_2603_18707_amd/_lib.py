"""ctypes binding of libgs.so: one Python function per C entry point, same names.

Argument marshalling only (tensor -> device pointer, struct packing, status ->
exception); every step of the path runs in the library's HIP kernels. Loading
fails loudly when libgs.so has not been built: there is no fallback.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs.so")

GS_OK, GS_EINVAL, GS_EUNSUPPORTED, GS_ECAPACITY, GS_EHIP = 0, -1, -2, -3, -4
# scratch held by gs_bin_sort_noalloc (GS_NOALLOC_SCRATCH_BYTES in gs.h)
GS_NOALLOC_SCRATCH_BYTES = 128 << 20
KERNEL_EXP, KERNEL_POLY = 0, 1
RADIUS_SIGMA3, RADIUS_POLY_UNIVERSAL, RADIUS_POLY_OPACITY, RADIUS_EXP_OPACITY = 0, 1, 2, 3
RECT_SQUARE, RECT_ELLIPSE_BOX = 0, 1


class GsKernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("order", ctypes.c_int32), ("radius_mode", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("coeffs", ctypes.c_double * 4)]


class GsParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_float), ("alpha_max", ctypes.c_float), ("t_min", ctypes.c_float),
                ("aa_v", ctypes.c_float), ("near_z", ctypes.c_float), ("radius_pad", ctypes.c_float),
                ("bg", ctypes.c_float * 3), ("tile", ctypes.c_int32), ("blend_threads", ctypes.c_int32),
                ("rect_mode", ctypes.c_int32), ("blend_stage", ctypes.c_int32)]


class GsCamera(ctypes.Structure):
    _fields_ = [("viewmat", ctypes.c_float * 16), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32)]


class GsScene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("means3d", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacities", ctypes.c_void_p), ("sh", ctypes.c_void_p),
                ("sh_degree", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class GsView(ctypes.Structure):
    _fields_ = [("cam", GsCamera), ("scene", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("image_offset", ctypes.c_int64), ("pixel_offset", ctypes.c_int64)]


class GsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libgs status {status}: {msg}")
        self.status = status


_lib = None

EXPORTS = ("gs_version", "gs_last_error", "gs_kernel_default", "gs_kernel_order2_tile_range", "gs_kernel_root",
           "gs_params_default",
           "gs_preprocess", "gs_bin_sort_workspace", "gs_bin_sort", "gs_bin_sort_noalloc", "gs_bin_sort_culled", "gs_rasterize_fwd", "gs_rasterize_fwd_mfma", "gs_rasterize_fwd_count",
           "gs_rasterize_bwd", "gs_preprocess_bwd", "gs_batch_layout", "gs_render_batched")


def lib():
    """The loaded library. Raises if libgs.so is missing (build it with
    ``python -m paper_2603_18707_amd.build``); nothing falls back to the CPU."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2603_18707_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.gs_version.restype = ctypes.c_char_p
        L.gs_last_error.restype = ctypes.c_char_p
        L.gs_kernel_default.argtypes = [I32, I32, I32, P]
        L.gs_kernel_order2_tile_range.argtypes = [I32, P]
        L.gs_kernel_root.argtypes = [P, P]
        L.gs_params_default.argtypes = [P]
        L.gs_preprocess.argtypes = [P, P, P, I64] + [P] * 5 + [I32] + [P] * 6 + [P]
        L.gs_bin_sort_workspace.argtypes = [I64, I64, I32, P]
        L.gs_bin_sort.argtypes = [I64, P, P, P, I32, I32, I64, P, ctypes.c_size_t] + [P] * 6 + [P]
        L.gs_bin_sort_noalloc.argtypes = [I64, P, P, P, I32, I32, I64] + [P] * 6 + [P]
        L.gs_bin_sort_culled.argtypes = [P, P, I64, P, P, P, P, P, I32, I32, I64, P, ctypes.c_size_t] + [P] * 6 + [P]
        L.gs_rasterize_fwd.argtypes = [P, P, P, I64] + [P] * 6 + [P] * 5 + [P]
        L.gs_rasterize_fwd_mfma.argtypes = [P, P, P, I64] + [P] * 6 + [P] * 5 + [P]
        L.gs_rasterize_fwd_count.argtypes = [P, P, P, I64] + [P] * 6 + [P] * 6 + [P]
        L.gs_rasterize_bwd.argtypes = [P, P, P, I64] + [P] * 6 + [P] * 3 + [P] * 3 + [P]
        L.gs_preprocess_bwd.argtypes = [P, P, P, I64] + [P] * 5 + [I32] + [P] * 4 + [P] * 5 + [P]
        L.gs_batch_layout.argtypes = [P, I32, P, I32, I64, P, P, P, P]
        L.gs_render_batched.argtypes = [P, P, P, I32, P, P, I32, I64, I32, P, ctypes.c_size_t, P, I64, P, P, P, I64,
                                        P, P, P, P]
        for name in EXPORTS[2:]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status):
    if status != GS_OK:
        raise GsError(status, lib().gs_last_error().decode())


def _ptr(t):
    """Device (or host) address of a tensor, or NULL for None."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


# ---------------------------------------------------------------------------
# host helpers
# ---------------------------------------------------------------------------

def gs_version() -> str:
    return lib().gs_version().decode()


def gs_kernel_default(kind: int, order: int, radius_mode: int) -> GsKernel:
    k = GsKernel()
    _check(lib().gs_kernel_default(kind, order, radius_mode, ctypes.byref(k)))
    return k


def gs_kernel_order2_tile_range(radius_mode: int) -> GsKernel:
    k = GsKernel()
    _check(lib().gs_kernel_order2_tile_range(radius_mode, ctypes.byref(k)))
    return k


def gs_kernel_root(kernel: GsKernel) -> float:
    x = ctypes.c_double()
    _check(lib().gs_kernel_root(ctypes.byref(kernel), ctypes.byref(x)))
    return x.value


def gs_params_default() -> GsParams:
    p = GsParams()
    _check(lib().gs_params_default(ctypes.byref(p)))
    return p


def make_kernel(kind: int, order: int, radius_mode: int, coeffs=None) -> GsKernel:
    """Library defaults for (kind, order, radius_mode), optionally with explicit coefficients."""
    k = GsKernel()
    k.kind, k.order, k.radius_mode, k.reserved = kind, order, radius_mode, 0
    if coeffs is None:
        return gs_kernel_default(kind, order, radius_mode)
    cc = list(coeffs) + [0.0] * (4 - len(coeffs))
    for i in range(4):
        k.coeffs[i] = float(cc[i])
    return k


def make_camera(cam) -> GsCamera:
    """From any object with viewmat [4,4], fx, fy, cx, cy, width, height."""
    c = GsCamera()
    vm = [float(v) for v in torch.as_tensor(cam.viewmat, dtype=torch.float32).reshape(-1).tolist()]
    for i in range(16):
        c.viewmat[i] = vm[i]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


# ---------------------------------------------------------------------------
# device entry points (same names and argument order as include/gs.h)
# ---------------------------------------------------------------------------

def gs_preprocess(cam, kernel, params, n, means3d, scales, quats, opacities, sh, sh_degree, means2d,
                  conic_opacity, rgb, depth, rect, tiles_touched, stream=None):
    _check(lib().gs_preprocess(ctypes.byref(cam), ctypes.byref(kernel), ctypes.byref(params), int(n),
                               _ptr(means3d), _ptr(scales), _ptr(quats), _ptr(opacities), _ptr(sh), int(sh_degree),
                               _ptr(means2d), _ptr(conic_opacity), _ptr(rgb), _ptr(depth), _ptr(rect),
                               _ptr(tiles_touched), _stream(stream)))


def gs_bin_sort_workspace(n, key_capacity, num_tiles) -> int:
    b = ctypes.c_size_t()
    _check(lib().gs_bin_sort_workspace(int(n), int(key_capacity), int(num_tiles), ctypes.byref(b)))
    return b.value


def gs_bin_sort(n, depth, rect, tiles_touched, grid_w, grid_h, key_capacity, workspace, workspace_bytes, keys,
                vals, ranges, tile_order, num_keys, overflow, stream=None):
    _check(lib().gs_bin_sort(int(n), _ptr(depth), _ptr(rect), _ptr(tiles_touched), int(grid_w), int(grid_h),
                             int(key_capacity), _ptr(workspace), int(workspace_bytes), _ptr(keys), _ptr(vals),
                             _ptr(ranges), _ptr(tile_order), _ptr(num_keys), _ptr(overflow), _stream(stream)))


def gs_bin_sort_noalloc(n, depth, rect, tiles_touched, grid_w, grid_h, key_capacity, keys, vals, ranges, tile_order,
                        num_keys, overflow, stream=None):
    _check(lib().gs_bin_sort_noalloc(int(n), _ptr(depth), _ptr(rect), _ptr(tiles_touched), int(grid_w), int(grid_h),
                                     int(key_capacity), _ptr(keys), _ptr(vals), _ptr(ranges), _ptr(tile_order),
                                     _ptr(num_keys), _ptr(overflow), _stream(stream)))


def gs_bin_sort_culled(kernel, params, n, depth, rect, tiles_touched, means2d, conic_opacity, grid_w, grid_h,
                       key_capacity, workspace, workspace_bytes, keys, vals, ranges, tile_order, num_keys, overflow,
                       stream=None):
    _check(lib().gs_bin_sort_culled(ctypes.byref(kernel), ctypes.byref(params), int(n), _ptr(depth), _ptr(rect),
                                    _ptr(tiles_touched), _ptr(means2d), _ptr(conic_opacity), int(grid_w), int(grid_h),
                                    int(key_capacity), _ptr(workspace), int(workspace_bytes), _ptr(keys), _ptr(vals),
                                    _ptr(ranges), _ptr(tile_order), _ptr(num_keys), _ptr(overflow), _stream(stream)))


def gs_rasterize_fwd(cam, kernel, params, n, means2d, conic_opacity, rgb, vals, ranges, tile_order, image, final_T,
                     n_contrib, last_contrib, n_eval=None, stream=None):
    _check(lib().gs_rasterize_fwd(ctypes.byref(cam), ctypes.byref(kernel), ctypes.byref(params), int(n),
                                  _ptr(means2d), _ptr(conic_opacity), _ptr(rgb), _ptr(vals), _ptr(ranges),
                                  _ptr(tile_order), _ptr(image), _ptr(final_T), _ptr(n_contrib), _ptr(last_contrib),
                                  _ptr(n_eval), _stream(stream)))


def gs_rasterize_fwd_mfma(cam, kernel, params, n, means2d, conic_opacity, rgb, vals, ranges, tile_order, image,
                          final_T, n_contrib, last_contrib, n_eval=None, stream=None):
    _check(lib().gs_rasterize_fwd_mfma(ctypes.byref(cam), ctypes.byref(kernel), ctypes.byref(params), int(n),
                                       _ptr(means2d), _ptr(conic_opacity), _ptr(rgb), _ptr(vals), _ptr(ranges),
                                       _ptr(tile_order), _ptr(image), _ptr(final_T), _ptr(n_contrib),
                                       _ptr(last_contrib), _ptr(n_eval), _stream(stream)))


def gs_rasterize_fwd_count(cam, kernel, params, n, means2d, conic_opacity, rgb, vals, ranges, tile_order, image,
                           final_T, n_contrib, last_contrib, n_eval, n_tested, stream=None):
    _check(lib().gs_rasterize_fwd_count(ctypes.byref(cam), ctypes.byref(kernel), ctypes.byref(params), int(n),
                                        _ptr(means2d), _ptr(conic_opacity), _ptr(rgb), _ptr(vals), _ptr(ranges),
                                        _ptr(tile_order), _ptr(image), _ptr(final_T), _ptr(n_contrib),
                                        _ptr(last_contrib), _ptr(n_eval), _ptr(n_tested), _stream(stream)))


def gs_rasterize_bwd(cam, kernel, params, n, means2d, conic_opacity, rgb, vals, ranges, tile_order, final_T,
                     last_contrib, dL_dimage, dL_dmeans2d, dL_dconic_opacity, dL_drgb, stream=None):
    _check(lib().gs_rasterize_bwd(ctypes.byref(cam), ctypes.byref(kernel), ctypes.byref(params), int(n),
                                  _ptr(means2d), _ptr(conic_opacity), _ptr(rgb), _ptr(vals), _ptr(ranges),
                                  _ptr(tile_order), _ptr(final_T), _ptr(last_contrib), _ptr(dL_dimage),
                                  _ptr(dL_dmeans2d), _ptr(dL_dconic_opacity), _ptr(dL_drgb), _stream(stream)))


def gs_preprocess_bwd(cam, kernel, params, n, means3d, scales, quats, opacities, sh, sh_degree, tiles_touched,
                      dL_dmeans2d, dL_dconic_opacity, dL_drgb, dL_dmeans3d, dL_dscales, dL_dquats, dL_dopacities,
                      dL_dsh, stream=None):
    _check(lib().gs_preprocess_bwd(ctypes.byref(cam), ctypes.byref(kernel), ctypes.byref(params), int(n),
                                   _ptr(means3d), _ptr(scales), _ptr(quats), _ptr(opacities), _ptr(sh),
                                   int(sh_degree), _ptr(tiles_touched), _ptr(dL_dmeans2d), _ptr(dL_dconic_opacity),
                                   _ptr(dL_drgb), _ptr(dL_dmeans3d), _ptr(dL_dscales), _ptr(dL_dquats),
                                   _ptr(dL_dopacities), _ptr(dL_dsh), _stream(stream)))


def gs_batch_layout(scenes, views, key_capacity):
    """(num_pairs, grid_w, grid_h, workspace_bytes) for ctypes arrays of GsScene / GsView."""
    n, gw, gh, b = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
    _check(lib().gs_batch_layout(scenes, len(scenes), views, len(views), int(key_capacity), ctypes.byref(n),
                                 ctypes.byref(gw), ctypes.byref(gh), ctypes.byref(b)))
    return n.value, gw.value, gh.value, b.value


def gs_render_batched(kernel, params, scenes, views, views_device, key_capacity, workgroups, workspace,
                      workspace_bytes, images, images_len, final_T, n_contrib, last_contrib, planes_len, num_keys,
                      overflow, stream=None, view_keys=None):
    _check(lib().gs_render_batched(ctypes.byref(kernel), ctypes.byref(params), scenes, len(scenes), views,
                                   _ptr(views_device), len(views), int(key_capacity), int(workgroups),
                                   _ptr(workspace), int(workspace_bytes), _ptr(images), int(images_len),
                                   _ptr(final_T), _ptr(n_contrib), _ptr(last_contrib), int(planes_len),
                                   _ptr(num_keys), _ptr(overflow), _ptr(view_keys), _stream(stream)))
