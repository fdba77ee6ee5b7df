"""The C-ABI library loads, exports every symbol include/gs.h declares, and
rejects bad arguments on the host before touching the GPU. No GPU needed."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2603_18707_amd import _lib as L
from tests.helpers import GOLDEN, ROOT


def _declared():
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = L.lib()
    names = _declared()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.EXPORTS)
    assert "gfx950" in L.gs_version()


def test_every_entry_point_with_parameters_declares_them():
    """ctypes passes undeclared arguments as C int: a pointer or stream would
    be truncated to 32 bits. Every binding declares its parameter types, and
    their count matches the header's prototype."""
    lib = L.lib()
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    for name in L.EXPORTS:
        proto = re.search(r"\b" + name + r"\s*\(([^)]*)\)", src).group(1).strip()
        nparams = 0 if proto in ("", "void") else proto.count(",") + 1
        if nparams == 0:
            continue
        argtypes = getattr(lib, name).argtypes
        assert argtypes is not None and len(argtypes) == nparams, (name, nparams, argtypes)


def test_default_coefficients():
    k1 = L.gs_kernel_default(L.KERNEL_POLY, 1, L.RADIUS_POLY_OPACITY)
    assert k1.coeffs[0] == 0.773 and abs(L.gs_kernel_root(k1) - 4.386) < 1e-12
    for order in (2, 3):
        k = L.gs_kernel_default(L.KERNEL_POLY, order, L.RADIUS_POLY_OPACITY)
        g = GOLDEN[f"fit{order}"]
        # the library's own fit agrees with the reference's independent fit
        assert np.allclose(list(k.coeffs)[:order + 1], g["c"][:order + 1], atol=5e-5)
        assert abs(L.gs_kernel_root(k) - g["x0"]) < 1e-3


def test_root_of_explicit_coefficients():
    for name in ("paper1", "fit1", "fit2", "fit3"):
        g = GOLDEN[name]
        k = L.make_kernel(L.KERNEL_POLY, g["order"], L.RADIUS_POLY_UNIVERSAL, g["c"])
        assert L.gs_kernel_root(k) == pytest.approx(g["x0"], rel=1e-13)


def _expect(status, fn, *a):
    with pytest.raises(L.GsError) as e:
        fn(*a)
    assert e.value.status == status
    return str(e.value)


def test_kernel_validation():
    k = L.make_kernel(L.KERNEL_POLY, 4, L.RADIUS_SIGMA3, (0.7, -0.1))
    _expect(L.GS_EINVAL, L.gs_kernel_root, k)
    k = L.make_kernel(7, 1, L.RADIUS_SIGMA3, (0.7, -0.1))
    _expect(L.GS_EINVAL, L.gs_kernel_root, k)
    k = L.make_kernel(L.KERNEL_POLY, 1, 9, (0.7, -0.1))
    _expect(L.GS_EINVAL, L.gs_kernel_root, k)
    k = L.make_kernel(L.KERNEL_POLY, 1, 0, (0.7, 0.1))      # increasing: no positive root
    _expect(L.GS_EUNSUPPORTED, L.gs_kernel_root, k)
    k = L.make_kernel(L.KERNEL_POLY, 3, 0, (1.0, -3.0, 3.0, -1.0))   # (1-x)^3: not strictly monotone
    _expect(L.GS_EUNSUPPORTED, L.gs_kernel_root, k)
    k = L.make_kernel(L.KERNEL_POLY, 1, 0, (0.7, -0.1))
    k.reserved = 1
    _expect(L.GS_EINVAL, L.gs_kernel_root, k)


class _Cam:
    viewmat = np.eye(4, dtype=np.float32)
    fx = fy = 100.0
    cx = cy = 32.0
    width = height = 64


def test_device_calls_reject_bad_arguments_on_host():
    cam = L.make_camera(_Cam())
    k = L.gs_kernel_default(L.KERNEL_POLY, 1, L.RADIUS_POLY_OPACITY)
    p = L.gs_params_default()
    null8 = [None] * 5
    out6 = [None] * 6
    # NULL arrays with n > 0
    _expect(L.GS_EINVAL, L.gs_preprocess, cam, k, p, 10, *null8, 0, *out6)
    # bad n / sh degree / tile / params / camera
    _expect(L.GS_EINVAL, L.gs_preprocess, cam, k, p, -1, *null8, 0, *out6)
    _expect(L.GS_EINVAL, L.gs_preprocess, cam, k, p, 0, *null8, 4, *out6)
    p2 = L.gs_params_default()
    p2.tile = 8
    _expect(L.GS_EUNSUPPORTED, L.gs_preprocess, cam, k, p2, 0, *null8, 0, *out6)
    p2 = L.gs_params_default()
    p2.near_z = 0.0
    _expect(L.GS_EINVAL, L.gs_preprocess, cam, k, p2, 0, *null8, 0, *out6)
    p2 = L.gs_params_default()
    p2.blend_stage = 3
    assert "blend_stage" in _expect(L.GS_EINVAL, L.gs_preprocess, cam, k, p2, 0, *null8, 0, *out6)
    c2 = L.make_camera(_Cam())
    c2.width = 0
    _expect(L.GS_EINVAL, L.gs_preprocess, c2, k, p, 0, *null8, 0, *out6)
    # misaligned outputs
    _expect(L.GS_EINVAL, L.gs_preprocess, cam, k, p, 1, 16, 16, 16, 16, 16, 0, 16, 20, 16, 16, 16, 16)
    msg = _expect(L.GS_EINVAL, L.gs_preprocess, cam, k, p, 1, 16, 16, 16, 16, 20, 3, 16, 16, 16, 16, 16, 16)
    assert "sh" in msg  # 16-byte SH rows are read with 16-byte loads
    # n = 0 is a no-op that enqueues nothing
    L.gs_preprocess(cam, k, p, 0, *null8, 0, *out6)
    # bin sort: workspace too small, capacity too large, grid invalid
    _expect(L.GS_EINVAL, L.gs_bin_sort, 10, 256, 256, 256, 4, 4, 100, 256, 10, 256, 256, 256, None, 256, 256)
    _expect(L.GS_EINVAL, L.gs_bin_sort_workspace, 10, 1 << 33, 16)
    _expect(L.GS_EINVAL, L.gs_bin_sort, 10, 256, 256, 256, 0, 4, 100, 256, 1 << 30, 256, 256, 256, None, 256, 256)
    # allocation-free bin sort: the grid check, and sizes beyond its scratch
    # (checked before any HIP call)
    _expect(L.GS_EINVAL, L.gs_bin_sort_noalloc, 10, 256, 256, 256, 0, 4, 100, 256, 256, 256, None, 256, 256)
    big = _expect(L.GS_ECAPACITY, L.gs_bin_sort_noalloc, 1_000_000, 256, 256, 256, 120, 68, 20_000_000,
                  256, 256, 256, None, 256, 256)
    assert "scratch" in big
    assert L.gs_bin_sort_workspace(1_000_000, 4_000_000, 120 * 68) <= L.GS_NOALLOC_SCRATCH_BYTES
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    assert "#define GS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)" in src
    # culled bin sort: the same checks, plus the records, the kernel and a grid below 2^22 tiles
    ws = L.gs_bin_sort_workspace(10, 100, 16)
    good = dict(depth=256, rect=256, tiles=256, m2=256, co=256)
    def culled(kern=k, par=p, n=10, gw=4, gh=4, ws_bytes=ws, **kw):
        a = {**good, **kw}
        return L.gs_bin_sort_culled(kern, par, n, a["depth"], a["rect"], a["tiles"], a["m2"], a["co"], gw, gh, 100,
                                    256, ws_bytes, 256, 256, 256, None, 256, 256)
    assert "NULL" in _expect(L.GS_EINVAL, lambda: culled(m2=None))
    assert "NULL" in _expect(L.GS_EINVAL, lambda: culled(co=None))
    assert "alignment" in _expect(L.GS_EINVAL, lambda: culled(co=264))
    assert "workspace" in _expect(L.GS_EINVAL, lambda: culled(ws_bytes=ws - 1))
    assert "2^22" in _expect(L.GS_EINVAL, lambda: culled(gw=4096, gh=1024))
    assert "32767" in _expect(L.GS_EINVAL, lambda: culled(gw=70000, gh=1))
    bad_k = L.gs_kernel_default(L.KERNEL_POLY, 1, L.RADIUS_POLY_OPACITY)
    bad_k.kind = 7
    _expect(L.GS_EINVAL, lambda: culled(kern=bad_k))
    p3 = L.gs_params_default()
    p3.eps = 0.0
    _expect(L.GS_EINVAL, lambda: culled(par=p3))
    # rasterize: NULL outputs
    _expect(L.GS_EINVAL, L.gs_rasterize_fwd, cam, k, p, 0, None, None, None, None, None, None, None, None, None, None)
    msg = _expect(L.GS_EINVAL, L.gs_rasterize_bwd, cam, k, p, 5, None, None, None, None, 256, None, 256, 256, 256,
                  None, None, None)
    assert "NULL" in msg


def test_workspace_grows_with_sizes():
    a = L.gs_bin_sort_workspace(1000, 10000, 64)
    b = L.gs_bin_sort_workspace(1000, 20000, 64)
    c = L.gs_bin_sort_workspace(1_000_000, 10000, 64)
    d = L.gs_bin_sort_workspace(1000, 10000, 1 << 20)
    assert 0 < a < b and a < c and a < d


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the public structs have the header's sizes and offsets (gcc)."""
    src = tmp_path / "sz.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "gs.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gs_kernel), sizeof(gs_params), sizeof(gs_camera),
         sizeof(gs_scene), sizeof(gs_view), offsetof(gs_view, image_offset), offsetof(gs_params, blend_threads),
         offsetof(gs_kernel, coeffs));
  return 0;
}
""")
    import subprocess
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(L.GsKernel), ctypes.sizeof(L.GsParams), ctypes.sizeof(L.GsCamera), ctypes.sizeof(L.GsScene),
            ctypes.sizeof(L.GsView), L.GsView.image_offset.offset, L.GsParams.blend_threads.offset,
            L.GsKernel.coeffs.offset]
    assert got == want


def test_batch_layout_validation():
    scenes = (L.GsScene * 2)()
    scenes[0].n, scenes[1].n = 1000, 70
    for s in scenes:
        s.means3d = s.scales = s.quats = s.opacities = s.sh = 4096
        s.sh_degree = 3
    views = (L.GsView * 3)()
    for i, (W, H, sc) in enumerate([(128, 64, 0), (33, 17, 1), (640, 360, 0)]):
        views[i].cam = L.make_camera(type("C", (), dict(viewmat=np.eye(4, dtype=np.float32), fx=100.0, fy=100.0,
                                                        cx=W / 2, cy=H / 2, width=W, height=H)))
        views[i].scene = sc
    pairs, gw, gh, ws = L.gs_batch_layout(scenes, views, 10000)
    assert pairs == 1024 + 128 + 1024          # each view padded to a multiple of 64 splats
    assert gw == 40 and gh == 4 + 2 + 23       # widest view's columns, all views' rows stacked
    assert ws > 0
    views[1].scene = 5
    _expect(L.GS_EINVAL, L.gs_batch_layout, scenes, views, 10000)
    views[1].scene = 1
    scenes[1].sh_degree = 2
    _expect(L.GS_EUNSUPPORTED, L.gs_batch_layout, scenes, views, 10000)
