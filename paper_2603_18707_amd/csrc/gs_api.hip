// extern "C" entry points of libgs: host-side argument checks, kernel
// resolution (coefficients, first root, radius multiplier) and launches.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "gs_coeffs.h"
#include "gs_internal.h"

namespace gs {

static thread_local char g_err[512] = "";

gs_status fail(gs_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

gs_status check_hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return GS_OK;
  return fail(GS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

namespace {

double peval(const double *c, int order, double x) {
  double s = c[order];
  for (int i = order - 1; i >= 0; --i) s = s * x + c[i];
  return s;
}

double pderiv(const double *c, int order, double x) {
  double s = order * c[order];
  for (int i = order - 1; i >= 1; --i) s = s * x + i * c[i];
  return s;
}

// first positive root of p by the closed forms of App. B, Newton-polished
double closed_root(const double *c, int order) {
  double x;
  if (order == 1) {
    x = -c[0] / c[1];
  } else if (order == 2) {
    const double disc = c[1] * c[1] - 4.0 * c[0] * c[2];
    if (disc < 0.0) return -1.0;
    x = 2.0 * c[0] / (-c[1] + std::sqrt(disc));
  } else {
    const double d0 = c[2] * c[2] - 3.0 * c[3] * c[1];
    const double d1 = 2.0 * c[2] * c[2] * c[2] - 9.0 * c[3] * c[2] * c[1] + 27.0 * c[3] * c[3] * c[0];
    const double s = d1 * d1 - 4.0 * d0 * d0 * d0;
    const double sq = std::sqrt(s > 0.0 ? s : 0.0);
    const double C = std::cbrt(d1 >= 0.0 ? 0.5 * (d1 + sq) : 0.5 * (d1 - sq));
    x = -(c[2] + C + d0 / C) / (3.0 * c[3]);
  }
  for (int it = 0; it < 3; ++it) {
    const double fp = pderiv(c, order, x);
    if (fp != 0.0) x -= peval(c, order, x) / fp;
  }
  return x;
}

bool finite_pos(float v) { return std::isfinite(v) && v > 0.0f; }

gs_status check_params(const gs_params *p) {
  if (!p) return fail(GS_EINVAL, "params is NULL");
  if (p->tile != 16) return fail(GS_EUNSUPPORTED, "tile = %d: only 16x16 tiles are supported", p->tile);
  if (!finite_pos(p->eps) || !(p->eps < 1.0f)) return fail(GS_EINVAL, "eps must be in (0, 1)");
  if (!finite_pos(p->alpha_max) || p->alpha_max > 1.0f) return fail(GS_EINVAL, "alpha_max must be in (0, 1]");
  if (!(p->t_min >= 0.0f && p->t_min < 1.0f)) return fail(GS_EINVAL, "t_min must be in [0, 1)");
  if (!(p->aa_v >= 0.0f) || !std::isfinite(p->aa_v)) return fail(GS_EINVAL, "aa_v must be finite and >= 0");
  if (!finite_pos(p->near_z)) return fail(GS_EINVAL, "near_z must be finite and > 0");
  if (!(p->radius_pad >= 1.0f) || !std::isfinite(p->radius_pad)) return fail(GS_EINVAL, "radius_pad must be >= 1");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(p->bg[i])) return fail(GS_EINVAL, "bg must be finite");
  if (p->blend_threads != 0 && p->blend_threads != 64 && p->blend_threads != 128 && p->blend_threads != 256)
    return fail(GS_EINVAL, "blend_threads %d must be 0, 64, 128 or 256", p->blend_threads);
  if (p->rect_mode != GS_RECT_SQUARE && p->rect_mode != GS_RECT_ELLIPSE_BOX)
    return fail(GS_EINVAL, "rect_mode %d must be 0 (square) or 1 (ellipse box)", p->rect_mode);
  if (p->blend_stage < 0 || p->blend_stage > 2)
    return fail(GS_EINVAL, "blend_stage %d must be 0, 1 or 2", p->blend_stage);
  return GS_OK;
}

gs_status check_camera(const gs_camera *c) {
  if (!c) return fail(GS_EINVAL, "camera is NULL");
  if (c->width < 1 || c->height < 1 || c->width > 32768 || c->height > 32768)
    return fail(GS_EINVAL, "image size %dx%d outside 1..32768", c->width, c->height);
  if (!finite_pos(c->fx) || !finite_pos(c->fy)) return fail(GS_EINVAL, "focal lengths must be finite and > 0");
  if (!std::isfinite(c->cx) || !std::isfinite(c->cy)) return fail(GS_EINVAL, "principal point must be finite");
  for (int i = 0; i < 12; ++i)
    if (!std::isfinite(c->viewmat[i])) return fail(GS_EINVAL, "viewmat must be finite");
  return GS_OK;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

gs_status resolve_kernel(const gs_kernel *k, Resolved *r) {
  if (!k) return fail(GS_EINVAL, "kernel is NULL");
  if (k->kind != GS_KERNEL_EXP && k->kind != GS_KERNEL_POLY) return fail(GS_EINVAL, "kernel kind %d", k->kind);
  if (k->radius_mode < GS_RADIUS_SIGMA3 || k->radius_mode > GS_RADIUS_EXP_OPACITY)
    return fail(GS_EINVAL, "radius_mode %d", k->radius_mode);
  if (k->reserved != 0) return fail(GS_EINVAL, "reserved field must be 0");
  std::memset(r, 0, sizeof(*r));
  r->kind = k->kind;
  r->radius_mode = k->radius_mode;
  r->order = k->order;
  const bool needs_poly = k->kind == GS_KERNEL_POLY || k->radius_mode == GS_RADIUS_POLY_UNIVERSAL ||
                          k->radius_mode == GS_RADIUS_POLY_OPACITY;
  if (!needs_poly) {
    r->order = 1;
    return GS_OK;
  }
  if (k->order < 1 || k->order > 3) return fail(GS_EINVAL, "polynomial order %d outside 1..3", k->order);
  for (int i = 0; i <= k->order; ++i) {
    if (!std::isfinite(k->coeffs[i])) return fail(GS_EINVAL, "coefficient c_%d is not finite", i);
    r->c[i] = k->coeffs[i];
  }
  const double *c = r->c;
  const int N = k->order;
  if (!(c[0] > 0.0)) return fail(GS_EUNSUPPORTED, "c_0 must be > 0");
  if (c[N] == 0.0) return fail(GS_EUNSUPPORTED, "leading coefficient c_%d is 0; use a lower order", N);
  if (N == 3 && !(c[2] * c[2] < 3.0 * c[1] * c[3]))
    return fail(GS_EUNSUPPORTED, "cubic kernel must be strictly monotone (one real root)");
  const double x0 = closed_root(c, N);
  if (!(x0 > 0.0) || !std::isfinite(x0)) return fail(GS_EUNSUPPORTED, "polynomial has no positive root");
  // p must decrease on [0, x0] so that every opacity bound is the unique root there:
  // p' has degree <= 2, so check both ends and an interior vertex
  bool dec = pderiv(c, N, 0.0) < 0.0 && pderiv(c, N, x0) < 0.0;
  if (N == 3) {
    const double xv = -c[2] / (3.0 * c[3]);
    if (xv > 0.0 && xv < x0) dec = dec && pderiv(c, N, xv) < 0.0;
  }
  if (!dec) return fail(GS_EUNSUPPORTED, "polynomial must decrease on [0, x0]");
  r->x0 = x0;
  return GS_OK;
}

}  // namespace gs

using namespace gs;

extern "C" {

const char *gs_version(void) { return "libgs 0.1 (gfx950)"; }

const char *gs_last_error(void) { return g_err; }

gs_status gs_kernel_default(int32_t kind, int32_t order, int32_t radius_mode, gs_kernel *out) {
  if (!out) return fail(GS_EINVAL, "out is NULL");
  if (order < 1 || order > 3) return fail(GS_EINVAL, "order %d outside 1..3", order);
  std::memset(out, 0, sizeof(*out));
  out->kind = kind;
  out->order = order;
  out->radius_mode = radius_mode;
  if (order == 1) {
    // Sec. 3.1: intercept 0.773, root at 4.386 (the printed labels read as swapped)
    out->coeffs[0] = 0.773;
    out->coeffs[1] = -0.773 / 4.386;
  } else {
    const double *t = order == 2 ? GS_FIT_ORDER2 : GS_FIT_ORDER3;
    for (int i = 0; i < 4; ++i) out->coeffs[i] = t[i];
  }
  Resolved r;
  return resolve_kernel(out, &r);
}

gs_status gs_kernel_order2_tile_range(int32_t radius_mode, gs_kernel *out) {
  if (!out) return fail(GS_EINVAL, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  out->kind = GS_KERNEL_POLY;
  out->order = 2;
  out->radius_mode = radius_mode;
  for (int i = 0; i < 4; ++i) out->coeffs[i] = GS_FIT_ORDER2_TILE16[i];
  Resolved r;
  return resolve_kernel(out, &r);
}

gs_status gs_kernel_root(const gs_kernel *kernel, double *x0_out) {
  if (!x0_out) return fail(GS_EINVAL, "x0_out is NULL");
  Resolved r;
  gs_status st = resolve_kernel(kernel, &r);
  if (st != GS_OK) return st;
  *x0_out = r.x0;
  return GS_OK;
}

gs_status gs_params_default(gs_params *out) {
  if (!out) return fail(GS_EINVAL, "out is NULL");
  out->eps = 1.0f / 255.0f;
  out->alpha_max = 0.99f;
  out->t_min = 1e-4f;
  out->aa_v = 0.3f;
  out->near_z = 0.2f;
  out->radius_pad = 1.0f + 1.0f / 1048576.0f;
  out->bg[0] = out->bg[1] = out->bg[2] = 0.0f;
  out->tile = 16;
  out->blend_threads = 0;
  out->rect_mode = GS_RECT_SQUARE;
  out->blend_stage = 0;
  return GS_OK;
}

gs_status gs_preprocess(const gs_camera *cam, const gs_kernel *kernel, const gs_params *params, int64_t n,
                        const float *means3d, const float *scales, const float *quats, const float *opacities,
                        const float *sh, int32_t sh_degree, float *means2d, float *conic_opacity, float *rgb,
                        float *depth, int32_t *rect, uint32_t *tiles_touched, void *stream) {
  gs_status st;
  if ((st = check_camera(cam)) != GS_OK || (st = check_params(params)) != GS_OK) return st;
  Resolved r;
  if ((st = resolve_kernel(kernel, &r)) != GS_OK) return st;
  if (n < 0 || n >= (1ll << 31)) return fail(GS_EINVAL, "n = %lld outside [0, 2^31)", (long long)n);
  if (sh_degree < 0 || sh_degree > 3) return fail(GS_EINVAL, "sh_degree %d outside 0..3", sh_degree);
  if (n == 0) return GS_OK;
  if (!means3d || !scales || !quats || !opacities || !sh || !means2d || !conic_opacity || !rgb || !depth || !rect ||
      !tiles_touched)
    return fail(GS_EINVAL, "NULL array argument");
  if (!aligned(means2d, 8) || !aligned(conic_opacity, 16) || !aligned(rect, 16) || !aligned(sh, 16))
    return fail(GS_EINVAL, "means2d needs 8-byte, conic_opacity, rect and sh 16-byte alignment");
  PreParams p;
  std::memset(&p, 0, sizeof(p));
  make_cam(cam, params->tile, &p.cam);
  p.radius_mode = r.radius_mode;
  p.order = r.order;
  p.sh_degree = sh_degree;
  p.tile = params->tile;
  p.rect_mode = params->rect_mode;
  for (int i = 0; i < 4; ++i) p.c[i] = r.c[i];
  p.k_universal = std::sqrt(r.x0);
  p.eps = params->eps;
  p.aa_v = params->aa_v;
  p.near_z = params->near_z;
  p.pad = params->radius_pad;
  PreOut o{means2d, conic_opacity, rgb, depth, rect, tiles_touched};
  return check_hip(launch_preprocess(p, n, means3d, scales, quats, opacities, sh, o, (hipStream_t)stream),
                   "gs_preprocess launch");
}

gs_status gs_bin_sort_workspace(int64_t n, int64_t key_capacity, int32_t num_tiles, size_t *bytes) {
  if (!bytes) return fail(GS_EINVAL, "bytes is NULL");
  if (n < 0 || n >= (1ll << 31)) return fail(GS_EINVAL, "n outside [0, 2^31)");
  if (key_capacity < 0 || key_capacity >= (1ll << 32)) return fail(GS_EINVAL, "key_capacity outside [0, 2^32)");
  if (num_tiles < 1) return fail(GS_EINVAL, "num_tiles must be >= 1");
  *bytes = binsort_workspace_bytes(n, key_capacity, num_tiles);
  return GS_OK;
}

gs_status gs_bin_sort(int64_t n, const float *depth, const int32_t *rect, const uint32_t *tiles_touched,
                      int32_t grid_w, int32_t grid_h, int64_t key_capacity, void *workspace, size_t workspace_bytes,
                      uint64_t *keys, uint32_t *vals, uint32_t *ranges, uint32_t *tile_order, int64_t *num_keys,
                      int32_t *overflow, void *stream) {
  if (grid_w < 1 || grid_h < 1 || (int64_t)grid_w * grid_h > (1ll << 30))
    return fail(GS_EINVAL, "tile grid %dx%d invalid", grid_w, grid_h);
  size_t need = 0;
  gs_status st = gs_bin_sort_workspace(n, key_capacity, grid_w * grid_h, &need);
  if (st != GS_OK) return st;
  if (!workspace || workspace_bytes < need)
    return fail(GS_EINVAL, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, need);
  if (!ranges || !num_keys || !overflow) return fail(GS_EINVAL, "NULL output argument");
  if (key_capacity > 0 && (!keys || !vals)) return fail(GS_EINVAL, "NULL keys or vals");
  if (n > 0 && (!depth || !rect || !tiles_touched)) return fail(GS_EINVAL, "NULL input argument");
  if (!aligned(workspace, 256) || (rect && !aligned(rect, 16)) || (keys && !aligned(keys, 8)))
    return fail(GS_EINVAL, "workspace needs 256-byte, rect 16-byte, keys 8-byte alignment");
  return check_hip(launch_binsort(n, depth, rect, tiles_touched, grid_w, grid_h, key_capacity, workspace,
                                  workspace_bytes, keys, vals, ranges, tile_order, num_keys, overflow,
                                  (hipStream_t)stream),
                   "gs_bin_sort launch");
}

// Workspace of gs_bin_sort_noalloc. In host code `scratch` names a host-side
// stand-in, not device memory: kernels get the address looked up per device.
static __device__ __align__(256) unsigned char scratch[GS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// the current device's copy of `scratch`, looked up on first use
gs_status device_scratch(void **out) {
  int dev = -1;
  gs_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (st != GS_OK) return st;
  if (dev < 0 || dev >= MAX_DEVICES) return fail(GS_EUNSUPPORTED, "device %d beyond the %d supported", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if ((st = check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)")) != GS_OK)
      return st;
    if (!ptr) return fail(GS_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GS_OK;
}
}  // namespace

gs_status gs_bin_sort_noalloc(int64_t n, const float *depth, const int32_t *rect, const uint32_t *tiles_touched,
                              int32_t grid_w, int32_t grid_h, int64_t key_capacity, uint64_t *keys, uint32_t *vals,
                              uint32_t *ranges, uint32_t *tile_order, int64_t *num_keys, int32_t *overflow,
                              void *stream) {
  if (grid_w < 1 || grid_h < 1 || (int64_t)grid_w * grid_h > (1ll << 30))
    return fail(GS_EINVAL, "tile grid %dx%d invalid", grid_w, grid_h);
  size_t need = 0;
  gs_status st = gs_bin_sort_workspace(n, key_capacity, grid_w * grid_h, &need);
  if (st != GS_OK) return st;
  if (need > GS_NOALLOC_SCRATCH_BYTES)
    return fail(GS_ECAPACITY, "gs_bin_sort_noalloc needs %zu bytes of scratch, more than the %zu it holds", need,
                (size_t)GS_NOALLOC_SCRATCH_BYTES);
  void *ws = nullptr;
  if ((st = device_scratch(&ws)) != GS_OK) return st;
  return gs_bin_sort(n, depth, rect, tiles_touched, grid_w, grid_h, key_capacity, ws, GS_NOALLOC_SCRATCH_BYTES,
                     keys, vals, ranges, tile_order, num_keys, overflow, stream);
}

// the kernel part of the blend parameters (no image size)
static gs_status make_kernel_params(const gs_kernel *kernel, const gs_params *params, BlendParams *b) {
  gs_status st;
  if ((st = check_params(params)) != GS_OK) return st;
  Resolved r;
  if ((st = resolve_kernel(kernel, &r)) != GS_OK) return st;
  std::memset(b, 0, sizeof(*b));
  b->blend = blend_kind(r);
  for (int i = 0; i < 4; ++i) b->c[i] = (float)r.c[i];
  b->x0 = (float)r.x0;
  b->eps = params->eps;
  b->log2_eps = std::log2(params->eps);
  b->alpha_max = params->alpha_max;
  b->t_min = params->t_min;
  for (int i = 0; i < 3; ++i) b->bg[i] = params->bg[i];
  b->threads = params->blend_threads ? params->blend_threads : 256;
  b->stage = params->blend_stage ? params->blend_stage : 2;
  return GS_OK;
}

static gs_status make_blend(const gs_camera *cam, const gs_kernel *kernel, const gs_params *params,
                            BlendParams *b) {
  gs_status st;
  if ((st = check_camera(cam)) != GS_OK || (st = make_kernel_params(kernel, params, b)) != GS_OK) return st;
  b->W = cam->width;
  b->H = cam->height;
  b->gx = (cam->width + params->tile - 1) / params->tile;
  b->gy = (cam->height + params->tile - 1) / params->tile;
  return GS_OK;
}

gs_status gs_bin_sort_culled(const gs_kernel *kernel, const gs_params *params, int64_t n, const float *depth,
                             const int32_t *rect, const uint32_t *tiles_touched, const float *means2d,
                             const float *conic_opacity, int32_t grid_w, int32_t grid_h, int64_t key_capacity,
                             void *workspace, size_t workspace_bytes, uint64_t *keys, uint32_t *vals,
                             uint32_t *ranges, uint32_t *tile_order, int64_t *num_keys, int32_t *overflow,
                             void *stream) {
  BlendParams b;
  gs_status st = make_kernel_params(kernel, params, &b);
  if (st != GS_OK) return st;
  if (grid_w < 1 || grid_h < 1 || (int64_t)grid_w * grid_h >= (1ll << 22))
    return fail(GS_EINVAL, "tile grid %dx%d invalid for culled binning (needs fewer than 2^22 tiles)", grid_w, grid_h);
  // the saved per-row runs hold a tile column in 16 bits
  if (grid_w > 32767) return fail(GS_EINVAL, "tile grid %d columns wide: culled binning takes at most 32767", grid_w);
  size_t need = 0;
  if ((st = gs_bin_sort_workspace(n, key_capacity, grid_w * grid_h, &need)) != GS_OK) return st;
  if (!workspace || workspace_bytes < need)
    return fail(GS_EINVAL, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, need);
  if (!ranges || !num_keys || !overflow) return fail(GS_EINVAL, "NULL output argument");
  if (key_capacity > 0 && (!keys || !vals)) return fail(GS_EINVAL, "NULL keys or vals");
  if (n > 0 && (!depth || !rect || !tiles_touched || !means2d || !conic_opacity))
    return fail(GS_EINVAL, "NULL input argument");
  if (!aligned(workspace, 256) || (rect && !aligned(rect, 16)) || (keys && !aligned(keys, 8)) ||
      (means2d && !aligned(means2d, 8)) || (conic_opacity && !aligned(conic_opacity, 16)))
    return fail(GS_EINVAL,
                "workspace needs 256-byte, rect and conic_opacity 16-byte, keys and means2d 8-byte alignment");
  return check_hip(launch_binsort_culled(n, depth, rect, tiles_touched, means2d, conic_opacity, b, grid_w,
                                         grid_h, key_capacity, workspace, workspace_bytes, keys, vals, ranges,
                                         tile_order, num_keys, overflow, (hipStream_t)stream),
                   "gs_bin_sort_culled launch");
}

gs_status gs_rasterize_fwd(const gs_camera *cam, const gs_kernel *kernel, const gs_params *params, int64_t n,
                           const float *means2d, const float *conic_opacity, const float *rgb,
                           const uint32_t *vals, const uint32_t *ranges, const uint32_t *tile_order, float *image,
                           float *final_T, uint32_t *n_contrib, uint32_t *last_contrib, uint32_t *n_eval,
                           void *stream) {
  BlendParams b;
  gs_status st = make_blend(cam, kernel, params, &b);
  if (st != GS_OK) return st;
  if (n < 0 || n >= (1ll << 31)) return fail(GS_EINVAL, "n outside [0, 2^31)");
  b.n = (uint32_t)n;
  if (!ranges || !image || !final_T || !n_contrib || !last_contrib) return fail(GS_EINVAL, "NULL argument");
  if (n > 0 && (!means2d || !conic_opacity || !rgb || !vals)) return fail(GS_EINVAL, "NULL splat argument");
  if ((means2d && !aligned(means2d, 8)) || (conic_opacity && !aligned(conic_opacity, 16)))
    return fail(GS_EINVAL, "means2d needs 8-byte, conic_opacity 16-byte alignment");
  BlendOut o{image, final_T, n_contrib, last_contrib, n_eval, nullptr};
  return check_hip(launch_blend_fwd(b, means2d, conic_opacity, rgb, vals, ranges, tile_order, o, (hipStream_t)stream),
                   "gs_rasterize_fwd launch");
}

gs_status gs_rasterize_fwd_mfma(const gs_camera *cam, const gs_kernel *kernel, const gs_params *params, int64_t n,
                                const float *means2d, const float *conic_opacity, const float *rgb,
                                const uint32_t *vals, const uint32_t *ranges, const uint32_t *tile_order,
                                float *image, float *final_T, uint32_t *n_contrib, uint32_t *last_contrib,
                                uint32_t *n_eval, void *stream) {
  BlendParams b;
  gs_status st = make_blend(cam, kernel, params, &b);
  if (st != GS_OK) return st;
  if (n < 0 || n >= (1ll << 31)) return fail(GS_EINVAL, "n outside [0, 2^31)");
  b.n = (uint32_t)n;
  if (!ranges || !image || !final_T || !n_contrib || !last_contrib) return fail(GS_EINVAL, "NULL argument");
  if (n > 0 && (!means2d || !conic_opacity || !rgb || !vals)) return fail(GS_EINVAL, "NULL splat argument");
  if ((means2d && !aligned(means2d, 8)) || (conic_opacity && !aligned(conic_opacity, 16)))
    return fail(GS_EINVAL, "means2d needs 8-byte, conic_opacity 16-byte alignment");
  BlendOut o{image, final_T, n_contrib, last_contrib, n_eval, nullptr};
  return check_hip(
      launch_blend_fwd_mfma(b, means2d, conic_opacity, rgb, vals, ranges, tile_order, o, (hipStream_t)stream),
      "gs_rasterize_fwd_mfma launch");
}

gs_status gs_rasterize_fwd_count(const gs_camera *cam, const gs_kernel *kernel, const gs_params *params, int64_t n,
                                 const float *means2d, const float *conic_opacity, const float *rgb,
                                 const uint32_t *vals, const uint32_t *ranges, const uint32_t *tile_order,
                                 float *image, float *final_T, uint32_t *n_contrib, uint32_t *last_contrib,
                                 uint32_t *n_eval, uint32_t *n_tested, void *stream) {
  BlendParams b;
  gs_status st = make_blend(cam, kernel, params, &b);
  if (st != GS_OK) return st;
  if (n < 0 || n >= (1ll << 31)) return fail(GS_EINVAL, "n outside [0, 2^31)");
  b.n = (uint32_t)n;
  if (!ranges || !image || !final_T || !n_contrib || !last_contrib || !n_tested)
    return fail(GS_EINVAL, "NULL argument");
  if (n > 0 && (!means2d || !conic_opacity || !rgb || !vals)) return fail(GS_EINVAL, "NULL splat argument");
  if ((means2d && !aligned(means2d, 8)) || (conic_opacity && !aligned(conic_opacity, 16)))
    return fail(GS_EINVAL, "means2d needs 8-byte, conic_opacity 16-byte alignment");
  BlendOut o{image, final_T, n_contrib, last_contrib, n_eval, n_tested};
  return check_hip(launch_blend_fwd(b, means2d, conic_opacity, rgb, vals, ranges, tile_order, o, (hipStream_t)stream),
                   "gs_rasterize_fwd_count launch");
}

gs_status gs_rasterize_bwd(const gs_camera *cam, const gs_kernel *kernel, const gs_params *params, int64_t n,
                           const float *means2d, const float *conic_opacity, const float *rgb,
                           const uint32_t *vals, const uint32_t *ranges, const uint32_t *tile_order,
                           const float *final_T, const uint32_t *last_contrib, const float *dL_dimage,
                           float *dL_dmeans2d, float *dL_dconic_opacity, float *dL_drgb, void *stream) {
  BlendParams b;
  gs_status st = make_blend(cam, kernel, params, &b);
  if (st != GS_OK) return st;
  if (n < 0 || n >= (1ll << 31)) return fail(GS_EINVAL, "n outside [0, 2^31)");
  b.n = (uint32_t)n;
  if (!ranges || !final_T || !last_contrib || !dL_dimage) return fail(GS_EINVAL, "NULL argument");
  if (n > 0 && (!means2d || !conic_opacity || !rgb || !vals || !dL_dmeans2d || !dL_dconic_opacity || !dL_drgb))
    return fail(GS_EINVAL, "NULL splat argument");
  if ((means2d && !aligned(means2d, 8)) || (conic_opacity && !aligned(conic_opacity, 16)) ||
      (dL_dmeans2d && !aligned(dL_dmeans2d, 8)) || (dL_dconic_opacity && !aligned(dL_dconic_opacity, 16)))
    return fail(GS_EINVAL, "2D records need 8 (means) and 16 (conic_opacity) byte alignment");
  return check_hip(launch_blend_bwd(b, n, means2d, conic_opacity, rgb, vals, ranges, tile_order, final_T, last_contrib,
                                    dL_dimage, dL_dmeans2d, dL_dconic_opacity, dL_drgb, (hipStream_t)stream),
                   "gs_rasterize_bwd launch");
}

gs_status gs_preprocess_bwd(const gs_camera *cam, const gs_kernel *kernel, const gs_params *params, int64_t n,
                            const float *means3d, const float *scales, const float *quats,
                            const float *opacities, const float *sh, int32_t sh_degree,
                            const uint32_t *tiles_touched, const float *dL_dmeans2d,
                            const float *dL_dconic_opacity, const float *dL_drgb, float *dL_dmeans3d,
                            float *dL_dscales, float *dL_dquats, float *dL_dopacities, float *dL_dsh,
                            void *stream) {
  gs_status st;
  if ((st = check_camera(cam)) != GS_OK || (st = check_params(params)) != GS_OK) return st;
  Resolved r;
  if ((st = resolve_kernel(kernel, &r)) != GS_OK) return st;
  if (n < 0 || n >= (1ll << 31)) return fail(GS_EINVAL, "n outside [0, 2^31)");
  if (sh_degree < 0 || sh_degree > 3) return fail(GS_EINVAL, "sh_degree %d outside 0..3", sh_degree);
  if (n == 0) return GS_OK;
  if (!means3d || !scales || !quats || !opacities || !sh || !tiles_touched || !dL_dmeans2d || !dL_dconic_opacity ||
      !dL_drgb || !dL_dmeans3d || !dL_dscales || !dL_dquats || !dL_dopacities || !dL_dsh)
    return fail(GS_EINVAL, "NULL array argument");
  if (!aligned(dL_dmeans2d, 8) || !aligned(dL_dconic_opacity, 16))
    return fail(GS_EINVAL, "2D gradients need 8 (means) and 16 (conic_opacity) byte alignment");
  PreParams p;
  std::memset(&p, 0, sizeof(p));
  make_cam(cam, params->tile, &p.cam);
  p.radius_mode = r.radius_mode;
  p.order = r.order;
  p.sh_degree = sh_degree;
  p.tile = params->tile;
  p.rect_mode = params->rect_mode;
  for (int i = 0; i < 4; ++i) p.c[i] = r.c[i];
  p.k_universal = std::sqrt(r.x0);
  p.eps = params->eps;
  p.aa_v = params->aa_v;
  p.near_z = params->near_z;
  p.pad = params->radius_pad;
  return check_hip(launch_preprocess_bwd(p, n, means3d, scales, quats, opacities, sh, tiles_touched, dL_dmeans2d,
                                         dL_dconic_opacity, dL_drgb, dL_dmeans3d, dL_dscales, dL_dquats,
                                         dL_dopacities, dL_dsh, (hipStream_t)stream),
                   "gs_preprocess_bwd launch");
}

static gs_status batch_check(const gs_scene *scenes, int32_t num_scenes, const gs_view *views, int32_t num_views,
                             int64_t key_capacity, int64_t *pairs, int32_t *gw, int32_t *gh) {
  if (!scenes || !views) return fail(GS_EINVAL, "NULL scenes or views");
  if (num_scenes < 1 || num_scenes > 16) return fail(GS_EUNSUPPORTED, "num_scenes %d outside 1..16", num_scenes);
  if (num_views < 1 || num_views > 4096) return fail(GS_EUNSUPPORTED, "num_views %d outside 1..4096", num_views);
  if (key_capacity < 0 || key_capacity >= (1ll << 32)) return fail(GS_EINVAL, "key_capacity outside [0, 2^32)");
  for (int i = 0; i < num_scenes; ++i) {
    const gs_scene &sc = scenes[i];
    if (sc.n < 0 || sc.n >= (1ll << 31)) return fail(GS_EINVAL, "scene %d: n outside [0, 2^31)", i);
    if (sc.sh_degree < 0 || sc.sh_degree > 3) return fail(GS_EINVAL, "scene %d: sh_degree outside 0..3", i);
    if (sc.sh_degree != scenes[0].sh_degree) return fail(GS_EUNSUPPORTED, "scenes must share one sh_degree");
    if (sc.reserved != 0) return fail(GS_EINVAL, "scene %d: reserved must be 0", i);
    if (sc.n > 0 && (!sc.means3d || !sc.scales || !sc.quats || !sc.opacities || !sc.sh))
      return fail(GS_EINVAL, "scene %d: NULL array", i);
    if (sc.n > 0 && !aligned(sc.sh, 16)) return fail(GS_EINVAL, "scene %d: sh needs 16-byte alignment", i);
  }
  int64_t p = 0, rows = 0;
  int32_t cols = 1;
  for (int v = 0; v < num_views; ++v) {
    gs_status st = check_camera(&views[v].cam);
    if (st != GS_OK) return st;
    if (views[v].scene < 0 || views[v].scene >= num_scenes) return fail(GS_EINVAL, "view %d: scene index", v);
    if (views[v].reserved != 0) return fail(GS_EINVAL, "view %d: reserved must be 0", v);
    p += (scenes[views[v].scene].n + 63) / 64 * 64;
    rows += (views[v].cam.height + 15) / 16;
    const int32_t gxv = (views[v].cam.width + 15) / 16;
    cols = gxv > cols ? gxv : cols;
  }
  if (p >= (1ll << 31)) return fail(GS_EUNSUPPORTED, "%lld pairs: more than 2^31", (long long)p);
  if (rows * cols > (1ll << 30)) return fail(GS_EUNSUPPORTED, "virtual tile grid too large");
  *pairs = p;
  *gw = cols;
  *gh = (int32_t)rows;
  return GS_OK;
}

gs_status gs_batch_layout(const gs_scene *scenes, int32_t num_scenes, const gs_view *views, int32_t num_views,
                          int64_t key_capacity, int64_t *num_pairs, int32_t *grid_w, int32_t *grid_h,
                          size_t *workspace_bytes) {
  if (!num_pairs || !grid_w || !grid_h || !workspace_bytes) return fail(GS_EINVAL, "NULL output");
  int64_t p;
  int32_t gw, gh;
  gs_status st = batch_check(scenes, num_scenes, views, num_views, key_capacity, &p, &gw, &gh);
  if (st != GS_OK) return st;
  *num_pairs = p;
  *grid_w = gw;
  *grid_h = gh;
  *workspace_bytes = batch_workspace_bytes(num_views, p, gw, gh, key_capacity);
  return GS_OK;
}

gs_status gs_render_batched(const gs_kernel *kernel, const gs_params *params, const gs_scene *scenes,
                            int32_t num_scenes, const gs_view *views, const gs_view *views_device,
                            int32_t num_views, int64_t key_capacity, int32_t workgroups, void *workspace,
                            size_t workspace_bytes, float *images, int64_t images_len, float *final_T,
                            uint32_t *n_contrib, uint32_t *last_contrib, int64_t planes_len, int64_t *num_keys,
                            int32_t *overflow, int64_t *view_keys, void *stream) {
  gs_status st;
  if ((st = check_params(params)) != GS_OK) return st;
  Resolved r;
  if ((st = resolve_kernel(kernel, &r)) != GS_OK) return st;
  int64_t pairs;
  int32_t gw, gh;
  if ((st = batch_check(scenes, num_scenes, views, num_views, key_capacity, &pairs, &gw, &gh)) != GS_OK) return st;
  if (!views_device || !workspace || !images || !final_T || !n_contrib || !last_contrib || !num_keys || !overflow)
    return fail(GS_EINVAL, "NULL argument");
  if (workgroups < 0 || workgroups > 65536) return fail(GS_EINVAL, "workgroups outside 0..65536");
  const size_t need = batch_workspace_bytes(num_views, pairs, gw, gh, key_capacity);
  if (workspace_bytes < need) return fail(GS_EINVAL, "workspace of %zu bytes is smaller than the %zu needed",
                                          workspace_bytes, need);
  if (!aligned(workspace, 256)) return fail(GS_EINVAL, "workspace needs 256-byte alignment");
  for (int v = 0; v < num_views; ++v) {
    const int64_t WH = (int64_t)views[v].cam.width * views[v].cam.height;
    if (views[v].image_offset < 0 || views[v].image_offset + 3 * WH > images_len || views[v].pixel_offset < 0 ||
        views[v].pixel_offset + WH > planes_len)
      return fail(GS_EINVAL, "view %d: output range outside the buffers", v);
  }
  PreParams p;
  std::memset(&p, 0, sizeof(p));
  p.radius_mode = r.radius_mode;
  p.order = r.order;
  p.sh_degree = scenes[0].sh_degree;
  p.tile = params->tile;
  p.rect_mode = params->rect_mode;
  for (int i = 0; i < 4; ++i) p.c[i] = r.c[i];
  p.k_universal = std::sqrt(r.x0);
  p.eps = params->eps;
  p.aa_v = params->aa_v;
  p.near_z = params->near_z;
  p.pad = params->radius_pad;
  BlendParams b;
  std::memset(&b, 0, sizeof(b));
  b.n = (uint32_t)pairs;
  b.blend = blend_kind(r);
  for (int i = 0; i < 4; ++i) b.c[i] = (float)r.c[i];
  b.x0 = (float)r.x0;
  b.eps = params->eps;
  b.log2_eps = std::log2(params->eps);
  b.alpha_max = params->alpha_max;
  b.t_min = params->t_min;
  for (int i = 0; i < 3; ++i) b.bg[i] = params->bg[i];
  b.threads = params->blend_threads ? params->blend_threads : 256;
  b.stage = params->blend_stage ? params->blend_stage : 2;
  return check_hip(launch_batch(p, b, scenes, num_scenes, views_device, num_views, pairs, gw, gh, key_capacity,
                                workgroups, workspace, images, images_len, final_T, n_contrib, last_contrib,
                                planes_len, num_keys, overflow, view_keys, (hipStream_t)stream),
                   "gs_render_batched launch");
}

}  // extern "C"
