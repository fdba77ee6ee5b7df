// Internal declarations shared by the libgs translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "gs.h"

namespace gs {

// ---------------------------------------------------------------------------
// kernel description resolved on the host
// ---------------------------------------------------------------------------
enum BlendKind : int { BLEND_EXP = 0, BLEND_POLY1 = 1, BLEND_POLY2 = 2, BLEND_POLY3 = 3 };

struct Resolved {
  int kind;          // GS_KERNEL_*
  int order;         // 1..3
  int radius_mode;   // GS_RADIUS_*
  double c[4];       // polynomial coefficients (zero above order)
  double x0;         // first positive root of the polynomial (0 if unused)
};

// fills r from a public gs_kernel; returns GS_OK or an error (message set)
gs_status resolve_kernel(const gs_kernel *k, Resolved *r);

// error reporting (thread-local message)
gs_status fail(gs_status s, const char *fmt, ...);
gs_status check_hip(hipError_t e, const char *what);

// ---------------------------------------------------------------------------
// preprocess
// ---------------------------------------------------------------------------
struct CamD {
  double R[9], t[3];
  double fx, fy, cx, cy;
  double limx, limy;     // 1.3 * tan(half field of view), per axis
  double campos[3];      // camera centre in world space
  int W, H, gx, gy;
};

struct PreParams {
  CamD cam;
  int radius_mode, order, sh_degree, tile, rect_mode;
  double c[4];
  double k_universal;    // sqrt(x0) for POLY_UNIVERSAL
  double eps, aa_v, near_z, pad;
};

struct PreOut {
  float *means2d, *conic_opacity, *rgb, *depth;
  int32_t *rect;
  uint32_t *tiles;
};

// camera in double precision, with the Jacobian clamp limits and the centre
__host__ __device__ inline void make_cam(const gs_camera *c, int tile, CamD *o) {
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) o->R[3 * r + k] = (double)c->viewmat[4 * r + k];
    o->t[r] = (double)c->viewmat[4 * r + 3];
  }
  o->fx = c->fx;
  o->fy = c->fy;
  o->cx = c->cx;
  o->cy = c->cy;
  o->limx = 1.3 * (c->width / (2.0 * o->fx));
  o->limy = 1.3 * (c->height / (2.0 * o->fy));
  for (int i = 0; i < 3; ++i)
    o->campos[i] = -(o->R[i] * o->t[0] + o->R[3 + i] * o->t[1] + o->R[6 + i] * o->t[2]);
  o->W = c->width;
  o->H = c->height;
  o->gx = (c->width + tile - 1) / tile;
  o->gy = (c->height + tile - 1) / tile;
}

hipError_t launch_preprocess(const PreParams &p, int64_t n, const float *means3d, const float *scales,
                             const float *quats, const float *opac, const float *sh, PreOut out,
                             hipStream_t s);

// ---------------------------------------------------------------------------
// binning and sorting
// ---------------------------------------------------------------------------
size_t binsort_workspace_bytes(int64_t n, int64_t capacity, int32_t num_tiles);
hipError_t launch_binsort(int64_t n, const float *depth, const int32_t *rect, const uint32_t *tiles,
                          int grid_w, int grid_h, int64_t capacity, void *ws, size_t ws_bytes, uint64_t *keys,
                          uint32_t *vals, uint32_t *ranges, uint32_t *tile_order, int64_t *num_keys,
                          int32_t *overflow, hipStream_t s);

// ---------------------------------------------------------------------------
// blending
// ---------------------------------------------------------------------------
struct BlendParams {
  int W, H, gx, gy;
  uint32_t n;            // splats the values index
  int blend;             // BlendKind
  float c[4];            // polynomial coefficients in float
  float x0;              // order-2 cut
  float eps, alpha_max, t_min;
  float log2_eps;        // log2(eps), for the exponential's threshold
  int threads;           // blend workgroup size per tile: 64, 128 or 256
  int stage;             // records each thread stages per batch: 1 or 2
  float bg[3];
};

// launch_binsort with tile culling: a splat's copy for a tile of its
// rectangle is emitted only when some pixel centre of the tile may pass the
// blend's inclusion test (bp supplies the kernel, eps and the blend kind;
// means2d and conic_opacity are the projected records). Needs
// grid_w * grid_h < 2^22 and grid_w <= 32767.
hipError_t launch_binsort_culled(int64_t n, const float *depth, const int32_t *rect, const uint32_t *tiles,
                                 const float *means2d, const float *conic_opacity, const BlendParams &bp,
                                 int grid_w, int grid_h, int64_t capacity, void *ws, size_t ws_bytes, uint64_t *keys,
                                 uint32_t *vals, uint32_t *ranges, uint32_t *tile_order, int64_t *num_keys,
                                 int32_t *overflow, hipStream_t s);

struct BlendOut {
  float *image, *final_T;
  uint32_t *n_contrib, *last_contrib, *n_eval;
  uint32_t *n_tested;    // set only by the counting entry point
};

int blend_kind(const Resolved &r);
hipError_t launch_blend_fwd(const BlendParams &p, const float *means2d, const float *conic_opacity,
                            const float *rgb, const uint32_t *vals, const uint32_t *ranges,
                            const uint32_t *tile_order, BlendOut out, hipStream_t s);

// the same blend with the quadric as a matrix product on MFMA (256 threads per tile)
hipError_t launch_blend_fwd_mfma(const BlendParams &p, const float *means2d, const float *conic_opacity,
                                 const float *rgb, const uint32_t *vals, const uint32_t *ranges,
                                 const uint32_t *tile_order, BlendOut out, hipStream_t s);

hipError_t launch_blend_bwd(const BlendParams &p, int64_t n, const float *means2d, const float *conic_opacity,
                            const float *rgb, const uint32_t *vals, const uint32_t *ranges,
                            const uint32_t *tile_order,
                            const float *final_T, const uint32_t *last_contrib, const float *dL_dimage,
                            float *dmeans2d, float *dconic_opacity, float *drgb, hipStream_t s);

hipError_t launch_preprocess_bwd(const PreParams &p, int64_t n, const float *means3d, const float *scales,
                                 const float *quats, const float *opac, const float *sh, const uint32_t *tiles,
                                 const float *dmeans2d, const float *dconic_opacity, const float *drgb,
                                 float *dmeans3d, float *dscales, float *dquats, float *dopac, float *dsh,
                                 hipStream_t s);

// batched rendering
size_t batch_workspace_bytes(int nviews, int64_t pairs, int gw, int gh, int64_t capacity);
hipError_t launch_batch(const PreParams &pre, const BlendParams &blend, const gs_scene *scenes, int nscenes,
                        const gs_view *views_dev, int nviews, int64_t pairs, int gw, int gh, int64_t capacity,
                        int workgroups, void *ws, float *images, int64_t images_len, float *final_T,
                        uint32_t *n_contrib, uint32_t *last_contrib, int64_t planes_len, int64_t *num_keys,
                        int32_t *overflow, int64_t *view_keys, hipStream_t s);

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace gs
