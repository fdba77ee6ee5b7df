// Front-to-back blending of the sorted per-tile splat lists.
//
// One workgroup of NT threads (64, 128 or 256: a launch parameter) per 16x16
// tile, P = 256 / NT pixels per lane. Each wave shades a compact block of the
// tile (an 8x8 quarter with 256 threads, an 8x16 half with 128, the whole
// tile with 64); a lane's P pixels share a column. The tile's list is walked
// in batches of NT x SB (SB = 1 or 2 records per lane, a launch parameter);
// each lane gathers its records, folds the kernel's constants into them and
// stages them in LDS, then every lane reads the batch by broadcast.
//
// Every kernel here is decreasing in the quadric Q on the part of its support
// that matters, so "alpha >= eps" is the same decision as "Q <= x_e", where
// x_e is the splat's opacity threshold: the root of o' p(x) = eps for a
// polynomial (App. B) or 2 ln(o'/eps) for the exponential (Sec. 3.2, Eq. 3).
// The inner loop therefore computes t = x_e - Q per pixel (a few FMAs, exact
// differences d = pixel - mean) and evaluates the kernel itself only where
// t >= 0. With t:
//   poly order 1:  alpha = eps + (-o' c_1) t                       (one FMA)
//   exp:           alpha = eps * 2^(t log2(e) / 2)                 (FMA + v_exp)
//   poly 2, 3:     alpha = o' p(x_e - t) by Horner; Q <= x_e < x_0, so the
//                  first-root cut of Eq. 6 never applies to a passing pair.
//
// The region t >= 0 is an ellipse, and the tighter x_e (the point of the
// opacity-dependent radius, Sec. 3.2) the smaller it is. While staging, each
// record gets a conservative box around that ellipse and a bit per wave
// telling whether the box meets the wave's pixel block; each wave then walks
// only its own records, in list order, eight per step with one branch per step.
// Skipped records cannot pass, so the images are those of a walk over the
// whole list.
#include <cmath>

#include "blend_common.h"
#include "gs_internal.h"

namespace gs {

namespace {

template <int KIND, int NT, bool COUNT, int SB>
__global__ __launch_bounds__(NT) void blend_fwd(BlendParams p, const float *__restrict__ means2d,
                                                const float *__restrict__ conic_opacity,
                                                const float *__restrict__ rgb, const uint32_t *__restrict__ vals,
                                                const uint32_t *__restrict__ ranges,
                                                const uint32_t *__restrict__ tile_order, BlendOut out) {
  const int ntiles = p.gx * p.gy;
  if ((int)blockIdx.x >= ntiles) return;
  const int tile = tile_order ? (int)min(tile_order[blockIdx.x], (uint32_t)(ntiles - 1)) : (int)blockIdx.x;
  blend_tile<KIND, NT, COUNT, SB>(p, tile % p.gx, tile / p.gx, ranges[2 * tile], ranges[2 * tile + 1], means2d, conic_opacity,
                       rgb, vals, out);
}

template <int KIND, bool COUNT, int SB>
void launch_stage(const BlendParams &p, const float *means2d, const float *conic_opacity, const float *rgb,
                  const uint32_t *vals, const uint32_t *ranges, const uint32_t *order, BlendOut out, hipStream_t s) {
  const dim3 grid(p.gx * p.gy);
  if (p.threads == 64)
    hipLaunchKernelGGL((blend_fwd<KIND, 64, COUNT, SB>), grid, dim3(64), 0, s, p, means2d, conic_opacity, rgb, vals,
                       ranges, order, out);
  else if (p.threads == 128)
    hipLaunchKernelGGL((blend_fwd<KIND, 128, COUNT, SB>), grid, dim3(128), 0, s, p, means2d, conic_opacity, rgb,
                       vals, ranges, order, out);
  else
    hipLaunchKernelGGL((blend_fwd<KIND, 256, COUNT, SB>), grid, dim3(256), 0, s, p, means2d, conic_opacity, rgb,
                       vals, ranges, order, out);
}

template <int KIND, bool COUNT>
hipError_t launch_shape(const BlendParams &p, const float *means2d, const float *conic_opacity, const float *rgb,
                        const uint32_t *vals, const uint32_t *ranges, const uint32_t *order, BlendOut out,
                        hipStream_t s) {
  if (p.stage == 1)
    launch_stage<KIND, COUNT, 1>(p, means2d, conic_opacity, rgb, vals, ranges, order, out, s);
  else
    launch_stage<KIND, COUNT, 2>(p, means2d, conic_opacity, rgb, vals, ranges, order, out, s);
  return hipGetLastError();
}

template <int KIND>
hipError_t launch_kind(const BlendParams &p, const float *means2d, const float *conic_opacity, const float *rgb,
                       const uint32_t *vals, const uint32_t *ranges, const uint32_t *order, BlendOut out,
                       hipStream_t s) {
  if (out.n_tested) return launch_shape<KIND, true>(p, means2d, conic_opacity, rgb, vals, ranges, order, out, s);
  return launch_shape<KIND, false>(p, means2d, conic_opacity, rgb, vals, ranges, order, out, s);
}

}  // namespace

int blend_kind(const Resolved &r) {
  if (r.kind == GS_KERNEL_EXP) return BLEND_EXP;
  return r.order == 1 ? BLEND_POLY1 : (r.order == 2 ? BLEND_POLY2 : BLEND_POLY3);
}

hipError_t launch_blend_fwd(const BlendParams &p, const float *means2d, const float *conic_opacity,
                            const float *rgb, const uint32_t *vals, const uint32_t *ranges,
                            const uint32_t *tile_order, BlendOut out, hipStream_t s) {
  switch (p.blend) {
    case BLEND_EXP:
      return launch_kind<BLEND_EXP>(p, means2d, conic_opacity, rgb, vals, ranges, tile_order, out, s);
    case BLEND_POLY1:
      return launch_kind<BLEND_POLY1>(p, means2d, conic_opacity, rgb, vals, ranges, tile_order, out, s);
    case BLEND_POLY2:
      return launch_kind<BLEND_POLY2>(p, means2d, conic_opacity, rgb, vals, ranges, tile_order, out, s);
    default:
      return launch_kind<BLEND_POLY3>(p, means2d, conic_opacity, rgb, vals, ranges, tile_order, out, s);
  }
}

}  // namespace gs
