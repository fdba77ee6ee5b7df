// Per-splat projection: EWA covariance, anti-aliasing, conic, bounding radius
// (3 sigma, universal or opacity-dependent polynomial root, exponential
// opacity bound), tile rectangle and spherical-harmonic colour.
//
// One thread per splat. The geometry that decides discrete outcomes (depth,
// culls, radius, rectangle) runs in double precision from the float inputs so
// that depth keys and rectangles are reproducible; the record the blender
// reads is rounded to float at the end. The stage is bound by HBM traffic
// (236 B in, 48 B out per splat at SH degree 3), not by the FP64 arithmetic.
#include <cmath>

#include "gs_internal.h"
#include "project_common.h"

namespace gs {

namespace {

// One wave per 64 splats: geometry per lane, then the wave stages its
// splats' SH coefficients (a contiguous block) through LDS chunk by chunk with
// coalesced loads; reading 48 floats per lane straight from global memory
// would touch 64 cache lines per load instruction.
template <int DEG>
__global__ __launch_bounds__(64) void preprocess_kernel(PreParams p, int64_t n, const float *__restrict__ means3d,
                                                        const float *__restrict__ scales,
                                                        const float *__restrict__ quats,
                                                        const float *__restrict__ opac,
                                                        const float *__restrict__ sh, PreOut out) {
  __shared__ float shs[64 * SH_ROW];
  const int64_t base = (int64_t)blockIdx.x * 64;
  const int64_t i = base + threadIdx.x;
  float Y[16];
  bool live = false;
  if (i < n) live = project_one<DEG>(p, i, means3d, scales, quats, opac, i, 0, out, Y);
  const float3 c = sh_colour_block<DEG>(sh, base, n, live, Y, shs);
  if (i < n) {
    out.rgb[3 * i] = c.x;
    out.rgb[3 * i + 1] = c.y;
    out.rgb[3 * i + 2] = c.z;
  }
}

}  // namespace

hipError_t launch_preprocess(const PreParams &p, int64_t n, const float *means3d, const float *scales,
                             const float *quats, const float *opac, const float *sh, PreOut out,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 grid(ceil_div(n, 64)), block(64);
  switch (p.sh_degree) {
    case 0:
      hipLaunchKernelGGL(preprocess_kernel<0>, grid, block, 0, s, p, n, means3d, scales, quats, opac, sh, out);
      break;
    case 1:
      hipLaunchKernelGGL(preprocess_kernel<1>, grid, block, 0, s, p, n, means3d, scales, quats, opac, sh, out);
      break;
    case 2:
      hipLaunchKernelGGL(preprocess_kernel<2>, grid, block, 0, s, p, n, means3d, scales, quats, opac, sh, out);
      break;
    default:
      hipLaunchKernelGGL(preprocess_kernel<3>, grid, block, 0, s, p, n, means3d, scales, quats, opac, sh, out);
      break;
  }
  return hipGetLastError();
}

}  // namespace gs
