// Per-splat projection: EWA covariance, anti-aliasing, conic, bounding radius
// (3 sigma, universal or opacity-dependent polynomial root, exponential
// opacity bound), tile rectangle and spherical-harmonic colour.
//
// One thread per splat. The geometry that decides discrete outcomes (depth,
// culls, radius, rectangle) runs in double precision from the float inputs so
// that depth keys and rectangles are reproducible; the record the blender
// reads is rounded to float at the end. The stage is bound by HBM traffic
// (236 B in, 60 B out per splat at SH degree 3), not by the FP64 arithmetic.
#include <cmath>

#include "gs_internal.h"
#include "project_common.h"

namespace gs {

namespace {

// One thread per splat (64-thread workgroups).
template <int DEG>
__global__ __launch_bounds__(64) void preprocess_kernel(PreParams p, int64_t n, const float *__restrict__ means3d,
                                                        const float *__restrict__ scales,
                                                        const float *__restrict__ quats,
                                                        const float *__restrict__ opac,
                                                        const float *__restrict__ sh, PreOut out) {
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  float Y[16];
  const bool live = project_one<DEG>(p, i, means3d, scales, quats, opac, i, 0, out, Y);
  const float3 c = sh_colour<DEG>(sh, i, live, Y);
  out.rgb[3 * i] = c.x;
  out.rgb[3 * i + 1] = c.y;
  out.rgb[3 * i + 2] = c.z;
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
