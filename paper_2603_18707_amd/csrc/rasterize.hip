// Front-to-back blending of the sorted per-tile splat lists.
//
// One workgroup of NT threads (64, 128 or 256: a launch parameter) per 16x16
// tile, P = 256 / NT pixels per lane: lane l owns column l % 16 and rows
// l / 16 + (NT / 16) k, k < P. The tile's list is walked in batches of NT;
// each lane gathers one splat record, folds the kernel's constants into it and
// stages it in LDS, then every lane reads the batch by broadcast, so one LDS
// read of a record serves P pixels.
//
// Every kernel here is decreasing in the quadric Q on the part of its support
// that matters, so "alpha >= eps" is the same decision as "Q <= x_e", where
// x_e is the splat's opacity threshold: the root of o' p(x) = eps for a
// polynomial (App. B) or 2 ln(o'/eps) for the exponential (Sec. 3.2, Eq. 3).
// The inner loop therefore computes t = x_e - Q for the four pixels (a few
// FMAs, exact differences d = pixel - mean) and evaluates the kernel itself
// only where t >= 0. With t:
//   poly order 1:  alpha = eps + (-o' c_1) t                       (one FMA)
//   exp:           alpha = eps * 2^(t log2(e) / 2)                 (FMA + v_exp)
//   poly 2, 3:     alpha = o' p(x_e - t) by Horner; Q <= x_e < x_0, so the
//                  first-root cut of Eq. 6 never applies to a passing pair.
// Pairs below the threshold, the vast majority when splats are small, cost the
// same for every kernel; the kernels differ in how many pairs culling leaves
// and in the arithmetic of the pairs that blend.
//
// A lane's rows are NT / 16 apart, so a small splat's footprint falls in one
// or two of its per-pixel branches and divergence stays low.
#include <cmath>

#include "blend_common.h"
#include "gs_internal.h"

namespace gs {

namespace {

template <int KIND, int NT>
__global__ __launch_bounds__(NT) void blend_fwd(BlendParams p, const float *__restrict__ means2d,
                                                const float *__restrict__ conic_opacity,
                                                const float *__restrict__ rgb, const uint32_t *__restrict__ vals,
                                                const uint32_t *__restrict__ ranges, BlendOut out) {
  constexpr int P = TS * TS / NT;   // pixels per lane
  constexpr int RS = NT / TS;       // row stride between a lane's pixels
  __shared__ float4 L0[NT], L1[NT], L2[NT];
  const int ntiles = p.gx * p.gy;
  const int tile = blockIdx.x;
  if (tile >= ntiles) return;
  const int lane = threadIdx.x;
  const int tx = tile % p.gx, ty = tile / p.gx;
  const int px = tx * TS + (lane & (TS - 1));
  const int py0 = ty * TS + lane / TS;
  const float fx = (float)px + 0.5f;
  float fy[P], T[P], C0[P], C1[P], C2[P];
  uint32_t ncon[P], last[P], nev[P];
  bool alive[P];
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    fy[k] = (float)(py0 + RS * k) + 0.5f;
    T[k] = 1.0f;
    C0[k] = C1[k] = C2[k] = 0.0f;
    ncon[k] = last[k] = 0u;
    nev[k] = end - start;
    alive[k] = px < p.W && (py0 + RS * k) < p.H;
  }

  for (uint32_t b = start; b < end; b += NT) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < P; ++k) any = any || alive[k];
    if (__syncthreads_or(any) == 0) break;  // every pixel of the tile has terminated
    const uint32_t idx = b + lane;
    if (idx < end) {
      uint32_t id = vals[idx];
      if (id >= p.n) id = 0;  // never taken for a list built by gs_bin_sort over these n splats
      const float2 m = reinterpret_cast<const float2 *>(means2d)[id];
      const float4 co = reinterpret_cast<const float4 *>(conic_opacity)[id];
      const float3 c = make_float3(rgb[3 * id], rgb[3 * id + 1], rgb[3 * id + 2]);
      float4 a0, a1, a2;
      fold<KIND>(m, co, c, p, a0, a1, a2);
      L0[lane] = a0;
      L1[lane] = a1;
      L2[lane] = a2;
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)NT, end - b);
    if (any) {
      for (int j = 0; j < cnt; ++j) {
        const float4 r0 = L0[j];
        const float4 r1 = L1[j];
        const float dx = fx - r0.x;
        const float adx = r0.z * dx;
        const float R0 = fmaf(-adx, dx, r1.y);
        const float Pq = r0.w * dx;
        float t[P];
        float mx = -1.0f;
#pragma unroll
        for (int k = 0; k < P; ++k) {
          const float dy = fy[k] - r0.y;
          t[k] = fmaf(-dy, fmaf(r1.x, dy, Pq), R0);
          mx = fmaxf(mx, t[k]);
        }
        if (mx >= 0.0f) {
          const uint32_t pos = b + j - start + 1;
#pragma unroll
          for (int k = 0; k < P; ++k) {
            if (t[k] >= 0.0f && alive[k]) {
              const float a = alpha_from<KIND>(t[k], r1, p);
              const float Tn = T[k] * (1.0f - a);
              if (Tn < p.t_min) {
                alive[k] = false;
                nev[k] = pos;
              } else {
                const float4 r2 = L2[j];
                const float w = a * T[k];
                C0[k] = fmaf(r2.x, w, C0[k]);
                C1[k] = fmaf(r2.y, w, C1[k]);
                C2[k] = fmaf(r2.z, w, C2[k]);
                T[k] = Tn;
                ++ncon[k];
                last[k] = pos;
              }
            }
          }
        }
      }
    }
    __syncthreads();
  }
  const size_t plane = (size_t)p.W * p.H;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int py = py0 + RS * k;
    if (px >= p.W || py >= p.H) continue;
    const size_t pix = (size_t)py * p.W + px;
    out.image[pix] = fmaf(T[k], p.bg[0], C0[k]);
    out.image[plane + pix] = fmaf(T[k], p.bg[1], C1[k]);
    out.image[2 * plane + pix] = fmaf(T[k], p.bg[2], C2[k]);
    out.final_T[pix] = T[k];
    out.n_contrib[pix] = ncon[k];
    out.last_contrib[pix] = last[k];
    if (out.n_eval) out.n_eval[pix] = nev[k];
  }
}

template <int KIND>
hipError_t launch_kind(const BlendParams &p, const float *means2d, const float *conic_opacity, const float *rgb,
                       const uint32_t *vals, const uint32_t *ranges, BlendOut out, hipStream_t s) {
  const dim3 grid(p.gx * p.gy);
  if (p.threads == 64)
    hipLaunchKernelGGL((blend_fwd<KIND, 64>), grid, dim3(64), 0, s, p, means2d, conic_opacity, rgb, vals, ranges,
                       out);
  else if (p.threads == 128)
    hipLaunchKernelGGL((blend_fwd<KIND, 128>), grid, dim3(128), 0, s, p, means2d, conic_opacity, rgb, vals, ranges,
                       out);
  else
    hipLaunchKernelGGL((blend_fwd<KIND, 256>), grid, dim3(256), 0, s, p, means2d, conic_opacity, rgb, vals, ranges,
                       out);
  return hipGetLastError();
}

}  // namespace

int blend_kind(const Resolved &r) {
  if (r.kind == GS_KERNEL_EXP) return BLEND_EXP;
  return r.order == 1 ? BLEND_POLY1 : (r.order == 2 ? BLEND_POLY2 : BLEND_POLY3);
}

hipError_t launch_blend_fwd(const BlendParams &p, const float *means2d, const float *conic_opacity,
                            const float *rgb, const uint32_t *vals, const uint32_t *ranges, BlendOut out,
                            hipStream_t s) {
  switch (p.blend) {
    case BLEND_EXP:
      return launch_kind<BLEND_EXP>(p, means2d, conic_opacity, rgb, vals, ranges, out, s);
    case BLEND_POLY1:
      return launch_kind<BLEND_POLY1>(p, means2d, conic_opacity, rgb, vals, ranges, out, s);
    case BLEND_POLY2:
      return launch_kind<BLEND_POLY2>(p, means2d, conic_opacity, rgb, vals, ranges, out, s);
    default:
      return launch_kind<BLEND_POLY3>(p, means2d, conic_opacity, rgb, vals, ranges, out, s);
  }
}

}  // namespace gs
