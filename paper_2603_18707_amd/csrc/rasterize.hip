// Front-to-back blending of the sorted per-tile splat lists.
//
// One 256-thread workgroup per 16x16 tile, one pixel per thread; wave w owns
// rows 4w..4w+3 of the tile. The tile's list is walked in batches of 256: each
// thread gathers one splat record, folds the kernel's constants into it and
// stages it in LDS; every lane then reads the records by broadcast. A pixel
// leaves the loop at the splat that would push T below t_min; a wave leaves
// when all its lanes have, and the workgroup stops fetching batches once every
// pixel is done.
//
// Folding the kernel into the record removes per-evaluation work:
//   poly order 1:  alpha = o c_0 + Q (o c_1)           conic pre-scaled by o c_1
//   exp:           alpha = exp2(log2 o - Q log2(e)/2)   conic pre-scaled by -log2(e)/2
//   poly 2, 3:     alpha = o p(Q), Horner on the plain quadric
// so order 1 costs 7 VALU operations for alpha, exp costs 7 plus one v_exp.
//
// Workgroups are dispatched round-robin over the eight XCDs; tile indices are
// remapped so each XCD renders one contiguous band of tiles and its L2 holds
// the splat records that band shares.
#include "gs_internal.h"

namespace gs {

namespace {

constexpr int TS = 16;
constexpr int BS = TS * TS;
constexpr int NXCD = 8;

// staged record: r0 = (u, v, a', 2 b'), r1 = (c', K, r, g), r2 = b, with the
// conic (a, b, c) scaled by the kernel's factor and K its folded constant
template <int KIND>
__device__ inline void fold(float u, float v, float4 co, float3 c, const BlendParams &p, float4 &r0, float4 &r1,
                            float &r2) {
  float sc, k;
  if (KIND == BLEND_POLY1) {
    sc = co.w * p.c[1];
    k = co.w * p.c[0];
  } else if (KIND == BLEND_EXP) {
    sc = -0.72134752044448170f;  // -log2(e) / 2
    k = log2f(co.w);
  } else {
    sc = 1.0f;
    k = co.w;
  }
  r0 = make_float4(u, v, co.x * sc, 2.0f * co.y * sc);
  r1 = make_float4(co.z * sc, k, c.x, c.y);
  r2 = c.z;
}

template <int KIND>
__device__ inline float alpha_of(float dx, float dy, const float4 &r0, const float4 &r1, const BlendParams &p) {
  // quadric (pre-scaled for POLY1 / EXP) plus the folded constant
  if (KIND == BLEND_POLY1) {
    return fminf(p.alpha_max, fmaf(r1.x * dy, dy, fmaf(dx, fmaf(r0.z, dx, r0.w * dy), r1.y)));
  } else if (KIND == BLEND_EXP) {
    const float e = fmaf(r1.x * dy, dy, fmaf(dx, fmaf(r0.z, dx, r0.w * dy), r1.y));
    return fminf(p.alpha_max, __builtin_amdgcn_exp2f(e));
  } else {
    const float Q = fmaf(r1.x * dy, dy, dx * fmaf(r0.z, dx, r0.w * dy));
    float f;
    if (KIND == BLEND_POLY2) {
      f = fmaf(fmaf(p.c[2], Q, p.c[1]), Q, p.c[0]);
      f = (Q < p.x0) ? f : 0.0f;  // first-root cut of the quadratic
    } else {
      f = fmaf(fmaf(fmaf(p.c[3], Q, p.c[2]), Q, p.c[1]), Q, p.c[0]);
    }
    return fminf(p.alpha_max, r1.y * fmaxf(f, 0.0f));
  }
}

template <int KIND>
__global__ __launch_bounds__(BS) void blend_fwd(BlendParams p, const float *__restrict__ means2d,
                                                const float *__restrict__ conic_opacity,
                                                const float *__restrict__ rgb, const uint32_t *__restrict__ vals,
                                                const uint32_t *__restrict__ ranges, BlendOut out) {
  __shared__ float4 s0[BS];
  __shared__ float4 s1[BS];
  __shared__ float s2[BS];

  // XCD-aware mapping: block b runs on XCD b % 8; give each XCD a contiguous band
  const int ntiles = p.gx * p.gy;
  const int per = (ntiles + NXCD - 1) / NXCD;
  const int tile = (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
  if (tile >= ntiles) return;
  const int tx = tile % p.gx, ty = tile / p.gx;
  const int px = tx * TS + (threadIdx.x & (TS - 1));
  const int py = ty * TS + threadIdx.x / TS;
  const bool inside = px < p.W && py < p.H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;

  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  uint32_t ncon = 0, last = 0, nev = end - start;
  bool done = !inside;

  for (uint32_t b = start; b < end; b += BS) {
    if (__syncthreads_count(done) == BS) break;
    const uint32_t idx = b + threadIdx.x;
    if (idx < end) {
      uint32_t id = vals[idx];
      if (id >= p.n) id = 0;  // never taken for a list built by gs_bin_sort over these n splats
      const float2 m = reinterpret_cast<const float2 *>(means2d)[id];
      const float4 co = reinterpret_cast<const float4 *>(conic_opacity)[id];
      const float3 c = make_float3(rgb[3 * id], rgb[3 * id + 1], rgb[3 * id + 2]);
      float4 r0, r1;
      float r2;
      fold<KIND>(m.x, m.y, co, c, p, r0, r1, r2);
      s0[threadIdx.x] = r0;
      s1[threadIdx.x] = r1;
      s2[threadIdx.x] = r2;
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)BS, end - b);
    if (!done) {
      for (int j = 0; j < cnt; ++j) {
        const float4 r0 = s0[j];
        const float4 r1 = s1[j];
        const float dx = fx - r0.x, dy = fy - r0.y;
        const float a = alpha_of<KIND>(dx, dy, r0, r1, p);
        if (a < p.eps) continue;
        const float Tn = T * (1.0f - a);
        if (Tn < p.t_min) {
          done = true;
          nev = b + j - start + 1;
          break;
        }
        const float wgt = a * T;
        C0 = fmaf(r1.z, wgt, C0);
        C1 = fmaf(r1.w, wgt, C1);
        C2 = fmaf(s2[j], wgt, C2);
        T = Tn;
        ++ncon;
        last = b + j - start + 1;
      }
    }
  }
  if (!inside) return;
  const size_t pix = (size_t)py * p.W + px, plane = (size_t)p.W * p.H;
  out.image[pix] = fmaf(T, p.bg[0], C0);
  out.image[plane + pix] = fmaf(T, p.bg[1], C1);
  out.image[2 * plane + pix] = fmaf(T, p.bg[2], C2);
  out.final_T[pix] = T;
  out.n_contrib[pix] = ncon;
  out.last_contrib[pix] = last;
  if (out.n_eval) out.n_eval[pix] = nev;
}

}  // namespace

int blend_kind(const Resolved &r) {
  if (r.kind == GS_KERNEL_EXP) return BLEND_EXP;
  return r.order == 1 ? BLEND_POLY1 : (r.order == 2 ? BLEND_POLY2 : BLEND_POLY3);
}

hipError_t launch_blend_fwd(const BlendParams &p, const float *means2d, const float *conic_opacity,
                            const float *rgb, const uint32_t *vals, const uint32_t *ranges, BlendOut out,
                            hipStream_t s) {
  const int ntiles = p.gx * p.gy;
  const int per = (ntiles + NXCD - 1) / NXCD;
  const dim3 grid(per * NXCD), block(BS);
  switch (p.blend) {
    case BLEND_EXP:
      hipLaunchKernelGGL(blend_fwd<BLEND_EXP>, grid, block, 0, s, p, means2d, conic_opacity, rgb, vals, ranges, out);
      break;
    case BLEND_POLY1:
      hipLaunchKernelGGL(blend_fwd<BLEND_POLY1>, grid, block, 0, s, p, means2d, conic_opacity, rgb, vals, ranges,
                         out);
      break;
    case BLEND_POLY2:
      hipLaunchKernelGGL(blend_fwd<BLEND_POLY2>, grid, block, 0, s, p, means2d, conic_opacity, rgb, vals, ranges,
                         out);
      break;
    default:
      hipLaunchKernelGGL(blend_fwd<BLEND_POLY3>, grid, block, 0, s, p, means2d, conic_opacity, rgb, vals, ranges,
                         out);
      break;
  }
  return hipGetLastError();
}

}  // namespace gs
