// Device helpers shared by the blend kernels (forward and adjoint): tile
// geometry, the per-splat record staged in LDS and the kernel's threshold and
// alpha. Forward and backward use these same functions, so both take every
// inclusion decision identically.
#pragma once

#include <cmath>

#include "gs_internal.h"

namespace gs {

namespace {

constexpr int TS = 16;
constexpr int WAVE = 64;
constexpr int PIX = 4;  // pixels per lane

// first root of o p(x) = eps for orders 2 and 3, in double (App. B closed
// forms, Newton-polished); -1 when p(0) < eps / o
__device__ inline double opacity_root_d(const BlendParams &p, int order, float o) {
  if (!(o > 0.0f)) return -1.0;
  double c[4] = {p.c[0], p.c[1], p.c[2], p.c[3]};
  const double cc = c[0] - (double)p.eps / (double)o;
  if (cc < 0.0) return -1.0;
  double x;
  if (order == 2) {
    const double disc = c[1] * c[1] - 4.0 * cc * c[2];
    if (disc < 0.0) return -1.0;
    x = 2.0 * cc / (-c[1] + sqrt(disc));
  } else {
    const double d0 = c[2] * c[2] - 3.0 * c[3] * c[1];
    const double d1 = 2.0 * c[2] * c[2] * c[2] - 9.0 * c[3] * c[2] * c[1] + 27.0 * c[3] * c[3] * cc;
    const double s = d1 * d1 - 4.0 * d0 * d0 * d0;
    const double sq = sqrt(s > 0.0 ? s : 0.0);
    const double C = cbrt(d1 >= 0.0 ? 0.5 * (d1 + sq) : 0.5 * (d1 - sq));
    x = -(c[2] + C + d0 / C) / (3.0 * c[3]);
  }
  c[0] = cc;
  for (int it = 0; it < 2; ++it) {
    double f = c[order], fp = order * c[order];
    for (int i = order - 1; i >= 0; --i) {
      f = fma(f, x, c[i]);
      if (i >= 1) fp = fma(fp, x, i * c[i]);
    }
    if (fp != 0.0) x -= f / fp;
  }
  return x;
}
__device__ inline float opacity_threshold64(const BlendParams &p, int order, float o) {
  return (float)opacity_root_d(p, order, o);
}

// Staged record, positions relative to the tile's corner (x0, y0):
//   s0 = (u - x0, v - y0, g, h), s1 = (c, x_e, S, o'), s2 = (r, g, b, 0)
// with the quadratic form of the conic (a, b, c) completed in dy:
//   Q = a dx^2 + 2 b dx dy + c dy^2 = c (dy + h dx)^2 + g dx^2,
//   h = b / c, g = (a c - b^2) / c.
// For a positive-definite conic both terms are non-negative, so the float
// evaluation of t = x_e - Q suffers no cancellation: its error stays a few
// ulps of x_e and Q. Long, thin footprints make the expanded terms orders of
// magnitude larger than Q at pixels near their axis (1e5 against 1 in large
// scenes), and an expanded evaluation loses that many ulps. The tile-local
// positions keep the pixel offsets free of the rounding of absolute image
// coordinates. A conic that is not positive definite gets x_e = -1 and a zero
// quadric: it never passes.
// The quadric value up to which alpha = o' k(Q) >= eps: the threshold of
// the inclusion test t = x_e - Q >= 0 (-1 when no pixel can pass).
template <int KIND>
__device__ inline float alpha_threshold(const BlendParams &p, float o) {
  if (KIND == BLEND_POLY1) return (o * p.c[0] >= p.eps) ? (p.eps / o - p.c[0]) / p.c[1] : -1.0f;
  if (KIND == BLEND_EXP) return (o >= p.eps) ? 1.38629436111989061f * (log2f(o) - p.log2_eps) : -1.0f;  // 2 ln(o/eps)
  return opacity_threshold64(p, KIND == BLEND_POLY2 ? 2 : 3, o);
}

// Tile culling bound: the largest Q at which the blend can include any pixel
// of a record with opacity o and conic (a, b, c); negative when it includes
// none (opacity below the cut-off, or a conic that is not positive
// definite). Starting from the threshold thr of alpha >= eps in double, it
// adds (1) 2^-16 (|thr| + 16) for the float rounding of x_e (a few ulps of
// thr, or of the root scale when eps / o nearly equals c_0, and the log2
// approximation of the exponential), giving T, and (2) for the float
// evaluation of t = x_e - Q at a tile-local pixel: with u = 2^-24 the float
// inclusion t' >= 0 implies sqrt(Q) <= sqrt(T)(1 + 9u) + D', where
// D' <= u (4 sqrt(T) + 16 sqrt(g) + 7 |b| sqrt(T / det) + 16 |b| / sqrt(c)
// + 32 sqrt(c)) sums the rounding of the tile-local offsets (at most 16 px
// from the tile's corner plus the offset), of g and h (the reciprocal is
// within 1 ulp) and of the products forming e = dy + h dx and t. The bound
// takes 32 times D'. Rounding of the double evaluation itself is covered by
// a final factor 1 + 2^-30. Everything is rounded as written (no fused
// multiply-adds), so any double implementation of the same formula takes
// the same decisions.
__device__ inline double cull_cut(const BlendParams &p, float o, float a, float b, float c) {
#pragma clang fp contract(off)
  if (!(o > 0.0f) || !(a > 0.0f) || !(c > 0.0f)) return -1.0;
  const double A = a, B = b, C = c;
  const double det = A * C - B * B;
  if (!(det > 0.0)) return -1.0;
  double thr;
  switch (p.blend) {
    case BLEND_POLY1: thr = ((double)p.eps / (double)o - (double)p.c[0]) / (double)p.c[1]; break;
    case BLEND_EXP: thr = 2.0 * log((double)o / (double)p.eps); break;
    case BLEND_POLY2: thr = opacity_root_d(p, 2, o); break;
    default: thr = opacity_root_d(p, 3, o); break;
  }
  const double T = thr + 0x1p-16 * (fabs(thr) + 16.0);
  if (!(T >= 0.0)) return -1.0;
  const double sT = sqrt(T), aB = fabs(B);
  const double D = 0x1p-19 * (4.0 * sT + 16.0 * sqrt(det / C) + 8.0 * aB * sqrt(T / det) + 16.0 * aB / sqrt(C) +
                              32.0 * sqrt(C));
  const double r = sT * (1.0 + 0x1p-18) + D;
  return r * r * (1.0 + 0x1p-30);
}

template <int KIND>
__device__ inline void fold(float2 m, float4 co, float3 c, float x0, float y0, const BlendParams &p, float4 &s0,
                            float4 &s1, float4 &s2) {
  const float o = co.w;
  float xe = alpha_threshold<KIND>(p, o), S = 0.0f;
  if (KIND == BLEND_POLY1) S = -o * p.c[1];
  // a c - b^2 in double: both products of floats are exact there
  const double det = fma((double)co.x, (double)co.z, -((double)co.y * (double)co.y));
  const bool pd = co.x > 0.0f && co.z > 0.0f && det > 0.0;
  const float rc = __builtin_amdgcn_rcpf(co.z);
  s0 = make_float4(m.x - x0, m.y - y0, pd ? (float)(det * (double)rc) : 0.0f, pd ? co.y * rc : 0.0f);
  s1 = make_float4(pd ? co.z : 0.0f, pd ? xe : -1.0f, S, o);
  s2 = make_float4(c.x, c.y, c.z, 0.0f);
}

// t = x_e - Q of a staged record at the tile-local pixel (fx, fy), in the
// order both blend directions use (they must take identical decisions).
// The dx-only part is split out for loops that reuse it over a column.
struct RowPart {
  float h, R0;  // h dx - v, x_e - g dx^2
};
__device__ inline RowPart row_part(const float4 &s0, float s1y, float fx) {
  const float dx = fx - s0.x;
  return RowPart{fmaf(s0.w, dx, -s0.y), fmaf(-s0.z * dx, dx, s1y)};
}
__device__ inline float t_at(const RowPart &r, float s1x, float fy) {
  const float e = fy + r.h;  // dy + h dx
  return fmaf(-s1x * e, e, r.R0);
}

template <int KIND>
__device__ inline float alpha_from(float t, const float4 &s1, const BlendParams &p) {
  float a;
  if (KIND == BLEND_POLY1) {
    a = fmaf(s1.z, t, p.eps);
  } else if (KIND == BLEND_EXP) {
    a = __builtin_amdgcn_exp2f(fmaf(t, 0.72134752044448170f, p.log2_eps));
  } else {
    const float Q = s1.y - t;
    const float f = (KIND == BLEND_POLY2) ? fmaf(fmaf(p.c[2], Q, p.c[1]), Q, p.c[0])
                                          : fmaf(fmaf(fmaf(p.c[3], Q, p.c[2]), Q, p.c[1]), Q, p.c[0]);
    a = s1.w * f;
  }
  return fminf(a, p.alpha_max);
}

// Conservative box around the pixels a record can pass: the region
// t = x_e - Q >= 0 is an ellipse with half extents sqrt(x_e a / det) in y and
// sqrt(x_e c / det) in x (det = a c - b^2, in double from the float conic).
// The box is widened by a margin that covers the float rounding of t: near
// the edge, t falls with distance at a rate ~2 x_e / extent, and its rounding
// error is below a few ulps of the largest expanded term in the box.
// Records that never pass get an empty box; a margin too wide to matter
// leaves the box unbounded (no culling).
__device__ inline void pass_box(const float4 &co, float xe_f, float &hx, float &hy) {
  const double a = co.x, b = co.y, c = co.z, xe = xe_f;
  const double det = a * c - b * b;
  if (!(xe >= 0.0) || !(det > 0.0) || !(a > 0.0) || !(c > 0.0)) {
    hx = hy = -__builtin_inff();
    return;
  }
  hx = hy = __builtin_inff();
  if (!(xe > 1e-12)) return;
  const double ey = sqrt(xe * a / det), ex = sqrt(xe * c / det);
  const double big = (a + 2.0 * fabs(b) + c) * (ex + ey) * (ex + ey) + xe;
  const double rel = 1e-3 + 1e-6 * big / xe;
  if (rel > 0.05) return;
  hx = (float)(ex * (1.0 + rel) + 0.01);
  hy = (float)(ey * (1.0 + rel) + 0.01);
}

// Blends one 16x16 tile (tile coordinates tx, ty of an image of p.W x p.H
// pixels) over its sorted list [start, end) of splat indices into `out`
// (pointers to this image's planes). Called by NT threads of a workgroup.
//
// Splats are staged NT x SB at a time (SB per thread). Each staged record gets a bit per wave of
// the workgroup telling whether its pass box meets the pixel block that wave
// shades; every wave then walks a compacted list of its records, still in
// list order, so splats that cannot reach a wave's pixels cost it nothing.
//
// COUNT adds a per-pixel count of the kernel evaluations performed (entries
// of the wave's list while the pixel is alive, the one that stops it
// included), written to out.n_tested: a measurement build, not for rendering.
template <int KIND, int NT, bool COUNT = false, int SB = 1>
__device__ inline void blend_tile(const BlendParams &p, int tx, int ty, uint32_t start, uint32_t end,
                                  const float *__restrict__ means2d, const float *__restrict__ conic_opacity,
                                  const float *__restrict__ rgb, const uint32_t *__restrict__ vals,
                                  const BlendOut &out) {
  constexpr int P = TS * TS / NT;   // pixels per lane
  constexpr int NW = NT / WAVE;     // waves per workgroup
  // each wave shades a WX x WY block of the tile (8x8 of 4 waves, 8x16 of 2,
  // the whole tile for 1): compact blocks meet fewer splat boxes than strips
  constexpr int WX = NW == 1 ? 16 : 8;
  constexpr int WY = TS * TS / NW / WX;
  constexpr int RS = WAVE / WX;     // row stride between a lane's pixels
  constexpr int G = 8;              // splats tested per step
  constexpr int NB = NT * SB;       // records staged per batch (SB per thread)
  static_assert(NT % G == 0 && G == 8, "a staged batch holds whole steps of eight 16-bit slots");
  __shared__ float4 L0[NB + 1], L1[NB + 1], L2[NB + 1];   // slot NB: neutral record
  __shared__ __align__(16) uint16_t lst[NW][NB + G];  // rows of 16-byte multiples, read 8 slots at a time
  __shared__ uint32_t wcnt[SB][NW][NW];                  // [staging round][staging wave][shading wave]
  const int lane = threadIdx.x, wv = lane / WAVE;
  const uint64_t lt = (1ull << (lane & (WAVE - 1))) - 1ull;
  const int wx0 = (wv % (TS / WX)) * WX, wy0 = (wv / (TS / WX)) * WY;
  const int l64 = lane & (WAVE - 1);
  const int px = tx * TS + wx0 + l64 % WX;
  const int py0 = ty * TS + wy0 + l64 / WX;
  const float fx = (float)(wx0 + l64 % WX) + 0.5f;  // pixel centres relative to the tile corner
  float fy[P], T[P], C0[P], C1[P], C2[P];
  uint32_t ncon[P], last[P], nev[P], tested[P];
  bool alive[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    tested[k] = 0u;
    fy[k] = (float)(wy0 + l64 / WX + RS * k) + 0.5f;
    T[k] = 1.0f;
    C0[k] = C1[k] = C2[k] = 0.0f;
    ncon[k] = last[k] = 0u;
    nev[k] = end - start;
    alive[k] = px < p.W && (py0 + RS * k) < p.H;
  }
  if (lane == 0) {
    // zero quadric and threshold -1: t = -1 everywhere
    L0[NB] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    L1[NB] = make_float4(0.0f, -1.0f, 0.0f, 0.0f);
  }
  const float tile_x0 = (float)(tx * TS), tile_y0 = (float)(ty * TS);

  for (uint32_t b = start; b < end; b += NB) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < P; ++k) any = any || alive[k];
    if (__syncthreads_or(any) == 0) break;  // every pixel of the tile has terminated
    uint32_t mask[SB];
#pragma unroll
    for (int r = 0; r < SB; ++r) {
      const int slot = lane + r * NT;  // list order: slot b + slot
      const uint32_t idx = b + slot;
      mask[r] = 0u;
      if (idx < end) {
        uint32_t id = vals[idx];
        if (id >= p.n) id = 0;  // never taken for a list built by gs_bin_sort over these n splats
        const float2 m = reinterpret_cast<const float2 *>(means2d)[id];
        const float4 co = reinterpret_cast<const float4 *>(conic_opacity)[id];
        const float3 c = make_float3(rgb[3 * id], rgb[3 * id + 1], rgb[3 * id + 2]);
        float4 a0, a1, a2;
        fold<KIND>(m, co, c, tile_x0, tile_y0, p, a0, a1, a2);
        L0[slot] = a0;
        L1[slot] = a1;
        L2[slot] = a2;
        float hx, hy;
        pass_box(co, a1.y, hx, hy);
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          // first pixel centre of wave w's block, tile-local like the record
          const float bx = 0.5f + (float)((w % (TS / WX)) * WX), by = 0.5f + (float)((w / (TS / WX)) * WY);
          if (a0.x + hx >= bx && a0.x - hx <= bx + (float)(WX - 1) && a0.y + hy >= by &&
              a0.y - hy <= by + (float)(WY - 1))
            mask[r] |= 1u << w;
        }
      }
    }
    uint64_t bal[SB][NW];
#pragma unroll
    for (int r = 0; r < SB; ++r)
#pragma unroll
      for (int w = 0; w < NW; ++w) bal[r][w] = __ballot((mask[r] >> w) & 1u);
    if ((lane & (WAVE - 1)) == 0) {
#pragma unroll
      for (int r = 0; r < SB; ++r)
#pragma unroll
        for (int w = 0; w < NW; ++w) wcnt[r][wv][w] = (uint32_t)__popcll(bal[r][w]);
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      uint32_t base = 0;  // shading wave w's records of the earlier rounds
#pragma unroll
      for (int r = 0; r < SB; ++r) {
        if ((mask[r] >> w) & 1u) {
          uint32_t off = base + (uint32_t)__popcll(bal[r][w] & lt);
          for (int s = 0; s < wv; ++s) off += wcnt[r][s][w];
          lst[w][off] = (uint16_t)(lane + r * NT);
        }
#pragma unroll
        for (int s = 0; s < NW; ++s) base += wcnt[r][s][w];
      }
    }
    uint32_t len = 0;
#pragma unroll
    for (int r = 0; r < SB; ++r)
#pragma unroll
      for (int s = 0; s < NW; ++s) len += wcnt[r][s][wv];
    if ((lane & (WAVE - 1)) < G) lst[wv][len + (lane & (WAVE - 1))] = (uint16_t)NB;
    __syncthreads();
    if (any) {
      // G splats per step: all G records are read and tested before the one
      // branch that skips the step when no pixel of the lane passes (most
      // steps); the blend then visits the G splats in list order
      // the next step's eight list slots are read while this step computes,
      // so a step starts with one LDS round trip (its records), not two
      uint4 jn = *reinterpret_cast<const uint4 *>(&lst[wv][0]);
      for (uint32_t i = 0; i < len; i += G) {
        const uint4 jc = jn;
        if (i + G < len) jn = *reinterpret_cast<const uint4 *>(&lst[wv][i + G]);
        const int js[G] = {(int)(jc.x & 0xFFFFu), (int)(jc.x >> 16), (int)(jc.y & 0xFFFFu), (int)(jc.y >> 16),
                           (int)(jc.z & 0xFFFFu), (int)(jc.z >> 16), (int)(jc.w & 0xFFFFu), (int)(jc.w >> 16)};
        float t[G][P];
        float mx = -1.0f;
#pragma unroll
        for (int q = 0; q < G; ++q) {
          const float4 r0 = L0[js[q]];
          const float2 r1 = *reinterpret_cast<const float2 *>(&L1[js[q]]);  // (c, x_e)
          const RowPart rp = row_part(r0, r1.y, fx);
#pragma unroll
          for (int k = 0; k < P; ++k) {
            t[q][k] = t_at(rp, r1.x, fy[k]);
            mx = fmaxf(mx, t[q][k]);
          }
        }
        if (COUNT && !(mx >= 0.0f)) {
          uint32_t nreal = 0;
#pragma unroll
          for (int q = 0; q < G; ++q) nreal += js[q] != NB;
#pragma unroll
          for (int k = 0; k < P; ++k) tested[k] += alive[k] ? nreal : 0u;
        }
        if (mx >= 0.0f) {
          float4 s1v[G], s2v[G];
#pragma unroll
          for (int q = 0; q < G; ++q) {
            s1v[q] = L1[js[q]];
            s2v[q] = L2[js[q]];
          }
#pragma unroll
          for (int q = 0; q < G; ++q) {
            const uint32_t pos = b + (uint32_t)js[q] - start + 1;
#pragma unroll
            for (int k = 0; k < P; ++k) {
              if (COUNT && js[q] != NB && alive[k]) ++tested[k];
              if (t[q][k] >= 0.0f && alive[k]) {  // the stop-or-blend choice below is by selects
                const float a = alpha_from<KIND>(t[q][k], s1v[q], p);
                const float Tn = T[k] * (1.0f - a);
                const bool stop = Tn < p.t_min;
                const float w = stop ? 0.0f : a * T[k];
                C0[k] = fmaf(s2v[q].x, w, C0[k]);
                C1[k] = fmaf(s2v[q].y, w, C1[k]);
                C2[k] = fmaf(s2v[q].z, w, C2[k]);
                T[k] = stop ? T[k] : Tn;
                ncon[k] += stop ? 0u : 1u;
                last[k] = stop ? last[k] : pos;
                nev[k] = stop ? pos : nev[k];
                alive[k] = !stop;
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
    if (COUNT) out.n_tested[pix] = tested[k];
  }
}

}  // namespace

}  // namespace gs
