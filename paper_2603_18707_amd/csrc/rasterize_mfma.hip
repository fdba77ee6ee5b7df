// Front-to-back blending with the quadric evaluated on the matrix cores.
//
// Sec. 5.1 observes that the quadric of every (pixel, splat) pair of a tile is
// a dot product: with the pixel's monomials m = (1, x, y, x^2, x y, y^2) and a
// coefficient vector per splat, Q (or here t = x_e - Q directly) for a block
// of pixels and a batch of splats is one small matrix product, the shape
// matrix units execute. On CDNA4 that product is v_mfma_f32_32x32x2_f32:
// 32 splats x 32 pixels, K = 2 per instruction, three instructions for K = 6.
//
// The expanded form cancels: far from the mean its terms exceed Q by orders
// of magnitude, and evaluated about a fixed origin in single precision it
// misses the 2e-4 pixel bar on long, thin footprints. Here each splat's
// coefficients are the Taylor expansion of t about the centre of the 8x8
// pixel block a wave shades, computed in double from the float record and
// rounded once: t(c + d) = t_c - G . d - (a d_x^2 + 2 b d_x d_y + c d_y^2),
// with t_c = x_e - Q(c) and G = 2 conic (c - mean). Within the block |d| <=
// 3.5 px, and where t is near 0 the terms stay within a few hundred, so the
// float product is off by at most a few 1e-5 in t (an alpha error below 3e-6
// at opacity 1 for the first-order kernel, measured on thin footprints).
//
// Layout. One workgroup of 256 threads per 16x16 tile, a wave per 8x8 block
// (as the vector blend). A wave's 64 pixels are two 32-pixel halves (rows
// 0-3 and 4-7 of the block), each the N dimension of one product; lane l
// supplies pixel l % 32's monomials as B and coefficient l / 32 (of the pair
// the instruction consumes) of splat row l % 32 as A. Output register r of
// lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32; the splats
// of a 32-record step are placed on the rows so that lanes 0-31 receive
// records 0-15 and lanes 32-63 records 16-31, in list order. Each lane thus
// holds t for two pixels (one per half) and sixteen consecutive records.
//
// Compositing. The lanes of the first record half blend their sixteen
// records exactly (front to back from the pixel's state, with the alpha
// clamp, the eps test and early termination before the stopping splat). The
// lanes of the second half blend theirs from T = 1 at the same time; the
// over operator is associative, so the halves combine as C = C_1 + T_1 C_2,
// T = T_1 T_2. A pixel whose second half would take T below t_min (rare:
// once per pixel at most) is replayed exactly from the first half's state.
// Rounding differs from a sequential walk only in the order of the
// transmittance products.
//
// Records are staged as in the vector blend (256 at a time, with a per-wave
// box test so each wave walks only the records that can reach its block),
// plus each record's six coefficients for each of the four wave blocks.
#include <cmath>

#include "blend_common.h"
#include "gs_internal.h"

namespace gs {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int MT = 256;          // threads per tile
constexpr int MW = MT / WAVE;    // waves, one per 8x8 block
constexpr int MSTEP = 32;        // records per matrix step
constexpr int NCOEF = 6;         // expansion coefficients per record and block

// The step record an A row carries: row 8 (r / 4) + 4 h + r % 4 lands in
// register r of the lanes of half h, which hold records 16 h + r
__device__ inline int record_of_row(int i) { return 16 * ((i >> 2) & 1) + 4 * (i >> 3) + (i & 3); }

struct Px {
  float T, C0, C1, C2;
  uint32_t ncon, last, nev;
  bool alive;
};

template <int KIND>
__device__ inline float alpha_mfma(float t, const float4 &rb, const float2 &oc, const BlendParams &p) {
  float a;
  if (KIND == BLEND_POLY1) {
    a = fmaf(rb.w, t, p.eps);  // rb.w = -o' c_1
  } else if (KIND == BLEND_EXP) {
    a = __builtin_amdgcn_exp2f(fmaf(t, 0.72134752044448170f, p.log2_eps));
  } else {
    const float Q = oc.y - t;  // oc = (o', x_e)
    const float f = (KIND == BLEND_POLY2) ? fmaf(fmaf(p.c[2], Q, p.c[1]), Q, p.c[0])
                                          : fmaf(fmaf(fmaf(p.c[3], Q, p.c[2]), Q, p.c[1]), Q, p.c[0]);
    a = oc.x * f;
  }
  return fminf(a, p.alpha_max);
}

template <int KIND>
__device__ inline void blend_pair(Px &s, float t, const float4 &rb, const float2 &oc, uint32_t pos, float tmin,
                                  const BlendParams &p) {
  const float a = alpha_mfma<KIND>(t, rb, oc, p);
  const float Tn = s.T * (1.0f - a);
  const bool stop = Tn < tmin;
  const float w = stop ? 0.0f : a * s.T;
  s.C0 = fmaf(rb.x, w, s.C0);
  s.C1 = fmaf(rb.y, w, s.C1);
  s.C2 = fmaf(rb.z, w, s.C2);
  s.T = stop ? s.T : Tn;
  s.ncon += stop ? 0u : 1u;
  s.last = stop ? s.last : pos;
  s.nev = stop ? pos : s.nev;
  s.alive = !stop;
}

// the lane's sixteen records of a step (slot words w8, two 16-bit slots
// each) over one of its pixels (state s, quadric terms d), front to back
template <int KIND>
__device__ inline void run_records(Px &s, const v16f &d, const uint32_t (&w8)[8], const float4 *__restrict__ Lb,
                                   const float2 *__restrict__ Lc, uint32_t pos0, float tmin, const BlendParams &p) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (d[r] >= 0.0f && s.alive) {
      const int j = (int)((w8[r >> 1] >> (16 * (r & 1))) & 0xFFFFu);
      const float4 rb = Lb[j];
      const float2 oc = (KIND == BLEND_POLY2 || KIND == BLEND_POLY3) ? Lc[j] : make_float2(0.0f, 0.0f);
      blend_pair<KIND>(s, d[r], rb, oc, pos0 + (uint32_t)j, tmin, p);
    }
  }
}

__device__ inline Px swap_halves(const Px &s) {
  Px o;
  o.T = __shfl_xor(s.T, 32, 64);
  o.C0 = __shfl_xor(s.C0, 32, 64);
  o.C1 = __shfl_xor(s.C1, 32, 64);
  o.C2 = __shfl_xor(s.C2, 32, 64);
  o.ncon = (uint32_t)__shfl_xor((int)s.ncon, 32, 64);
  o.last = (uint32_t)__shfl_xor((int)s.last, 32, 64);
  o.nev = (uint32_t)__shfl_xor((int)s.nev, 32, 64);
  o.alive = __shfl_xor((int)s.alive, 32, 64) != 0;
  return o;
}

template <int KIND>
__global__ __launch_bounds__(MT) void blend_fwd_mfma(BlendParams p, const float *__restrict__ means2d,
                                                     const float *__restrict__ conic_opacity,
                                                     const float *__restrict__ rgb, const uint32_t *__restrict__ vals,
                                                     const uint32_t *__restrict__ ranges,
                                                     const uint32_t *__restrict__ tile_order, BlendOut out) {
  __shared__ float coef[MW][NCOEF][MT + 1];                 // [block][coefficient][record], slot MT neutral
  __shared__ float4 Lb[MT + 1];                             // (r, g, b, -o' c_1)
  __shared__ float2 Lc[MT + 1];                             // (o', x_e)
  __shared__ __align__(16) uint16_t lst[MW][MT + MSTEP];    // each wave's records, padded by a step
  __shared__ uint32_t wcnt[MW][MW];
  const int ntiles = p.gx * p.gy;
  if ((int)blockIdx.x >= ntiles) return;
  const int tile = tile_order ? (int)min(tile_order[blockIdx.x], (uint32_t)(ntiles - 1)) : (int)blockIdx.x;
  const int tx = tile % p.gx, ty = tile / p.gx;
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];

  const int lane = threadIdx.x, wv = lane / WAVE, l64 = lane & (WAVE - 1);
  const int hb = l64 >> 5, col32 = l64 & 31;
  const uint64_t lt = (1ull << l64) - 1ull;
  const int wx0 = (wv & 1) * 8, wy0 = (wv >> 1) * 8;
  // this lane's two pixels: column col32 % 8, rows col32 / 8 and col32 / 8 + 4 of the wave's block
  const int pcx = col32 & 7, pr0 = col32 >> 3;
  const int px = tx * TS + wx0 + pcx;
  // B operands: monomials (1, x, y, x^2, x y, y^2) of the pixel centres relative to the block centre;
  // instruction m takes monomials 2m (lanes 0-31) and 2m + 1 (lanes 32-63)
  float bm[2][3];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float x = (float)pcx - 3.5f, y = (float)(pr0 + 4 * h) - 3.5f;
    const float mono[NCOEF] = {1.0f, x, y, x * x, x * y, y * y};
#pragma unroll
    for (int m = 0; m < 3; ++m) bm[h][m] = mono[2 * m + hb];
  }
  Px st[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    st[h] = Px{1.0f, 0.0f, 0.0f, 0.0f, 0u, 0u, end - start, false};
    st[h].alive = px < p.W && (ty * TS + wy0 + pr0 + 4 * h) < p.H;
  }
  if (lane == 0) {
    for (int w = 0; w < MW; ++w) {
      coef[w][0][MT] = -1.0f;  // t = -1 at every pixel
      for (int k = 1; k < NCOEF; ++k) coef[w][k][MT] = 0.0f;
    }
    Lb[MT] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    Lc[MT] = make_float2(0.0f, -1.0f);
  }
  const float tile_x0 = (float)(tx * TS), tile_y0 = (float)(ty * TS);
  const v16f zero = {};

  for (uint32_t b = start; b < end; b += MT) {
    const bool any = st[0].alive || st[1].alive;
    if (__syncthreads_or(any) == 0) break;  // every pixel of the tile has terminated
    const uint32_t idx = b + lane;
    uint32_t mask = 0u;
    if (idx < end) {
      uint32_t id = vals[idx];
      if (id >= p.n) id = 0;  // never taken for a list built by gs_bin_sort over these n splats
      const float2 m = reinterpret_cast<const float2 *>(means2d)[id];
      const float4 co = reinterpret_cast<const float4 *>(conic_opacity)[id];
      const float o = co.w;
      const float xe = alpha_threshold<KIND>(p, o);
      Lb[lane] = make_float4(rgb[3 * id], rgb[3 * id + 1], rgb[3 * id + 2], KIND == BLEND_POLY1 ? -o * p.c[1] : 0.0f);
      Lc[lane] = make_float2(o, xe);
      const double A = co.x, B = co.y, C = co.z;
      const bool pd = co.x > 0.0f && co.z > 0.0f && fma(A, C, -(B * B)) > 0.0 && xe >= 0.0f;
#pragma unroll 1
      for (int w = 0; w < MW; ++w) {
        if (pd) {
          // expansion about the block centre, in double from the float record
          const double dx0 = (double)(tile_x0 + (float)((w & 1) * 8 + 4)) - (double)m.x;
          const double dy0 = (double)(tile_y0 + (float)((w >> 1) * 8 + 4)) - (double)m.y;
          const double q0 = A * dx0 * dx0 + 2.0 * B * dx0 * dy0 + C * dy0 * dy0;
          coef[w][0][lane] = (float)((double)xe - q0);
          coef[w][1][lane] = (float)(-2.0 * (A * dx0 + B * dy0));
          coef[w][2][lane] = (float)(-2.0 * (B * dx0 + C * dy0));
          coef[w][3][lane] = -co.x;
          coef[w][4][lane] = -2.0f * co.y;
          coef[w][5][lane] = -co.z;
        } else {
          coef[w][0][lane] = -1.0f;
          for (int k = 1; k < NCOEF; ++k) coef[w][k][lane] = 0.0f;
        }
      }
      float hx, hy;
      pass_box(co, pd ? xe : -1.0f, hx, hy);
      const float mx = m.x - tile_x0, my = m.y - tile_y0;
#pragma unroll
      for (int w = 0; w < MW; ++w) {
        const float bx = 0.5f + (float)((w & 1) * 8), by = 0.5f + (float)((w >> 1) * 8);
        if (mx + hx >= bx && mx - hx <= bx + 7.0f && my + hy >= by && my - hy <= by + 7.0f) mask |= 1u << w;
      }
    }
    uint64_t bal[MW];
#pragma unroll
    for (int w = 0; w < MW; ++w) bal[w] = __ballot((mask >> w) & 1u);
    if (l64 == 0) {
#pragma unroll
      for (int w = 0; w < MW; ++w) wcnt[wv][w] = (uint32_t)__popcll(bal[w]);
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < MW; ++w) {
      if ((mask >> w) & 1u) {
        uint32_t off = (uint32_t)__popcll(bal[w] & lt);
        for (int s = 0; s < wv; ++s) off += wcnt[s][w];
        lst[w][off] = (uint16_t)lane;
      }
    }
    uint32_t len = 0;
#pragma unroll
    for (int s = 0; s < MW; ++s) len += wcnt[s][wv];
    if (l64 < MSTEP) lst[wv][len + l64] = (uint16_t)MT;
    __syncthreads();
    if (__ballot(st[0].alive || st[1].alive) != 0ull) {
      const uint32_t pos0 = b - start + 1;
      const int arec = record_of_row(col32);  // the record of the A row this lane supplies
      for (uint32_t i = 0; i < len; i += MSTEP) {
        const int ja = lst[wv][i + arec];
        float a[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) a[m] = coef[wv][2 * m + hb][ja];
        // this half's sixteen slots
        const uint4 sa = *reinterpret_cast<const uint4 *>(&lst[wv][i + 16 * hb]);
        const uint4 sb = *reinterpret_cast<const uint4 *>(&lst[wv][i + 16 * hb + 8]);
        const uint32_t w8[8] = {sa.x, sa.y, sa.z, sa.w, sb.x, sb.y, sb.z, sb.w};
#pragma unroll
        for (int h = 0; h < 2; ++h) {  // the lane's two pixels, one product each
          v16f d = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0], bm[h][0], zero, 0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1], bm[h][1], d, 0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2], bm[h][2], d, 0, 0, 0);
          float mxt = -1.0f;
#pragma unroll
          for (int r = 0; r < 16; ++r) mxt = fmaxf(mxt, d[r]);
          if (__ballot(mxt >= 0.0f && st[h].alive) == 0ull) continue;
          // the first half's lanes walk their records exactly from the pixel
          // state; the second half's from T = 1, without termination
          Px w = st[h];
          if (hb) {
            w.T = 1.0f;
            w.C0 = w.C1 = w.C2 = 0.0f;
            w.ncon = 0u;
          }
          run_records<KIND>(w, d, w8, Lb, Lc, pos0, hb ? 0.0f : p.t_min, p);
          // both halves combine the same values into the same state
          const Px o = swap_halves(w);
          const Px &h1 = hb ? o : w;  // the first half, exact
          const Px &h2 = hb ? w : o;  // the second half, from T = 1
          Px f = h1;
          bool need = false;
          if (h1.alive) {
            const float Te = h1.T * h2.T;
            if (Te < p.t_min) {
              need = true;  // the pixel stops in the second half
            } else {
              f.T = Te;
              f.C0 = fmaf(h1.T, h2.C0, h1.C0);
              f.C1 = fmaf(h1.T, h2.C1, h1.C1);
              f.C2 = fmaf(h1.T, h2.C2, h1.C2);
              f.ncon = h1.ncon + h2.ncon;
              f.last = h2.ncon ? h2.last : h1.last;
            }
          }
          if (__ballot(need) != 0ull) {
            // rare: the second half's lanes walk their records again,
            // exactly, from the first half's state; the first half's lanes
            // take the result
            Px g = f;
            if (!(hb && need)) g.alive = false;
            run_records<KIND>(g, d, w8, Lb, Lc, pos0, p.t_min, p);
            const Px og = swap_halves(g);
            if (need) f = hb ? g : og;
          }
          st[h] = f;
        }
      }
    }
    __syncthreads();
  }
  if (hb) return;  // both halves hold the same pixel state; the first writes it
  const size_t plane = (size_t)p.W * p.H;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int py = ty * TS + wy0 + pr0 + 4 * h;
    if (px >= p.W || py >= p.H) continue;
    const size_t pix = (size_t)py * p.W + px;
    out.image[pix] = fmaf(st[h].T, p.bg[0], st[h].C0);
    out.image[plane + pix] = fmaf(st[h].T, p.bg[1], st[h].C1);
    out.image[2 * plane + pix] = fmaf(st[h].T, p.bg[2], st[h].C2);
    out.final_T[pix] = st[h].T;
    out.n_contrib[pix] = st[h].ncon;
    out.last_contrib[pix] = st[h].last;
    if (out.n_eval) out.n_eval[pix] = st[h].nev;
  }
}

}  // namespace

hipError_t launch_blend_fwd_mfma(const BlendParams &p, const float *means2d, const float *conic_opacity,
                                 const float *rgb, const uint32_t *vals, const uint32_t *ranges,
                                 const uint32_t *tile_order, BlendOut out, hipStream_t s) {
  const dim3 grid(p.gx * p.gy), block(MT);
  switch (p.blend) {
    case BLEND_EXP:
      hipLaunchKernelGGL(blend_fwd_mfma<BLEND_EXP>, grid, block, 0, s, p, means2d, conic_opacity, rgb, vals, ranges,
                         tile_order, out);
      break;
    case BLEND_POLY1:
      hipLaunchKernelGGL(blend_fwd_mfma<BLEND_POLY1>, grid, block, 0, s, p, means2d, conic_opacity, rgb, vals,
                         ranges, tile_order, out);
      break;
    case BLEND_POLY2:
      hipLaunchKernelGGL(blend_fwd_mfma<BLEND_POLY2>, grid, block, 0, s, p, means2d, conic_opacity, rgb, vals,
                         ranges, tile_order, out);
      break;
    default:
      hipLaunchKernelGGL(blend_fwd_mfma<BLEND_POLY3>, grid, block, 0, s, p, means2d, conic_opacity, rgb, vals,
                         ranges, tile_order, out);
      break;
  }
  return hipGetLastError();
}

}  // namespace gs
