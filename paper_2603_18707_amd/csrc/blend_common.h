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
__device__ inline float opacity_threshold64(const BlendParams &p, int order, float o) {
  if (!(o > 0.0f)) return -1.0f;
  double c[4] = {p.c[0], p.c[1], p.c[2], p.c[3]};
  const double cc = c[0] - (double)p.eps / (double)o;
  if (cc < 0.0) return -1.0f;
  double x;
  if (order == 2) {
    const double disc = c[1] * c[1] - 4.0 * cc * c[2];
    if (disc < 0.0) return -1.0f;
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
  return (float)x;
}

// staged record: s0 = (u, v, a, 2b), s1 = (c, x_e, S, o'), s2 = (r, g, b, 0)
template <int KIND>
__device__ inline void fold(float2 m, float4 co, float3 c, const BlendParams &p, float4 &s0, float4 &s1,
                            float4 &s2) {
  const float o = co.w;
  float xe, S = 0.0f;
  if (KIND == BLEND_POLY1) {
    xe = (o * p.c[0] >= p.eps) ? (p.eps / o - p.c[0]) / p.c[1] : -1.0f;
    S = -o * p.c[1];
  } else if (KIND == BLEND_EXP) {
    xe = (o >= p.eps) ? 1.38629436111989061f * (log2f(o) - p.log2_eps) : -1.0f;  // 2 ln(o / eps)
  } else {
    xe = opacity_threshold64(p, KIND == BLEND_POLY2 ? 2 : 3, o);
  }
  s0 = make_float4(m.x, m.y, co.x, 2.0f * co.y);
  s1 = make_float4(co.z, xe, S, o);
  s2 = make_float4(c.x, c.y, c.z, 0.0f);
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

}  // namespace

}  // namespace gs
