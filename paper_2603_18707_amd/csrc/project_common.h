// Device code of the per-splat projection, shared by the single-view and the
// batched preprocess kernels (see preprocess.hip for the method).
#pragma once

#include <cmath>

#include "gs_internal.h"

namespace gs {

namespace {

__device__ inline long clamp_floor(double e, long lo, long hi) {
  if (!(e >= (double)lo)) return lo;  // also NaN
  if (e >= (double)hi + 1.0) return hi;
  long f = (long)floor(e);
  return f < lo ? lo : (f > hi ? hi : f);
}

__device__ inline double poly_eval(const double *c, int order, double x) {
  double s = c[order];
  for (int i = order - 1; i >= 0; --i) s = fma(s, x, c[i]);
  return s;
}

__device__ inline double poly_deriv(const double *c, int order, double x) {
  double s = order * c[order];
  for (int i = order - 1; i >= 1; --i) s = fma(s, x, i * c[i]);
  return s;
}

// First positive root of p(x) = target by the closed forms of App. B (linear;
// quadratic formula in its cancellation-free form; Cardano's formula with the
// cube-root branch chosen to avoid cancellation), polished by two Newton steps
// in double precision. -1 when p(0) < target (no root in the decreasing part).
// The host has checked that p decreases on [0, x_0], so the root is unique there.
__device__ double opacity_root(const double *c, int order, double target) {
  const double cc = c[0] - target;
  if (cc < 0.0) return -1.0;
  if (cc == 0.0) return 0.0;
  double x;
  if (order == 1) {
    x = -cc / c[1];
  } else if (order == 2) {
    const double disc = c[1] * c[1] - 4.0 * cc * c[2];
    if (disc < 0.0) return -1.0;
    x = 2.0 * cc / (-c[1] + sqrt(disc));
  } else {
    const double d0 = c[2] * c[2] - 3.0 * c[3] * c[1];
    const double d1 = 2.0 * c[2] * c[2] * c[2] - 9.0 * c[3] * c[2] * c[1] + 27.0 * c[3] * c[3] * cc;
    const double s = d1 * d1 - 4.0 * d0 * d0 * d0;  // > 0: a monotone cubic has one real root
    const double sq = sqrt(s > 0.0 ? s : 0.0);
    const double C = cbrt(d1 >= 0.0 ? 0.5 * (d1 + sq) : 0.5 * (d1 - sq));
    x = -(c[2] + C + d0 / C) / (3.0 * c[3]);
  }
  if (order > 1) {  // the linear case is exact already
    const double cs[4] = {cc, c[1], c[2], c[3]};
    for (int it = 0; it < 2; ++it) {
      const double f = poly_eval(cs, order, x), fp = poly_deriv(cs, order, x);
      if (fp != 0.0) x -= f / fp;
    }
  }
  return x > 0.0 ? x : 0.0;
}

// Real spherical harmonics up to degree 3 (3DGS ordering and signs) at the
// unit direction (x, y, z), in single precision (colour decides nothing
// discrete; its error stays below 1e-6 of the [0, 1] range).
template <int DEG>
__device__ inline void sh_basis(float x, float y, float z, float Y[16]) {
  Y[0] = 0.28209479177387814f;  // sqrt(1 / (4 pi))
  if (DEG >= 1) {
    const float k1 = 0.48860251190291992f;  // sqrt(3 / (4 pi))
    Y[1] = -k1 * y;
    Y[2] = k1 * z;
    Y[3] = -k1 * x;
  }
  if (DEG >= 2) {
    const float a = 1.0925484305920792f, b = 0.31539156525252005f, c = 0.54627421529603959f;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = a * x * y;
    Y[5] = -a * y * z;
    Y[6] = b * (2.0f * zz - xx - yy);
    Y[7] = -a * x * z;
    Y[8] = c * (xx - yy);
  }
  if (DEG >= 3) {
    const float a = 0.59004358992664352f, b = 2.8906114426405538f, c = 0.45704579946446572f;
    const float d = 0.37317633259011540f, e = 1.4453057213202769f;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[9] = -a * y * (3.0f * xx - yy);
    Y[10] = b * x * y * z;
    Y[11] = -c * y * (4.0f * zz - xx - yy);
    Y[12] = d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -c * x * (4.0f * zz - xx - yy);
    Y[14] = e * z * (xx - yy);
    Y[15] = -a * x * (xx - 3.0f * yy);
  }
}

// rgb = max(sum_k Y_k sh_k + 0.5, 0) for splat i, 0 when culled. Each lane
// reads its own coefficient row (16-byte loads when the row is a multiple of
// 16 bytes, as at degree 1 and 3): the rows of a wave are one contiguous
// block, so its cache lines are fetched once and reused across the loads,
// and no LDS, barrier or second pass over the block is needed.
template <int DEG>
__device__ inline float3 sh_colour(const float *__restrict__ sh, int64_t i, bool live, const float Y[16]) {
  constexpr int NB = (DEG + 1) * (DEG + 1);
  constexpr int NSH3 = 3 * NB;
  if (!live) return make_float3(0.f, 0.f, 0.f);
  float f[NSH3];
  if constexpr (NSH3 % 4 == 0) {
    const float4 *row = reinterpret_cast<const float4 *>(sh + i * NSH3);
#pragma unroll
    for (int q = 0; q < NSH3 / 4; ++q) {
      const float4 v = row[q];
      f[4 * q] = v.x;
      f[4 * q + 1] = v.y;
      f[4 * q + 2] = v.z;
      f[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < NSH3; ++q) f[q] = sh[i * NSH3 + q];
  }
  float a0 = 0.5f, a1 = 0.5f, a2 = 0.5f;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    a0 = fmaf(Y[k], f[3 * k], a0);
    a1 = fmaf(Y[k], f[3 * k + 1], a1);
    a2 = fmaf(Y[k], f[3 * k + 2], a2);
  }
  return make_float3(fmaxf(a0, 0.0f), fmaxf(a1, 0.0f), fmaxf(a2, 0.0f));
}

// |S'| for S' = M diag(s)^2 M^T, M = TW Rq: the squared norm of the cross
// product of the rows of M diag(s) (Lagrange's identity), evaluated as
// sum_k sig_k^2 n_k^2 with n = Rq^T (TW_0 x TW_1) (a rotation commutes with
// the cross product) and sig = (s1 s2, s0 s2, s0 s1). A sum of squares keeps
// its relative accuracy for thin footprints, where Sxx Syy - Sxy^2 cancels
// completely and the anti-aliasing opacity scale would be rounding noise.
__device__ inline double proj_cov_det(const double TW[2][3], const double Rq[3][3], double s0, double s1,
                                      double s2) {
  const double c0 = TW[0][1] * TW[1][2] - TW[0][2] * TW[1][1];
  const double c1 = TW[0][2] * TW[1][0] - TW[0][0] * TW[1][2];
  const double c2 = TW[0][0] * TW[1][1] - TW[0][1] * TW[1][0];
  const double sg[3] = {s1 * s2, s0 * s2, s0 * s1};
  double det = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double n = Rq[0][k] * c0 + Rq[1][k] * c1 + Rq[2][k] * c2;
    det += (sg[k] * n) * (sg[k] * n);
  }
  return det;
}

// Projects splat i of a scene and writes output record o. Tile rows are
// offset by row_base (non-zero when several views share one virtual grid).
// Returns whether the splat survived the culls; then Y holds its SH basis
// values along the ray from the camera centre (rgb is written by the caller,
// see sh_colour).
template <int DEG>
__device__ inline bool project_one(const PreParams &p, int64_t i, const float *__restrict__ means3d,
                                   const float *__restrict__ scales, const float *__restrict__ quats,
                                   const float *__restrict__ opac, int64_t o, int row_base, const PreOut &out,
                                   float Y[16]) {
  bool live = false;
  const CamD &cam = p.cam;
  // every input of the splat is loaded up front, so the loads are in flight
  // together instead of one round trip after each cull test
  const float fmx = means3d[3 * i], fmy = means3d[3 * i + 1], fmz = means3d[3 * i + 2];
  const float fqw = quats[4 * i], fqx = quats[4 * i + 1], fqy = quats[4 * i + 2], fqz = quats[4 * i + 3];
  const float fs0 = scales[3 * i], fs1 = scales[3 * i + 1], fs2 = scales[3 * i + 2];
  const float fop = opac[i];
  const double mx = fmx, my = fmy, mz = fmz;
  double t[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) t[r] = cam.R[3 * r] * mx + cam.R[3 * r + 1] * my + cam.R[3 * r + 2] * mz + cam.t[r];

  out.depth[o] = (float)t[2];
  float2 m2 = make_float2(0.f, 0.f);
  float4 co = make_float4(0.f, 0.f, 0.f, 0.f);
  int4 rc = make_int4(0, 0, -1, -1);
  uint32_t ntiles = 0;

  do {
    if (t[2] < p.near_z) break;
    // 3D covariance R(q) diag(s)^2 R(q)^T
    double qw = fqw, qx = fqx, qy = fqy, qz = fqz;
    const double qn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qn; qx *= qn; qy *= qn; qz *= qn;
    const double Rq[3][3] = {{1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
                             {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
                             {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
    const double s0 = fs0, s1 = fs1, s2 = fs2;
    const double ss[3] = {s0 * s0, s1 * s1, s2 * s2};
    // EWA: T = J W (2x3), S' = T Sigma T^T computed as (T Rq) diag(ss) (T Rq)^T
    const double tz = t[2], iz = 1.0 / tz;
    double txz = t[0] * iz, tyz = t[1] * iz;
    txz = fmin(fmax(txz, -cam.limx), cam.limx);
    tyz = fmin(fmax(tyz, -cam.limy), cam.limy);
    const double J00 = cam.fx * iz, J02 = -cam.fx * txz * iz;
    const double J11 = cam.fy * iz, J12 = -cam.fy * tyz * iz;
    double TW[2][3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      TW[0][b] = J00 * cam.R[b] + J02 * cam.R[6 + b];
      TW[1][b] = J11 * cam.R[3 + b] + J12 * cam.R[6 + b];
    }
    double M[2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k) M[a][k] = TW[a][0] * Rq[0][k] + TW[a][1] * Rq[1][k] + TW[a][2] * Rq[2][k];
    const double Sxx = M[0][0] * M[0][0] * ss[0] + M[0][1] * M[0][1] * ss[1] + M[0][2] * M[0][2] * ss[2];
    const double Sxy = M[0][0] * M[1][0] * ss[0] + M[0][1] * M[1][1] * ss[1] + M[0][2] * M[1][2] * ss[2];
    const double Syy = M[1][0] * M[1][0] * ss[0] + M[1][1] * M[1][1] * ss[1] + M[1][2] * M[1][2] * ss[2];

    // anti-aliasing: add v to the diagonal, scale opacity by sqrt(|S'| / |S'+vI|)
    const double det0 = proj_cov_det(TW, Rq, s0, s1, s2);
    const double Axx = Sxx + p.aa_v, Ayy = Syy + p.aa_v;
    const double deta = Axx * Ayy - Sxy * Sxy;
    if (!(deta > 0.0)) break;
    const double ideta = 1.0 / deta;
    const double ratio = det0 * ideta;
    const double o = (double)fop * sqrt(ratio > 0.0 ? ratio : 0.0);

    // bounding radius multiplier
    double k;
    if (p.radius_mode == GS_RADIUS_SIGMA3) {
      k = 3.0;
    } else if (p.radius_mode == GS_RADIUS_POLY_UNIVERSAL) {
      k = p.k_universal;
    } else if (p.radius_mode == GS_RADIUS_POLY_OPACITY) {
      const double xr = (o > 0.0) ? opacity_root(p.c, p.order, p.eps / o) : -1.0;
      if (xr < 0.0) break;
      k = sqrt(xr);
    } else {
      if (!(o >= p.eps)) break;
      k = sqrt(2.0 * log(o / p.eps));
    }
    const double mid = 0.5 * (Axx + Ayy);
    const double disc = mid * mid - deta;
    const double lmax = mid + sqrt(disc > 0.0 ? disc : 0.0);
    const double r = k * sqrt(lmax) * p.pad;
    // half sides: the bounding square of radius r, or the ellipse Q = k^2's own box
    const double hx = p.rect_mode == GS_RECT_ELLIPSE_BOX ? k * sqrt(Axx) * p.pad : r;
    const double hy = p.rect_mode == GS_RECT_ELLIPSE_BOX ? k * sqrt(Ayy) * p.pad : r;
    const double u = cam.fx * t[0] * iz + cam.cx;
    const double v = cam.fy * t[1] * iz + cam.cy;
    // x / T as x * (1 / T): exact, T being a power of two (16, checked on the host)
    const double iT = 1.0 / (double)p.tile;
    const long xlo = clamp_floor((u - hx) * iT, 0, cam.gx), xhi = clamp_floor((u + hx) * iT, -1, cam.gx - 1);
    const long ylo = clamp_floor((v - hy) * iT, 0, cam.gy), yhi = clamp_floor((v + hy) * iT, -1, cam.gy - 1);
    if (xhi >= xlo && yhi >= ylo) {
      rc = make_int4((int)xlo, (int)ylo + row_base, (int)xhi, (int)yhi + row_base);
      ntiles = (uint32_t)((xhi - xlo + 1) * (yhi - ylo + 1));
    }
    m2 = make_float2((float)u, (float)v);
    co = make_float4((float)(Ayy * ideta), (float)(-Sxy * ideta), (float)(Axx * ideta), (float)o);

    // colour basis along the ray from the camera centre
    const double d0 = mx - cam.campos[0], d1 = my - cam.campos[1], d2 = mz - cam.campos[2];
    const double dn = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    sh_basis<DEG>((float)(d0 * dn), (float)(d1 * dn), (float)(d2 * dn), Y);
    live = true;
  } while (false);

  reinterpret_cast<float2 *>(out.means2d)[o] = m2;
  reinterpret_cast<float4 *>(out.conic_opacity)[o] = co;
  reinterpret_cast<int4 *>(out.rect)[o] = rc;
  out.tiles[o] = ntiles;
  return live;
}

}  // namespace

}  // namespace gs
