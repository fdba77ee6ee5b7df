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
  const double cs[4] = {cc, c[1], c[2], c[3]};
  for (int it = 0; it < 2; ++it) {
    const double f = poly_eval(cs, order, x), fp = poly_deriv(cs, order, x);
    if (fp != 0.0) x -= f / fp;
  }
  return x > 0.0 ? x : 0.0;
}

// Real spherical harmonics up to degree 3 (3DGS ordering and signs), times
// the coefficients of one channel layout [nsh][3], accumulated in double.
template <int DEG>
__device__ inline void sh_colour(double x, double y, double z, const float *sh, double out[3]) {
  constexpr int deg = DEG;
  const double PI = 3.14159265358979323846;
  double Y[16];
  Y[0] = sqrt(1.0 / (4.0 * PI));
  int nb = 1;
  if (deg >= 1) {
    const double k1 = sqrt(3.0 / (4.0 * PI));
    Y[1] = -k1 * y;
    Y[2] = k1 * z;
    Y[3] = -k1 * x;
    nb = 4;
  }
  if (deg >= 2) {
    const double a = sqrt(15.0 / (4.0 * PI)), b = sqrt(5.0 / (16.0 * PI)), c = sqrt(15.0 / (16.0 * PI));
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = a * x * y;
    Y[5] = -a * y * z;
    Y[6] = b * (2.0 * zz - xx - yy);
    Y[7] = -a * x * z;
    Y[8] = c * (xx - yy);
    nb = 9;
  }
  if (deg >= 3) {
    const double a = sqrt(35.0 / (32.0 * PI)), b = sqrt(105.0 / (4.0 * PI)), c = sqrt(21.0 / (32.0 * PI));
    const double d = sqrt(7.0 / (16.0 * PI)), e = sqrt(105.0 / (16.0 * PI));
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[9] = -a * y * (3.0 * xx - yy);
    Y[10] = b * x * y * z;
    Y[11] = -c * y * (4.0 * zz - xx - yy);
    Y[12] = d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -c * x * (4.0 * zz - xx - yy);
    Y[14] = e * z * (xx - yy);
    Y[15] = -a * x * (xx - 3.0 * yy);
    nb = 16;
  }
  double r = 0.0, g = 0.0, bl = 0.0;
  for (int k = 0; k < nb; ++k) {
    r = fma(Y[k], (double)sh[3 * k + 0], r);
    g = fma(Y[k], (double)sh[3 * k + 1], g);
    bl = fma(Y[k], (double)sh[3 * k + 2], bl);
  }
  out[0] = r;
  out[1] = g;
  out[2] = bl;
}

// One wave per 64 splats. The wave first copies its splats' SH coefficients
// (a contiguous block) into LDS with coalesced loads, padded to an odd row
// stride so the per-lane reads hit distinct banks; reading 48 floats per lane
// straight from global memory would touch 64 cache lines per instruction.
template <int DEG>
__global__ __launch_bounds__(64) void preprocess_kernel(PreParams p, int64_t n, const float *__restrict__ means3d,
                                                        const float *__restrict__ scales,
                                                        const float *__restrict__ quats,
                                                        const float *__restrict__ opac,
                                                        const float *__restrict__ sh, PreOut out) {
  constexpr int NSH3 = 3 * (DEG + 1) * (DEG + 1);
  constexpr int ROW = NSH3 + 1;
  __shared__ float shs[64 * ROW];
  const int64_t base = (int64_t)blockIdx.x * 64;
  const int lane = threadIdx.x;
  {
    const int64_t cnt = (n - base) < 64 ? (n - base) : 64;
    const float *src = sh + base * NSH3;
    const int total = (int)cnt * NSH3;
    for (int e = lane; e < total; e += 64) {
      const int s = e / NSH3, k = e - s * NSH3;
      shs[s * ROW + k] = src[e];
    }
  }
  __syncthreads();
  const int64_t i = base + lane;
  if (i >= n) return;
  const CamD &cam = p.cam;
  const double mx = means3d[3 * i], my = means3d[3 * i + 1], mz = means3d[3 * i + 2];
  double t[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) t[r] = cam.R[3 * r] * mx + cam.R[3 * r + 1] * my + cam.R[3 * r + 2] * mz + cam.t[r];

  out.depth[i] = (float)t[2];
  float2 m2 = make_float2(0.f, 0.f);
  float4 co = make_float4(0.f, 0.f, 0.f, 0.f);
  float col[3] = {0.f, 0.f, 0.f};
  int4 rc = make_int4(0, 0, -1, -1);
  uint32_t ntiles = 0;

  do {
    if (t[2] < p.near_z) break;
    // 3D covariance R(q) diag(s)^2 R(q)^T
    double qw = quats[4 * i], qx = quats[4 * i + 1], qy = quats[4 * i + 2], qz = quats[4 * i + 3];
    const double qn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qn; qx *= qn; qy *= qn; qz *= qn;
    const double Rq[3][3] = {{1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
                             {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
                             {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
    const double s0 = scales[3 * i], s1 = scales[3 * i + 1], s2 = scales[3 * i + 2];
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
    const double det0 = Sxx * Syy - Sxy * Sxy;
    const double Axx = Sxx + p.aa_v, Ayy = Syy + p.aa_v;
    const double deta = Axx * Ayy - Sxy * Sxy;
    if (!(deta > 0.0)) break;
    const double ratio = det0 / deta;
    const double o = (double)opac[i] * sqrt(ratio > 0.0 ? ratio : 0.0);

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
    const double u = cam.fx * t[0] * iz + cam.cx;
    const double v = cam.fy * t[1] * iz + cam.cy;
    const double T = (double)p.tile;
    const long xlo = clamp_floor((u - r) / T, 0, cam.gx), xhi = clamp_floor((u + r) / T, -1, cam.gx - 1);
    const long ylo = clamp_floor((v - r) / T, 0, cam.gy), yhi = clamp_floor((v + r) / T, -1, cam.gy - 1);
    if (xhi >= xlo && yhi >= ylo) {
      rc = make_int4((int)xlo, (int)ylo, (int)xhi, (int)yhi);
      ntiles = (uint32_t)((xhi - xlo + 1) * (yhi - ylo + 1));
    }
    m2 = make_float2((float)u, (float)v);
    co = make_float4((float)(Ayy / deta), (float)(-Sxy / deta), (float)(Axx / deta), (float)o);

    // colour along the ray from the camera centre
    double d0 = mx - cam.campos[0], d1 = my - cam.campos[1], d2 = mz - cam.campos[2];
    const double dn = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    double c3[3];
    sh_colour<DEG>(d0 * dn, d1 * dn, d2 * dn, shs + lane * ROW, c3);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) col[ch] = (float)fmax(c3[ch] + 0.5, 0.0);
  } while (false);

  reinterpret_cast<float2 *>(out.means2d)[i] = m2;
  reinterpret_cast<float4 *>(out.conic_opacity)[i] = co;
  out.rgb[3 * i] = col[0];
  out.rgb[3 * i + 1] = col[1];
  out.rgb[3 * i + 2] = col[2];
  reinterpret_cast<int4 *>(out.rect)[i] = rc;
  out.tiles[i] = ntiles;
}

}  // namespace

void make_cam(const gs_camera *c, int tile, CamD *o) {
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
