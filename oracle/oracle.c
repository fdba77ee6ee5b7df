/*
 * FP64 brute-force reference ("oracle") for tile-based 3D Gaussian Splatting
 * with either the truncated exponential kernel g(x) = exp(-x/2) or the
 * ReLU-activated polynomial kernels f_N(x) = max(sum_i c_i x^i, 0) of
 * "From ex(p) to poly: Gaussian Splatting with Polynomial Kernels"
 * (Mueller, Winter, Steinberger).
 *
 * TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only code that loads this library.
 * The GPU product path shares no code, header, table or constant with it.
 *
 * What is computed, in the paper's order:
 *   - projection of each splat to the image plane and its screen-space
 *     covariance (Sec. 2, Eq. 1, the EWA splatting of the 3DGS formulation);
 *   - Mip-Splatting-like anti-aliasing: a value v added to the diagonal of
 *     the projected covariance, opacity scaled by sqrt(|S'| / |S' + vI|)
 *     (Sec. 3.4, Eqs. 7-9 show the ratio holds for any kernel);
 *   - the bounding radius r = k * sqrt(lambda_max) (Sec. 2.1) with k from
 *     3 sigma, the universal polynomial root (Eq. 5 / App. B with eps = 0),
 *     the opacity-dependent polynomial root (Eq. 4 / App. B), or the
 *     opacity-aware exponential bound (Eq. 3);
 *   - front-to-back alpha compositing of depth-ordered splats per pixel with
 *     the kernel of Eq. 2 (and the first-root cut of Eq. 6 for order 2).
 *
 * Every pixel is tested against every splat in depth order; no tile list is
 * built. The tile rectangle enters only as the membership predicate "the
 * pixel's tile lies in the splat's rectangle" (with tile culling on, "and
 * the tile passes the tile test"), since that is what decides which splats
 * a tile-based rasterizer ever evaluates for a pixel.
 *
 * Roots are found by a plain scan plus bisection, never by the closed forms,
 * so the closed forms of Eq. 3-5 and App. B can be checked against it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_KERNEL_EXP = 0, ORC_KERNEL_POLY = 1 };
enum { ORC_RECT_SQUARE = 0, ORC_RECT_ELLIPSE_BOX = 1 };
enum {
  ORC_RADIUS_SIGMA3 = 0,
  ORC_RADIUS_POLY_UNIVERSAL = 1,
  ORC_RADIUS_POLY_OPACITY = 2,
  ORC_RADIUS_EXP_OPACITY = 3
};

/* per-splat flag bits */
enum { ORC_SPLAT_EDGE_NEAR = 1, ORC_SPLAT_CULL_NEAR = 2 };
/* per-pixel flag bits */
enum { ORC_PIX_ALPHA_NEAR = 1, ORC_PIX_T_NEAR = 2, ORC_PIX_EDGE_NEAR = 4, ORC_PIX_CULL_NEAR = 8 };

typedef struct {
  int32_t kind;        /* ORC_KERNEL_* */
  int32_t order;       /* polynomial order 1..3 */
  int32_t radius_mode; /* ORC_RADIUS_* */
  int32_t tile;        /* tile edge in pixels */
  double c[4];         /* polynomial coefficients c_0..c_3 (unused ones 0) */
  double eps;          /* contribution threshold, 1/255 in 3DGS */
  double alpha_max;    /* alpha clamp */
  double t_min;        /* early-termination transmittance */
  double aa_v;         /* anti-aliasing variance added to the diagonal, px^2 */
  double near_z;       /* near plane */
  double radius_pad;   /* radius multiplier (>= 1) making every rectangle conservative */
  double bg[3];        /* background colour */
  double alpha_band;   /* |alpha - eps| below this flags a pixel */
  double t_band_rel;   /* |T' - t_min| below t_min * this flags a pixel */
  int32_t rect_mode;   /* ORC_RECT_*: bounding square of radius r, or the ellipse's own box */
  int32_t tile_cull;   /* 1: a splat is in a tile's list only if the tile passes the tile test */
} orc_cfg;

typedef struct {
  double R[9];  /* world -> camera rotation, row-major */
  double t[3];  /* world -> camera translation */
  double fx, fy, cx, cy;
  int32_t width, height;
} orc_cam;

/* ------------------------------------------------------------------ */
/* kernel functions (Eq. 2, Eq. 6)                                      */
/* ------------------------------------------------------------------ */

/* p(x) = c_0 + c_1 x + c_2 x^2 + c_3 x^3, written as the plain sum. */
double orc_poly(const double *c, int order, double x) {
  double s = 0.0, xp = 1.0;
  for (int i = 0; i <= order; ++i) {
    s += c[i] * xp;
    xp *= x;
  }
  return s;
}

/* Smallest x >= 0 with p(x) = target: App. B bounds each splat by the first
 * real positive root of the shifted polynomial. Scans [0, xmax] in steps of h for the first sign change of
 * p(x) - target, then bisects to full double precision and returns the upper
 * end of the final bracket, so p(root) - target <= 0 holds as evaluated. Returns -1 when
 * p(0) < target (no non-negative solution in the decreasing branch) or when
 * no sign change is found up to xmax. */
double orc_first_root(const double *c, int order, double target) {
  double f0 = orc_poly(c, order, 0.0) - target;
  if (f0 < 0.0) return -1.0;
  if (f0 == 0.0) return 0.0;
  const double h = 1.0 / 1024.0, xmax = 4096.0;
  double a = 0.0;
  for (;;) {
    double b = a + h;
    if (b > xmax) return -1.0;
    double fb = orc_poly(c, order, b) - target;
    if (fb <= 0.0) {
      if (fb == 0.0) return b;
      double lo = a, hi = b;
      for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double fm = orc_poly(c, order, mid) - target;
        if (fm > 0.0) lo = mid; else hi = mid;
      }
      return hi; /* the smallest double found with p(x) - target <= 0 */
    }
    a = b;
  }
}

/* the kernel k(Q) applied to the quadric value Q */
double orc_kernel(const orc_cfg *cfg, double x0, double Q) {
  if (cfg->kind == ORC_KERNEL_EXP) return exp(-0.5 * Q);
  /* Eq. 6: order 2 uses the polynomial only before its first root */
  if (cfg->order == 2 && Q >= x0) return 0.0;
  double p = orc_poly(cfg->c, cfg->order, Q);
  return p > 0.0 ? p : 0.0;
}

/* k(Q) for an array of quadric values */
void orc_kernel_many(const orc_cfg *cfg, int64_t m, const double *Q, double *out) {
  double x0 = (cfg->kind == ORC_KERNEL_POLY) ? orc_first_root(cfg->c, cfg->order, 0.0) : 0.0;
  for (int64_t i = 0; i < m; ++i) out[i] = orc_kernel(cfg, x0, Q[i]);
}

/* ------------------------------------------------------------------ */
/* real spherical harmonics up to degree 3, orthonormal on the sphere  */
/* ------------------------------------------------------------------ */

/* Y_k(d) for k = 0..(deg+1)^2-1 at the unit direction (x, y, z), in the
 * ordering and sign convention used by 3DGS colour coefficients
 * (m = -l..l within each band, Condon-Shortley phase on odd m). */
void orc_sh_basis(int deg, double x, double y, double z, double *Y) {
  const double PI = 3.14159265358979323846;
  Y[0] = sqrt(1.0 / (4.0 * PI));
  if (deg < 1) return;
  double k1 = sqrt(3.0 / (4.0 * PI));
  Y[1] = -k1 * y;
  Y[2] = k1 * z;
  Y[3] = -k1 * x;
  if (deg < 2) return;
  double k2a = sqrt(15.0 / (4.0 * PI));
  double k2b = sqrt(5.0 / (16.0 * PI));
  double k2c = sqrt(15.0 / (16.0 * PI));
  Y[4] = k2a * x * y;
  Y[5] = -k2a * y * z;
  Y[6] = k2b * (2.0 * z * z - x * x - y * y);
  Y[7] = -k2a * x * z;
  Y[8] = k2c * (x * x - y * y);
  if (deg < 3) return;
  double k3a = sqrt(35.0 / (32.0 * PI));
  double k3b = sqrt(105.0 / (4.0 * PI));
  double k3c = sqrt(21.0 / (32.0 * PI));
  double k3d = sqrt(7.0 / (16.0 * PI));
  double k3e = sqrt(105.0 / (16.0 * PI));
  Y[9] = -k3a * y * (3.0 * x * x - y * y);
  Y[10] = k3b * x * y * z;
  Y[11] = -k3c * y * (4.0 * z * z - x * x - y * y);
  Y[12] = k3d * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
  Y[13] = -k3c * x * (4.0 * z * z - x * x - y * y);
  Y[14] = k3e * z * (x * x - y * y);
  Y[15] = -k3a * x * (x * x - 3.0 * y * y);
}

/* ------------------------------------------------------------------ */
/* projection of one splat                                              */
/* ------------------------------------------------------------------ */

static int near_integer(double e) { return fabs(e - nearbyint(e)) < 1e-9; }

static long clamp_floor(double e, long lo, long hi) {
  if (!(e >= (double)lo)) return lo; /* also catches NaN */
  if (e >= (double)hi + 1.0) return hi;
  long f = (long)floor(e);
  if (f < lo) f = lo;
  if (f > hi) f = hi;
  return f;
}

/* Could another FP64 evaluation of X, at most w away from this one, round
 * to a different float? When a float rounding midpoint (or X itself being
 * one) lies within w of X, returns 1 and the float on the far side of that
 * midpoint in *alt; otherwise 0 and the float of X. */
static int float_rounding_alt(double X, double w, double *alt) {
  float f = (float)X;
  *alt = (double)f;
  if (!isfinite(X)) return 0;
  double up = (double)nextafterf(f, INFINITY), dn = (double)nextafterf(f, -INFINITY);
  double mu = 0.5 * ((double)f + up), md = 0.5 * ((double)f + dn); /* exact in double */
  if (fabs(X - mu) <= w && fabs(X - mu) <= fabs(X - md)) {
    *alt = up;
    return 1;
  }
  if (fabs(X - md) <= w) {
    *alt = dn;
    return 1;
  }
  return 0;
}

/* Projects n splats. Inputs (double; the single-precision scene converts
 * exactly) are the scene in activated form: scales are
 * standard deviations, quats are (w, x, y, z) and need not be normalised,
 * opacity in [0, 1], sh is [n][(deg+1)^2][3].
 * Outputs (per splat): means2d[2], conic[3] = upper triangle (a, b, c) of
 * the inverse of the anti-aliased covariance, opac = anti-aliased opacity,
 * rgb[3], depth (camera z), depth32 (z rounded to float), radius (pixels),
 * rect[4] = inclusive tile rectangle (x_lo, y_lo, x_hi, y_hi) or
 * (0, 0, -1, -1) when empty, tiles = tiles in the rectangle, flags.
 *
 * Record rounding. The renderer consumes the record rounded to float, and
 * any FP64 evaluation of it (this one or another program's, by another
 * route) carries rounding error; where a float rounding midpoint lies that
 * close, two correct programs may hold floats one ulp apart. A first-order
 * running error bound E is carried through the computation of each of
 * u, v, a, b, c and o (unit roundoff 2^-53 times 16 per step, above the
 * n u of a sum of n <= 11 rounded products,
 * applied to sums of absolute values, so it bounds any evaluation order of
 * the same formulas); rec_err [n][6] receives E (may be NULL), and bit k of
 * rec_amb [n] is set when entry k (u, v, a, b, c, o) has a rounding
 * midpoint within 2 E: two evaluations each within E of the exact value
 * can round that entry apart, no others can. rec_alt [n][6] (may be NULL)
 * holds the float on the other side of that midpoint (the entry's own
 * float where the bit is clear): for such an entry both floats are correct. The thin footprints of large
 * anisotropic splats are where this matters: the anti-aliased determinant
 * A00 A11 - S01^2 still cancels by up to ~1e5 (v bounds it), and the raw
 * |Sigma'| by up to 1e11 and more, which is why |Sigma'| is evaluated as a
 * sum of squares (below). */
void orc_project(const orc_cfg *cfg, const orc_cam *cam, int64_t n,
                 const double *means3d, const double *scales, const double *quats,
                 const double *opacity, const double *sh, int32_t sh_degree,
                 double *means2d, double *conic, double *opac, double *rgb,
                 double *depth, float *depth32, double *radius, int32_t *rect,
                 int64_t *tiles, uint8_t *flags, uint8_t *rec_amb, double *rec_err, double *rec_alt) {
  const int T = cfg->tile;
  const long gx = (cam->width + T - 1) / T, gy = (cam->height + T - 1) / T;
  const int nsh = (sh_degree + 1) * (sh_degree + 1);
  const double x0 = (cfg->kind == ORC_KERNEL_POLY || cfg->radius_mode == ORC_RADIUS_POLY_UNIVERSAL ||
                     cfg->radius_mode == ORC_RADIUS_POLY_OPACITY)
                        ? orc_first_root(cfg->c, cfg->order, 0.0)
                        : 0.0;
  const double *Rc = cam->R;
  /* camera centre in world space: -R^T t */
  double campos[3];
  for (int i = 0; i < 3; ++i)
    campos[i] = -(Rc[0 * 3 + i] * cam->t[0] + Rc[1 * 3 + i] * cam->t[1] + Rc[2 * 3 + i] * cam->t[2]);

#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double m[3] = {means3d[3 * i], means3d[3 * i + 1], means3d[3 * i + 2]};
    double tc[3];
    for (int r = 0; r < 3; ++r)
      tc[r] = Rc[3 * r + 0] * m[0] + Rc[3 * r + 1] * m[1] + Rc[3 * r + 2] * m[2] + cam->t[r];

    means2d[2 * i] = means2d[2 * i + 1] = 0.0;
    conic[3 * i] = conic[3 * i + 1] = conic[3 * i + 2] = 0.0;
    opac[i] = 0.0;
    rgb[3 * i] = rgb[3 * i + 1] = rgb[3 * i + 2] = 0.0;
    depth[i] = tc[2];
    depth32[i] = (float)tc[2];
    radius[i] = 0.0;
    rect[4 * i] = 0; rect[4 * i + 1] = 0; rect[4 * i + 2] = -1; rect[4 * i + 3] = -1;
    tiles[i] = 0;
    flags[i] = 0;
    if (rec_amb) rec_amb[i] = 0;
    if (rec_err)
      for (int k2 = 0; k2 < 6; ++k2) rec_err[6 * i + k2] = 0.0;
    if (rec_alt)
      for (int k2 = 0; k2 < 6; ++k2) rec_alt[6 * i + k2] = 0.0;

    if (tc[2] < cfg->near_z) continue;

    /* 3D covariance: Sigma = R(q) diag(s)^2 R(q)^T */
    double qw = quats[4 * i], qx = quats[4 * i + 1], qy = quats[4 * i + 2], qz = quats[4 * i + 3];
    double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw /= qn; qx /= qn; qy /= qn; qz /= qn;
    double Rq[3][3] = {
        {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
        {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
        {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
    double s2[3] = {scales[3 * i] * scales[3 * i], scales[3 * i + 1] * scales[3 * i + 1],
                    scales[3 * i + 2] * scales[3 * i + 2]};
    double Sig[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += Rq[a][k] * s2[k] * Rq[b][k];
        Sig[a][b] = acc;
      }

    /* EWA: Sigma' = J W Sigma W^T J^T, J the Jacobian of the perspective map
     * at the camera-space mean, with x/z and y/z clamped to 1.3 tan(fov/2). */
    double tz = tc[2];
    double limx = 1.3 * (cam->width / (2.0 * cam->fx));
    double limy = 1.3 * (cam->height / (2.0 * cam->fy));
    double txz = tc[0] / tz, tyz = tc[1] / tz;
    if (txz < -limx) txz = -limx;
    if (txz > limx) txz = limx;
    if (tyz < -limy) tyz = -limy;
    if (tyz > limy) tyz = limy;
    double J[2][3] = {{cam->fx / tz, 0.0, -cam->fx * txz / tz},
                      {0.0, cam->fy / tz, -cam->fy * tyz / tz}};
    double TW[2][3];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += J[a][k] * Rc[3 * k + b];
        TW[a][b] = acc;
      }
    double S2[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) acc += TW[a][k] * Sig[k][l] * TW[b][l];
        S2[a][b] = acc;
      }
    double sxy = 0.5 * (S2[0][1] + S2[1][0]);

    /* anti-aliasing (Sec. 3.4). |Sigma'| is the determinant of M M^T with
     * M = TW Rq diag(s) (2x3); by Lagrange's identity that is the squared norm
     * of the cross product of M's rows. A rotation commutes with the cross
     * product and a diagonal scaling maps x cross y to (s1 s2, s0 s2, s0 s1)
     * times it, so |Sigma'| = sum_k sig_k^2 n_k^2 with n = Rq^T (TW_0 x TW_1)
     * and sig = (s1 s2, s0 s2, s0 s1): a sum of squares, which keeps its
     * relative accuracy where S00 S11 - S01^2 cancels (thin footprints, whose
     * opacity scale sqrt(|Sigma'| / |Sigma' + vI|) is otherwise lost). */
    double cw[3] = {TW[0][1] * TW[1][2] - TW[0][2] * TW[1][1], TW[0][2] * TW[1][0] - TW[0][0] * TW[1][2],
                    TW[0][0] * TW[1][1] - TW[0][1] * TW[1][0]};
    double nl[3], sg[3] = {scales[3 * i + 1] * scales[3 * i + 2], scales[3 * i] * scales[3 * i + 2],
                           scales[3 * i] * scales[3 * i + 1]};
    double det0 = 0.0;
    for (int k = 0; k < 3; ++k) {
      nl[k] = Rq[0][k] * cw[0] + Rq[1][k] * cw[1] + Rq[2][k] * cw[2];
      det0 += sg[k] * sg[k] * nl[k] * nl[k];
    }
    double A00 = S2[0][0] + cfg->aa_v, A11 = S2[1][1] + cfg->aa_v;
    double deta = A00 * A11 - sxy * sxy;
    if (!(deta > 0.0)) continue;
    double ratio = det0 / deta;
    double o = opacity[i] * sqrt(ratio > 0.0 ? ratio : 0.0);

    double u = cam->fx * tc[0] / tz + cam->cx;
    double v = cam->fy * tc[1] / tz + cam->cy;

    /* bounding radius, r = k sqrt(lambda_max) (Sec. 2.1 and Sec. 3.2) */
    double mid = 0.5 * (A00 + A11);
    double disc = mid * mid - deta;
    double lmax = mid + sqrt(disc > 0.0 ? disc : 0.0);
    double k;
    int cull = 0, cull_near = 0;
    switch (cfg->radius_mode) {
      case ORC_RADIUS_SIGMA3:
        k = 3.0;
        break;
      case ORC_RADIUS_POLY_UNIVERSAL:
        k = sqrt(x0);
        break;
      case ORC_RADIUS_POLY_OPACITY: {
        /* opacity-dependent: first root of o p(x) = eps, i.e. p(x) = eps / o */
        double target = cfg->eps / o;
        double c0 = cfg->c[0];
        cull_near = fabs(o * c0 - cfg->eps) <= 1e-9 * cfg->eps;
        double xr = (o > 0.0) ? orc_first_root(cfg->c, cfg->order, target) : -1.0;
        if (xr < 0.0) { cull = 1; k = 0.0; } else k = sqrt(xr);
        break;
      }
      default: { /* ORC_RADIUS_EXP_OPACITY: the Mahalanobis radius where o exp(-x/2) = eps */
        cull_near = fabs(o - cfg->eps) <= 1e-9 * cfg->eps;
        if (!(o >= cfg->eps)) { cull = 1; k = 0.0; } else k = sqrt(2.0 * log(o / cfg->eps));
        break;
      }
    }
    if (cull_near) flags[i] |= ORC_SPLAT_CULL_NEAR;
    if (cull) continue;
    double r = k * sqrt(lmax) * cfg->radius_pad;
    /* the rectangle's half sides: the square of radius r around the mean
     * (Sec. 2.1), or the axis-aligned box of the ellipse Q = k^2, whose half
     * sides are k times the standard deviations along x and y (the square
     * roots of the anti-aliased covariance's diagonal) */
    double hx = r, hy = r;
    if (cfg->rect_mode == ORC_RECT_ELLIPSE_BOX) {
      hx = k * sqrt(A00) * cfg->radius_pad;
      hy = k * sqrt(A11) * cfg->radius_pad;
    }

    double ex0 = (u - hx) / T, ex1 = (u + hx) / T, ey0 = (v - hy) / T, ey1 = (v + hy) / T;
    if (near_integer(ex0) || near_integer(ex1) || near_integer(ey0) || near_integer(ey1))
      flags[i] |= ORC_SPLAT_EDGE_NEAR;
    long xlo = clamp_floor(ex0, 0, gx), xhi = clamp_floor(ex1, -1, gx - 1);
    long ylo = clamp_floor(ey0, 0, gy), yhi = clamp_floor(ey1, -1, gy - 1);
    long nt = (xhi >= xlo && yhi >= ylo) ? (xhi - xlo + 1) * (yhi - ylo + 1) : 0;

    /* running error bounds of the record (see the comment above) */
    {
      const double g = 16.0 * 0x1p-53;
      double etc[3];
      for (int r2 = 0; r2 < 3; ++r2)
        etc[r2] = g * (fabs(Rc[3 * r2]) * fabs(m[0]) + fabs(Rc[3 * r2 + 1]) * fabs(m[1]) +
                       fabs(Rc[3 * r2 + 2]) * fabs(m[2]) + fabs(cam->t[r2]));
      const double az = fabs(tz);
      /* x/z, y/z and their bounds; a clamped one is a constant */
      double etxz = (fabs(tc[0] / tz) >= limx) ? g * limx : etc[0] / az + fabs(tc[0]) * etc[2] / (az * az) + g * fabs(txz);
      double etyz = (fabs(tc[1] / tz) >= limy) ? g * limy : etc[1] / az + fabs(tc[1]) * etc[2] / (az * az) + g * fabs(tyz);
      double eJ[2][3] = {{cam->fx * etc[2] / (az * az) + g * fabs(J[0][0]), 0.0,
                          cam->fx * (etxz / az + fabs(txz) * etc[2] / (az * az)) + g * fabs(J[0][2])},
                         {0.0, cam->fy * etc[2] / (az * az) + g * fabs(J[1][1]),
                          cam->fy * (etyz / az + fabs(tyz) * etc[2] / (az * az)) + g * fabs(J[1][2])}};
      double eTW[2][3], aTW[2][3];
      for (int a2 = 0; a2 < 2; ++a2)
        for (int b2 = 0; b2 < 3; ++b2) {
          double e = 0.0, sa = 0.0;
          for (int k2 = 0; k2 < 3; ++k2) {
            e += eJ[a2][k2] * fabs(Rc[3 * k2 + b2]);
            sa += fabs(J[a2][k2]) * fabs(Rc[3 * k2 + b2]);
          }
          eTW[a2][b2] = e + g * sa;
          aTW[a2][b2] = fabs(TW[a2][b2]) + eTW[a2][b2];
        }
      /* Sigma: every rotation entry within 4 g of its value (normalised quaternion) */
      double eSig[3][3], aSig[3][3];
      for (int a2 = 0; a2 < 3; ++a2)
        for (int b2 = 0; b2 < 3; ++b2) {
          double e = 0.0, sa = 0.0;
          for (int k2 = 0; k2 < 3; ++k2) {
            e += 4.0 * g * (fabs(Rq[a2][k2]) + fabs(Rq[b2][k2]) + 4.0 * g) * s2[k2];
            sa += fabs(Rq[a2][k2]) * s2[k2] * fabs(Rq[b2][k2]);
          }
          eSig[a2][b2] = e + 2.0 * g * sa;
          aSig[a2][b2] = fabs(Sig[a2][b2]) + eSig[a2][b2];
        }
      double eS2[2][2];
      for (int a2 = 0; a2 < 2; ++a2)
        for (int b2 = 0; b2 < 2; ++b2) {
          double e = 0.0, sa = 0.0;
          for (int k2 = 0; k2 < 3; ++k2)
            for (int l2 = 0; l2 < 3; ++l2) {
              e += eTW[a2][k2] * aSig[k2][l2] * aTW[b2][l2] + fabs(TW[a2][k2]) * eSig[k2][l2] * aTW[b2][l2] +
                   fabs(TW[a2][k2]) * fabs(Sig[k2][l2]) * eTW[b2][l2];
              sa += fabs(TW[a2][k2]) * fabs(Sig[k2][l2]) * fabs(TW[b2][l2]);
            }
          eS2[a2][b2] = e + g * sa;
        }
      const double exy = 0.5 * (eS2[0][1] + eS2[1][0]) + g * fabs(sxy);
      const double eA00 = eS2[0][0] + g * A00, eA11 = eS2[1][1] + g * A11;
      const double edeta = eA00 * A11 + A00 * eA11 + 2.0 * fabs(sxy) * exy + g * (A00 * A11 + sxy * sxy);
      /* |Sigma'| as the sum of squares above: the cross product of TW's rows,
       * its rotation into the splat's frame (rotation entries within 4 g) and
       * the weighted squares (sig_k exact: a product of two floats) */
      double ecw[3], edet0 = 3.0 * g * det0;
      for (int k2 = 0; k2 < 3; ++k2) {
        const int a2 = (k2 + 1) % 3, b2 = (k2 + 2) % 3;
        ecw[k2] = eTW[0][a2] * aTW[1][b2] + fabs(TW[0][a2]) * eTW[1][b2] + eTW[0][b2] * aTW[1][a2] +
                  fabs(TW[0][b2]) * eTW[1][a2] + g * (fabs(TW[0][a2] * TW[1][b2]) + fabs(TW[0][b2] * TW[1][a2]));
      }
      for (int k2 = 0; k2 < 3; ++k2) {
        double en = 0.0;
        for (int j2 = 0; j2 < 3; ++j2)
          en += (fabs(Rq[j2][k2]) + 4.0 * g) * ecw[j2] + 4.0 * g * fabs(cw[j2]) + g * fabs(Rq[j2][k2] * cw[j2]);
        edet0 += sg[k2] * sg[k2] * (2.0 * fabs(nl[k2]) * en + en * en);
      }
      double E[6];
      E[0] = cam->fx * (etc[0] / az + fabs(tc[0]) * etc[2] / (az * az)) + g * (fabs(u) + fabs(cam->cx));
      E[1] = cam->fy * (etc[1] / az + fabs(tc[1]) * etc[2] / (az * az)) + g * (fabs(v) + fabs(cam->cy));
      if (edeta < 0.5 * deta) {
        const double id2 = 1.0 / (deta * deta);
        E[2] = eA11 / deta + A11 * edeta * id2 + g * fabs(A11 / deta);
        E[3] = exy / deta + fabs(sxy) * edeta * id2 + g * fabs(sxy / deta);
        E[4] = eA00 / deta + A00 * edeta * id2 + g * fabs(A00 / deta);
        const double eratio = edet0 / deta + fabs(det0) * edeta * id2 + g * fabs(ratio);
        const double rhi = ratio + eratio, rlo = ratio - eratio;
        E[5] = opacity[i] * (sqrt(rhi > 0.0 ? rhi : 0.0) - sqrt(rlo > 0.0 ? rlo : 0.0)) + g * o;
      } else {
        E[2] = E[3] = E[4] = E[5] = INFINITY;
      }
      const double X[6] = {u, v, A11 / deta, -sxy / deta, A00 / deta, o};
      uint8_t amb = 0;
      for (int k2 = 0; k2 < 6; ++k2) {
        double alt;
        if (float_rounding_alt(X[k2], 2.0 * E[k2], &alt)) amb |= (uint8_t)(1u << k2);
        if (rec_alt) rec_alt[6 * i + k2] = alt;
        if (rec_err) rec_err[6 * i + k2] = E[k2];
      }
      if (rec_amb) rec_amb[i] = amb;
    }

    means2d[2 * i] = u;
    means2d[2 * i + 1] = v;
    conic[3 * i] = A11 / deta;
    conic[3 * i + 1] = -sxy / deta;
    conic[3 * i + 2] = A00 / deta;
    opac[i] = o;
    radius[i] = r;
    /* an empty rectangle is stored as (0, 0, -1, -1), except for a splat whose
     * edge sits on a tile boundary: there the clamped bounds are kept so the
     * renderer can flag the pixels next to that edge */
    if (nt > 0 || (flags[i] & ORC_SPLAT_EDGE_NEAR)) {
      rect[4 * i] = (int32_t)xlo; rect[4 * i + 1] = (int32_t)ylo;
      rect[4 * i + 2] = (int32_t)xhi; rect[4 * i + 3] = (int32_t)yhi;
    }
    tiles[i] = nt;

    /* view-dependent colour, direction from the camera centre to the mean */
    double d[3] = {m[0] - campos[0], m[1] - campos[1], m[2] - campos[2]};
    double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double Y[16];
    orc_sh_basis(sh_degree, d[0] / dn, d[1] / dn, d[2] / dn, Y);
    for (int ch = 0; ch < 3; ++ch) {
      double acc = 0.0;
      for (int kk = 0; kk < nsh; ++kk) acc += Y[kk] * sh[(i * nsh + kk) * 3 + ch];
      acc += 0.5;
      rgb[3 * i + ch] = acc > 0.0 ? acc : 0.0;
    }
  }
}

/* ------------------------------------------------------------------ */
/* depth order                                                          */
/* ------------------------------------------------------------------ */

typedef struct { float d; int64_t i; } orc_order_item;

static int order_cmp(const void *a, const void *b) {
  const orc_order_item *x = (const orc_order_item *)a, *y = (const orc_order_item *)b;
  if (x->d < y->d) return -1;
  if (x->d > y->d) return 1;
  return (x->i < y->i) ? -1 : (x->i > y->i);
}

/* Splat order for compositing: ascending depth32, ties broken by index. */
void orc_depth_order(int64_t n, const float *depth32, int64_t *order_out) {
  orc_order_item *it = (orc_order_item *)malloc(sizeof(orc_order_item) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) { it[i].d = depth32[i]; it[i].i = i; }
  qsort(it, (size_t)n, sizeof(orc_order_item), order_cmp);
  for (int64_t i = 0; i < n; ++i) order_out[i] = it[i].i;
  free(it);
}

/* ------------------------------------------------------------------ */
/* compositing                                                          */
/* ------------------------------------------------------------------ */

/* Renders npix pixels given by integer coordinates px[2*j], px[2*j+1].
 * The splat records are the projection outputs (any precision the caller
 * chooses to round them to, held here as doubles); order is the depth order.
 * Per pixel: colour[3], final transmittance, number of blended splats,
 * number of evaluated splats (candidates up to and including a terminating
 * one), 1 + list position of the last blended splat (0 if none), and flags
 * for decisions that sit too close to a threshold to be reproduced by a
 * single-precision evaluation. splat_flags may be NULL. */
/* ------------------------------------------------------------------ */
/* per-tile culling (the tile test of StopThePop, Sec. 2.1 and Sec. 4)   */
/* ------------------------------------------------------------------ */
/*
 * A splat enters a tile's list only when the point of the tile where it
 * contributes most can pass alpha >= eps. The kernels decrease in Q, so that
 * point minimises Q over the rectangle holding the tile's pixel centres, and
 * the test is: that minimum <= cut. cut is not the exact threshold but a
 * bound that makes the test safe for a float renderer: the threshold of
 * alpha >= eps on Q for the kernel with float coefficients, in double, plus
 * (1) 2^-16 (|thr| + 16), giving T, and (2) the widening
 * cut = (sqrt(T) (1 + 2^-18) + D)^2 (1 + 2^-30) with
 * D = 2^-19 (4 sqrt(T) + 16 sqrt(det/c) + 8 |b| sqrt(T/det) + 16 |b|/sqrt(c)
 * + 32 sqrt(c)), det = a c - b^2 of the conic (a, b, c). These terms bound
 * the rounding of a float evaluation of the quadric at tile-local pixel
 * offsets with a wide margin; the oracle takes them as part of the
 * definition (a renderer that culls with the same formula keeps the same
 * copies). Below, every operation is a plain IEEE double operation in the
 * order written (the library is built without contraction), so a renderer
 * computing the same formula in double takes the same decision unless Q's
 * minimum lies within a few ulps of cut; such decisions are reported near.
 */

/* threshold on Q of o k(Q) >= eps for the kernel with float coefficients
 * (the renderer's), negative when no Q passes */
static double cull_threshold(const orc_cfg *cfg, double o) {
  const double eps = (double)(float)cfg->eps;
  if (cfg->kind == ORC_KERNEL_EXP) return 2.0 * log(o / eps); /* o exp(-Q/2) = eps */
  double cf[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i <= cfg->order; ++i) cf[i] = (double)(float)cfg->c[i];
  if (cfg->order == 1) return (eps / o - cf[0]) / cf[1]; /* o (c_0 + c_1 Q) = eps */
  return orc_first_root(cf, cfg->order, eps / o);        /* -1 when o c_0 < eps */
}

/* the cut above for a record (opacity o, conic a, b, c); -1 when no pixel
 * can pass (o <= 0, conic not positive definite, T < 0) */
double orc_cull_cut(const orc_cfg *cfg, double o, double a, double b, double c) {
  if (!(o > 0.0) || !(a > 0.0) || !(c > 0.0)) return -1.0;
  const double det = a * c - b * b;
  if (!(det > 0.0)) return -1.0;
  const double thr = cull_threshold(cfg, o);
  const double T = thr + 0x1p-16 * (fabs(thr) + 16.0);
  if (!(T >= 0.0)) return -1.0;
  const double sT = sqrt(T), ab = fabs(b);
  const double D = 0x1p-19 * (4.0 * sT + 16.0 * sqrt(det / c) + 8.0 * ab * sqrt(T / det) + 16.0 * ab / sqrt(c) +
                              32.0 * sqrt(c));
  const double r = sT * (1.0 + 0x1p-18) + D;
  return r * r * (1.0 + 0x1p-30);
}

/* least Q = a dx^2 + 2 b dx dy + c dy^2 over the rectangle [x0, x1] x [y0, y1]
 * of offsets from the mean, for a positive-definite conic: 0 when the mean is
 * inside; otherwise the minimum lies on an edge. Along an edge of fixed dy
 * completing the square gives Q = a (dx + b dy / a)^2 + (det / a) dy^2, least
 * at dx = -b dy / a clamped to the edge; likewise along an edge of fixed dx
 * with the roles of a and c exchanged. */
double orc_rect_min_q(double a, double b, double c, double x0, double x1, double y0, double y1) {
  if (x0 <= 0.0 && x1 >= 0.0 && y0 <= 0.0 && y1 >= 0.0) return 0.0;
  const double det = a * c - b * b;
  double best = INFINITY;
  const double ys[2] = {y0, y1}, xs[2] = {x0, x1};
  for (int e = 0; e < 2; ++e) {
    double y = ys[e], xv = -(b * y) / a;
    double dx = fmin(fmax(xv, x0), x1) - xv;
    double q = a * (dx * dx) + (det / a) * (y * y);
    if (q < best) best = q;
    double x = xs[e], yv = -(b * x) / c;
    double dy = fmin(fmax(yv, y0), y1) - yv;
    q = c * (dy * dy) + (det / c) * (x * x);
    if (q < best) best = q;
  }
  return best;
}

/* the tile test for splat (mean u, v; conic a, b, c; cut) and tile (tx, ty):
 * 1 keep, 0 drop; *near = 1 when the minimum is within 2^-40 of cut
 * (relative), where a double evaluation in another order may decide the
 * other way */
int orc_tile_keep(double u, double v, double a, double b, double c, double cut, int tx, int ty, int T, int *near) {
  *near = 0;
  if (!(cut >= 0.0)) return 0;
  const double x0 = ((double)(tx * T) + 0.5) - u, x1 = ((double)(tx * T + T) - 0.5) - u;
  const double y0 = ((double)(ty * T) + 0.5) - v, y1 = ((double)(ty * T + T) - 0.5) - v;
  const double q = orc_rect_min_q(a, b, c, x0, x1, y0, y1);
  if (fabs(q - cut) <= 0x1p-40 * cut) *near = 1;
  return q <= cut;
}

/* cut for every splat of a projection (records as doubles) */
void orc_cull_cuts(const orc_cfg *cfg, int64_t n, const double *conic, const double *opac, double *cut) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    cut[i] = orc_cull_cut(cfg, opac[i], conic[3 * i], conic[3 * i + 1], conic[3 * i + 2]);
}

/* kept copies per tile (hist [gw * gh]) and near decisions per tile
 * (near [gw * gh]) over every tile of every splat's rectangle */
void orc_cull_histogram(const orc_cfg *cfg, int64_t n, const double *means2d, const double *conic,
                        const double *cut, const int32_t *rect, int gw, int gh, int64_t *hist, int64_t *near) {
  const int64_t nt = (int64_t)gw * gh;
  memset(hist, 0, sizeof(int64_t) * nt);
  memset(near, 0, sizeof(int64_t) * nt);
#pragma omp parallel
  {
    int64_t *h = calloc((size_t)(2 * nt), sizeof(int64_t));
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      const int32_t *r = rect + 4 * i;
      for (int ty = r[1]; ty <= r[3]; ++ty)
        for (int tx = r[0]; tx <= r[2]; ++tx) {
          int nr;
          int k = orc_tile_keep(means2d[2 * i], means2d[2 * i + 1], conic[3 * i], conic[3 * i + 1],
                                conic[3 * i + 2], cut[i], tx, ty, cfg->tile, &nr);
          h[(int64_t)ty * gw + tx] += k;
          h[nt + (int64_t)ty * gw + tx] += nr;
        }
    }
#pragma omp critical
    for (int64_t t = 0; t < nt; ++t) {
      hist[t] += h[t];
      near[t] += h[nt + t];
    }
    free(h);
  }
}

/* the test for every copy of every rectangle, in the order the copies are
 * listed before sorting (splats in index order, each rectangle's tiles
 * row-major): keep [sum of rectangle areas], starting at start[i] for splat i;
 * returns the number of near decisions */
int64_t orc_cull_copy_mask(const orc_cfg *cfg, int64_t n, const double *means2d, const double *conic,
                           const double *cut, const int32_t *rect, const int64_t *start, uint8_t *keep) {
  int64_t nnear = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : nnear)
  for (int64_t i = 0; i < n; ++i) {
    const int32_t *r = rect + 4 * i;
    int64_t k = start[i];
    for (int ty = r[1]; ty <= r[3]; ++ty)
      for (int tx = r[0]; tx <= r[2]; ++tx) {
        int nr;
        keep[k++] = (uint8_t)orc_tile_keep(means2d[2 * i], means2d[2 * i + 1], conic[3 * i], conic[3 * i + 1],
                                           conic[3 * i + 2], cut[i], tx, ty, cfg->tile, &nr);
        nnear += nr;
      }
  }
  return nnear;
}

/* per splat: whether tile (tx, ty) is in its rectangle and passes the test
 * (keep [n]) and whether that decision is near (near [n]) */
void orc_cull_tile_members(const orc_cfg *cfg, int64_t n, const double *means2d, const double *conic,
                           const double *cut, const int32_t *rect, int tx, int ty, uint8_t *keep, uint8_t *near) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const int32_t *r = rect + 4 * i;
    keep[i] = near[i] = 0;
    if (tx < r[0] || tx > r[2] || ty < r[1] || ty > r[3]) continue;
    int nr;
    keep[i] = (uint8_t)orc_tile_keep(means2d[2 * i], means2d[2 * i + 1], conic[3 * i], conic[3 * i + 1],
                                     conic[3 * i + 2], cut[i], tx, ty, cfg->tile, &nr);
    near[i] = (uint8_t)nr;
  }
}

/* Brute-force compositing of the requested pixels (see the file header).
 *
 * reach (may be NULL, else [npix, 2]): per pixel, bounds on how far the
 * colour (any channel) and the final T can move
 * when the decisions the pixel's flags mark are taken the other way (reading
 * G13). Every colour is non-negative, so what a pixel still gathers from
 * transmittance T on lies in [0, T (R + B)], R the largest rgb entry of any
 * splat and B the largest background entry. Hence
 *   - a pair whose inclusion is uncertain (alpha within the band of eps, a
 *     rectangle edge or a tile-culling test within rounding) and that can
 *     have alpha a there changes the colour by at most a T (rgb_i + R + B):
 *     its own term, and the factor (1 - a) on everything behind it; it
 *     also leaves T uncertain by the relative amount a;
 *   - a stop decision within its band, widened by that accumulated
 *     uncertainty of T, changes it by at most T (R + B), the whole remainder,
 *     which also covers every later decision.
 * reach is the sum of these terms (0 for unflagged pixels); the bound on T
 * takes the same terms without the colour factors (a T, and T). */
void orc_render_pixels(const orc_cfg *cfg, int64_t n, const int64_t *order,
                       const double *means2d, const double *conic, const double *opac,
                       const double *rgb, const int32_t *rect, const uint8_t *splat_flags,
                       int64_t npix, const int32_t *px, double *color, double *final_T,
                       int32_t *n_contrib, int32_t *n_eval, int32_t *last_contrib,
                       uint8_t *pix_flags, double *reach) {
  const int T = cfg->tile;
  const double x0 = (cfg->kind == ORC_KERNEL_POLY) ? orc_first_root(cfg->c, cfg->order, 0.0) : 0.0;
  double *cut = NULL;
  if (cfg->tile_cull) {
    cut = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    orc_cull_cuts(cfg, n, conic, opac, cut);
  }
  double crange = 0.0; /* R + B of the reach bound */
  for (int64_t i = 0; i < 3 * n; ++i)
    if (rgb[i] > crange) crange = rgb[i];
  {
    double bmax = 0.0;
    for (int ch = 0; ch < 3; ++ch)
      if (fabs(cfg->bg[ch]) > bmax) bmax = fabs(cfg->bg[ch]);
    crange += bmax;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t j = 0; j < npix; ++j) {
    int x = px[2 * j], y = px[2 * j + 1];
    int tx = x / T, ty = y / T;
    double cx = x + 0.5, cy = y + 0.5;
    double Tr = 1.0, C[3] = {0.0, 0.0, 0.0};
    int32_t ncon = 0, nev = 0, last = 0;
    uint8_t fl = 0;
    double rch = 0.0, rchT = 0.0, unc = 0.0; /* reach of colour and of T so far; relative uncertainty of Tr */
    int capped = 0;              /* a stop decision was uncertain: rch covers the rest */
    for (int64_t s = 0; s < n; ++s) {
      int64_t i = order[s];
      const int32_t *rc = rect + 4 * i;
      int uncertain = 0; /* membership of this pair in the pixel's list may differ */
      if (splat_flags && (splat_flags[i] & ORC_SPLAT_EDGE_NEAR)) {
        /* a rectangle edge this close to a tile boundary may land on either side */
        if (tx >= rc[0] - 1 && tx <= rc[2] + 1 && ty >= rc[1] - 1 && ty <= rc[3] + 1 &&
            (tx <= rc[0] || tx >= rc[2] || ty <= rc[1] || ty >= rc[3])) {
          fl |= ORC_PIX_EDGE_NEAR;
          uncertain = 1;
        }
      }
      int member = tx >= rc[0] && tx <= rc[2] && ty >= rc[1] && ty <= rc[3];
      if (member && cut) { /* tile culling: the list holds the splat only if the tile passes */
        int nr;
        int keep = orc_tile_keep(means2d[2 * i], means2d[2 * i + 1], conic[3 * i], conic[3 * i + 1],
                                 conic[3 * i + 2], cut[i], tx, ty, T, &nr);
        if (nr) {
          fl |= ORC_PIX_CULL_NEAR;
          uncertain = 1;
        }
        member = keep;
      }
      if (!member && !uncertain) continue;
      double dx = cx - means2d[2 * i], dy = cy - means2d[2 * i + 1];
      double A = conic[3 * i], B = conic[3 * i + 1], Cc = conic[3 * i + 2];
      double Q = A * dx * dx + 2.0 * B * dx * dy + Cc * dy * dy;
      double a = opac[i] * orc_kernel(cfg, x0, Q);
      if (a > cfg->alpha_max) a = cfg->alpha_max;
      const double rgbi = fmax(rgb[3 * i], fmax(rgb[3 * i + 1], rgb[3 * i + 2]));
      const int anear = member && fabs(a - cfg->eps) <= cfg->alpha_band;
      if (anear) fl |= ORC_PIX_ALPHA_NEAR;
      if (!capped && ((uncertain && a >= cfg->eps - cfg->alpha_band) || anear)) {
        /* this pair may be blended or not: its own term and the factor on what lies behind */
        const double ah = a > cfg->eps + cfg->alpha_band ? a : cfg->eps + cfg->alpha_band;
        rch += ah * Tr * (rgbi + crange);
        rchT += ah * Tr;
        unc += ah;
      }
      if (!member) continue;
      ++nev;
      if (a < cfg->eps) continue;
      double Tn = Tr * (1.0 - a);
      const int tnear = fabs(Tn - cfg->t_min) <= cfg->t_band_rel * cfg->t_min;
      if (tnear) fl |= ORC_PIX_T_NEAR;
      if (!capped && (tnear || (unc > 0.0 && fabs(Tn - cfg->t_min) <= (cfg->t_band_rel + unc) * fmax(Tn, cfg->t_min)))) {
        /* the stop may fall here or not: everything from here on is uncertain */
        fl |= ORC_PIX_T_NEAR;
        rch += Tr * crange;
        rchT += Tr;
        capped = 1;
      }
      if (Tn < cfg->t_min) break;
      for (int ch = 0; ch < 3; ++ch) C[ch] += rgb[3 * i + ch] * a * Tr;
      Tr = Tn;
      ++ncon;
      last = nev;
    }
    for (int ch = 0; ch < 3; ++ch) color[3 * j + ch] = C[ch] + Tr * cfg->bg[ch];
    final_T[j] = Tr;
    n_contrib[j] = ncon;
    n_eval[j] = nev;
    last_contrib[j] = last;
    pix_flags[j] = fl;
    if (reach) {
      reach[2 * j] = fl ? rch : 0.0;
      reach[2 * j + 1] = fl ? rchT : 0.0;
    }
  }
  free(cut);
}

/* number of threads OpenMP will use */
int orc_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
