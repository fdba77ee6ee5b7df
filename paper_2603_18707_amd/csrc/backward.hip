// Adjoint of blending (gs_rasterize_bwd) and of the projection (gs_preprocess_bwd).
//
// Blending adjoint: one workgroup of 256 threads per 16x16 tile, one pixel
// per lane, each wave an 8x8 block, with the forward's staged record,
// inclusion test and per-wave box test, so every (pixel, splat) decision
// matches the forward's and a wave visits only the records that can reach
// its block. The tile's list is staged back to front in batches of 256 from
// the last blended position of any pixel, and each wave walks its records
// back to front from its own pixels' last position. Per pixel the
// transmittance before a splat is recovered as T_i = T_{i+1} / (1 - alpha_i)
// from the stored final T, and the colour behind it follows the recurrence
// S_{i-1} = alpha_i c_i + (1 - alpha_i) S_i, so nothing per pair is stored.
// With g = dL/dC:
//   dL/dc_i     = alpha_i T_i g
//   dL/dalpha_i = T_i (c_i - S_i) . g - T_final / (1 - alpha_i) (bg . g)
// and alpha = min(alpha_max, o' k(Q)) gives dL/do' and dL/dQ (zero when the
// clamp is active); Q = d^T conic d gives the conic and mean gradients. An
// included pair has alpha >= eps > 0, so a polynomial kernel is strictly
// positive there: the ReLU kink never enters. Each lane adds its pair's nine
// partial gradients to the staged record's accumulators in LDS; after a
// batch, one thread per record adds them to global memory, so a splat costs
// nine global atomics per tile, whatever the number of pixels and waves.
//
// Projection adjoint: one thread per splat in double precision, the chain
// rule through the SH colour, the opacity factor sqrt(|S'| / |S' + vI|), the
// conic inverse, EWA (with the Jacobian's clamp), the camera transform, the
// rotation-scale factorisation and the quaternion normalisation.
#include <cmath>

#include "blend_common.h"
#include "gs_internal.h"
#include "project_common.h"

namespace gs {

namespace {

__global__ void zero_f32(float *p, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) p[i] = 0.0f;
}

// derivative of the polynomial at Q
__device__ inline float dpoly(const BlendParams &p, int order, float Q) {
  if (order == 1) return p.c[1];
  if (order == 2) return fmaf(2.0f * p.c[2], Q, p.c[1]);
  return fmaf(fmaf(3.0f * p.c[3], Q, 2.0f * p.c[2]), Q, p.c[1]);
}

__device__ inline float poly(const BlendParams &p, int order, float Q) {
  if (order == 1) return fmaf(p.c[1], Q, p.c[0]);
  if (order == 2) return fmaf(fmaf(p.c[2], Q, p.c[1]), Q, p.c[0]);
  return fmaf(fmaf(fmaf(p.c[3], Q, p.c[2]), Q, p.c[1]), Q, p.c[0]);
}

// Sums of v over the four rows of 16 lanes of the wave, each in every lane of
// its row: pairs, quads, half rows and rows by DPP moves (every lane of the
// wave must be active).
template <int CTRL, int ROWS>
__device__ inline float dpp_term(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
__device__ inline float row_sum(float v) {
  v += dpp_term<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_term<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_term<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_term<0x140, 0xF>(v);  // row_mirror
  return v;
}

constexpr int BT = 256;            // threads per tile in the adjoint
constexpr int BW = BT / WAVE;       // waves, each an 8x8 block
constexpr int NG = 9;               // partial gradients per record

template <int KIND>
__global__ __launch_bounds__(BT) void blend_bwd(BlendParams p, const float *__restrict__ means2d,
                                                const float *__restrict__ conic_opacity,
                                                const float *__restrict__ rgb, const uint32_t *__restrict__ vals,
                                                const uint32_t *__restrict__ ranges,
                                                const uint32_t *__restrict__ tile_order,
                                                const float *__restrict__ final_T,
                                                const uint32_t *__restrict__ last_contrib,
                                                const float *__restrict__ dL_dimage, float *__restrict__ dmeans2d,
                                                float *__restrict__ dconic, float *__restrict__ drgb) {
  __shared__ float4 L0[BT], L1[BT], L2[BT];
  __shared__ float2 L3[BT];              // (a, b) of the conic, for the gradients
  __shared__ uint32_t Lid[BT];
  __shared__ float G[NG][BT];            // the staged records' gradient accumulators
  __shared__ uint16_t lst[BW][BT];
  __shared__ uint32_t wcnt[BW][BW];
  __shared__ uint32_t wlast[BW];
  constexpr int ORDER = KIND == BLEND_POLY2 ? 2 : (KIND == BLEND_POLY3 ? 3 : 1);
  const int ntiles = p.gx * p.gy;
  if ((int)blockIdx.x >= ntiles) return;
  const int tile = tile_order ? (int)min(tile_order[blockIdx.x], (uint32_t)(ntiles - 1)) : (int)blockIdx.x;
  const int lane = threadIdx.x, wv = lane / WAVE, l64 = lane & (WAVE - 1);
  const uint64_t lt = (1ull << l64) - 1ull;
  const int tx = tile % p.gx, ty = tile / p.gx;
  const int wx0 = (wv & 1) * 8, wy0 = (wv >> 1) * 8;
  const int px = tx * TS + wx0 + (l64 & 7), py = ty * TS + wy0 + (l64 >> 3);
  const float fx = (float)(wx0 + (l64 & 7)) + 0.5f;  // pixel centre relative to the tile corner
  const float fy = (float)(wy0 + (l64 >> 3)) + 0.5f;
  const size_t plane = (size_t)p.W * p.H;
  float Tf = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
  uint32_t lastc = 0u;
  if (px < p.W && py < p.H) {
    const size_t pix = (size_t)py * p.W + px;
    Tf = final_T[pix];
    lastc = last_contrib[pix];
    g0 = dL_dimage[pix];
    g1 = dL_dimage[plane + pix];
    g2 = dL_dimage[2 * plane + pix];
  }
  float T = Tf, S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;
  const float bgg = p.bg[0] * g0 + p.bg[1] * g1 + p.bg[2] * g2;
  // the last blended position of the wave's and the tile's pixels
  uint32_t wmax = lastc;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) wmax = max(wmax, (uint32_t)__shfl_xor((int)wmax, o, 64));
  if (l64 == 0) wlast[wv] = wmax;
  __syncthreads();
  uint32_t maxlast = 0;
#pragma unroll
  for (int w = 0; w < BW; ++w) maxlast = max(maxlast, wlast[w]);

  const uint32_t start = ranges[2 * tile];
  const float tile_x0 = (float)(tx * TS), tile_y0 = (float)(ty * TS);
  // positions are 1-based within the tile: pos = index - start + 1
  for (int64_t hi = (int64_t)maxlast; hi > 0; hi -= BT) {
    const int64_t lo = hi - BT > 0 ? hi - BT : 0;
    const int cnt = (int)(hi - lo);
    // stage positions lo+1 .. hi (list indices start+lo .. start+hi-1); lane j holds position lo+1+j
    uint32_t mask = 0u;
#pragma unroll
    for (int k = 0; k < NG; ++k) G[k][lane] = 0.0f;
    if (lane < cnt) {
      uint32_t id = vals[start + lo + lane];
      if (id >= p.n) id = 0;  // never taken for a list built by gs_bin_sort over these n splats
      const float2 m = reinterpret_cast<const float2 *>(means2d)[id];
      const float4 co = reinterpret_cast<const float4 *>(conic_opacity)[id];
      const float3 c = make_float3(rgb[3 * id], rgb[3 * id + 1], rgb[3 * id + 2]);
      float4 a0, a1, a2;
      fold<KIND>(m, co, c, tile_x0, tile_y0, p, a0, a1, a2);
      L0[lane] = a0;
      L1[lane] = a1;
      L2[lane] = a2;
      L3[lane] = make_float2(co.x, co.y);
      Lid[lane] = id;
      float hx, hy;
      pass_box(co, a1.y, hx, hy);
#pragma unroll
      for (int w = 0; w < BW; ++w) {
        const float bx = 0.5f + (float)((w & 1) * 8), by = 0.5f + (float)((w >> 1) * 8);
        if (a0.x + hx >= bx && a0.x - hx <= bx + 7.0f && a0.y + hy >= by && a0.y - hy <= by + 7.0f) mask |= 1u << w;
      }
    }
    uint64_t bal[BW];
#pragma unroll
    for (int w = 0; w < BW; ++w) bal[w] = __ballot((mask >> w) & 1u);
    if (l64 == 0) {
#pragma unroll
      for (int w = 0; w < BW; ++w) wcnt[wv][w] = (uint32_t)__popcll(bal[w]);
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < BW; ++w) {
      if ((mask >> w) & 1u) {
        uint32_t off = (uint32_t)__popcll(bal[w] & lt);
        for (int s = 0; s < wv; ++s) off += wcnt[s][w];
        lst[w][off] = (uint16_t)lane;
      }
    }
    uint32_t len = 0;
#pragma unroll
    for (int s = 0; s < BW; ++s) len += wcnt[s][wv];
    __syncthreads();
    // this wave's records, back to front; a record's nine partial gradients
    // are summed over each row of 16 lanes (lanes that do not pass add zeros)
    // and added to its LDS accumulators by one lane per row with a passing
    // pixel, instead of one float atomic per passing pixel on the same words
    for (int q = (int)len - 1; q >= 0; --q) {
      const int j = lst[wv][q];
      const uint32_t pos = (uint32_t)(lo + 1 + j);
      if (pos > wmax) continue;  // beyond every pixel of the wave
      const float4 r0 = L0[j];
      const float4 r1 = L1[j];
      const float t = t_at(row_part(r0, r1.y, fx), r1.x, fy);
      const bool pass = t >= 0.0f && pos <= lastc;
      const uint64_t pm = __builtin_amdgcn_ballot_w64(pass);
      if (pm == 0ull) continue;  // uniform
      float c[NG];
#pragma unroll
      for (int k = 0; k < NG; ++k) c[k] = 0.0f;
      if (pass) {
        const float4 r2 = L2[j];
        const float2 ab = L3[j];
        const float o = r1.w;
        const float a = alpha_from<KIND>(t, r1, p);
        const float oma = 1.0f - a;
        const float ioma = __builtin_amdgcn_rcpf(oma);
        T = T * ioma;  // transmittance before this splat
        const float w = a * T;
        const float dLda = T * ((r2.x - S0) * g0 + (r2.y - S1) * g1 + (r2.z - S2) * g2) - Tf * ioma * bgg;
        S0 = fmaf(a, r2.x - S0, S0);
        S1 = fmaf(a, r2.y - S1, S1);
        S2 = fmaf(a, r2.z - S2, S2);
        c[6] = w * g0;
        c[7] = w * g1;
        c[8] = w * g2;
        // alpha = o' k(Q) unless clamped; Q from the same t the decisions used
        const float Q = r1.y - t;
        float kq, dk;
        if (KIND == BLEND_EXP) {
          kq = __expf(-0.5f * Q);
          dk = -0.5f * kq;
        } else {
          kq = poly(p, ORDER, Q);
          dk = dpoly(p, ORDER, Q);
        }
        if (!(o * kq > p.alpha_max)) {
          const float dx = fx - r0.x, dy = fy - r0.y;
          const float dLdQ = dLda * o * dk;
          c[5] = dLda * kq;
          c[2] = dLdQ * dx * dx;
          c[3] = dLdQ * 2.0f * dx * dy;
          c[4] = dLdQ * dy * dy;
          // Q depends on the mean through d = pixel - mean
          c[0] = dLdQ * -2.0f * (ab.x * dx + ab.y * dy);
          c[1] = dLdQ * -2.0f * (ab.y * dx + r1.x * dy);
        }
      }
#pragma unroll
      for (int k = 0; k < NG; ++k) c[k] = row_sum(c[k]);
      if ((l64 & 15) == 15 && ((pm >> (l64 & 48)) & 0xFFFFull) != 0ull) {
#pragma unroll
        for (int k = 0; k < NG; ++k) atomicAdd(&G[k][j], c[k]);
      }
    }
    __syncthreads();
    if (lane < cnt) {
      float gv[NG];
      bool any = false;
#pragma unroll
      for (int k = 0; k < NG; ++k) {
        gv[k] = G[k][lane];
        any = any || gv[k] != 0.0f;
      }
      if (any) {
        const uint32_t id = Lid[lane];
        atomicAdd(&dmeans2d[2 * id], gv[0]);
        atomicAdd(&dmeans2d[2 * id + 1], gv[1]);
        atomicAdd(&dconic[4 * id], gv[2]);
        atomicAdd(&dconic[4 * id + 1], gv[3]);
        atomicAdd(&dconic[4 * id + 2], gv[4]);
        atomicAdd(&dconic[4 * id + 3], gv[5]);
        atomicAdd(&drgb[3 * id], gv[6]);
        atomicAdd(&drgb[3 * id + 1], gv[7]);
        atomicAdd(&drgb[3 * id + 2], gv[8]);
      }
    }
    __syncthreads();  // the staging area is reused
  }
}

// ---------------------------------------------------------------------------
// projection adjoint
// ---------------------------------------------------------------------------

// Gradients of the real SH basis (sh_basis, in the same single precision
// and with the same constants) with respect to the unit direction (x, y, z)
template <int DEG>
__device__ inline void sh_basis_dir_grad(float x, float y, float z, float dY[16][3]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) dY[k][0] = dY[k][1] = dY[k][2] = 0.0f;
  if (DEG >= 1) {
    const float k1 = 0.48860251190291992f;
    dY[1][1] = -k1;
    dY[2][2] = k1;
    dY[3][0] = -k1;
  }
  if (DEG >= 2) {
    const float a = 1.0925484305920792f, b = 0.31539156525252005f, c = 0.54627421529603959f;
    dY[4][0] = a * y; dY[4][1] = a * x;
    dY[5][1] = -a * z; dY[5][2] = -a * y;
    dY[6][0] = -2.0f * b * x; dY[6][1] = -2.0f * b * y; dY[6][2] = 4.0f * b * z;
    dY[7][0] = -a * z; dY[7][2] = -a * x;
    dY[8][0] = 2.0f * c * x; dY[8][1] = -2.0f * c * y;
  }
  if (DEG >= 3) {
    const float a = 0.59004358992664352f, b = 2.8906114426405538f, c = 0.45704579946446572f;
    const float d = 0.37317633259011540f, e = 1.4453057213202769f;
    const float xx = x * x, yy = y * y, zz = z * z;
    dY[9][0] = -6.0f * a * x * y; dY[9][1] = -a * (3.0f * xx - 3.0f * yy);
    dY[10][0] = b * y * z; dY[10][1] = b * x * z; dY[10][2] = b * x * y;
    dY[11][0] = 2.0f * c * x * y; dY[11][1] = -c * (4.0f * zz - xx - 3.0f * yy); dY[11][2] = -8.0f * c * y * z;
    dY[12][0] = -6.0f * d * x * z; dY[12][1] = -6.0f * d * y * z; dY[12][2] = d * (6.0f * zz - 3.0f * xx - 3.0f * yy);
    dY[13][0] = -c * (4.0f * zz - 3.0f * xx - yy); dY[13][1] = 2.0f * c * x * y; dY[13][2] = -8.0f * c * x * z;
    dY[14][0] = 2.0f * e * x * z; dY[14][1] = -2.0f * e * y * z; dY[14][2] = e * (xx - yy);
    dY[15][0] = -a * (3.0f * xx - 3.0f * yy); dY[15][1] = 6.0f * a * x * y;
  }
}

// the SH degree is a template parameter so that the basis values and their
// gradients stay in registers (fully unrolled, constant indices)
template <int DEG>
__global__ __launch_bounds__(128) void preprocess_bwd_kernel(
    PreParams p, int64_t n, const float *__restrict__ means3d, const float *__restrict__ scales,
    const float *__restrict__ quats, const float *__restrict__ opac, const float *__restrict__ sh,
    const uint32_t *__restrict__ tiles, const float *__restrict__ dmeans2d, const float *__restrict__ dconic,
    const float *__restrict__ drgb, float *__restrict__ dmeans3d, float *__restrict__ dscales,
    float *__restrict__ dquats, float *__restrict__ dopac, float *__restrict__ dsh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  constexpr int nsh = (DEG + 1) * (DEG + 1);
  double gmu[3] = {0.0, 0.0, 0.0}, gs3[3] = {0.0, 0.0, 0.0}, gq[4] = {0.0, 0.0, 0.0, 0.0}, gop = 0.0;
  const bool live = tiles[i] != 0u;
  if (!live) {
#pragma unroll
    for (int k = 0; k < nsh * 3; ++k) dsh[(size_t)i * nsh * 3 + k] = 0.0f;
  } else {
    const CamD &cam = p.cam;
    const double mx = means3d[3 * i], my = means3d[3 * i + 1], mz = means3d[3 * i + 2];
    double t[3];
    for (int r = 0; r < 3; ++r) t[r] = cam.R[3 * r] * mx + cam.R[3 * r + 1] * my + cam.R[3 * r + 2] * mz + cam.t[r];

    // ---- colour: rgb = max(sum_k Y_k(d) sh_k + 0.5, 0), d = (mu - campos) / |mu - campos|, in
    // single precision exactly as the forward evaluates it (same direction, basis and FMA order), so the
    // clamp's pass-through decision is the forward's
    {
      const double v0 = mx - cam.campos[0], v1 = my - cam.campos[1], v2 = mz - cam.campos[2];
      const double vn2 = v0 * v0 + v1 * v1 + v2 * v2;
      const double dn = 1.0 / sqrt(vn2);
      const float xf = (float)(v0 * dn), yf = (float)(v1 * dn), zf = (float)(v2 * dn);
      float Y[16], dY[16][3];
      sh_basis<DEG>(xf, yf, zf, Y);
      sh_basis_dir_grad<DEG>(xf, yf, zf, dY);
      const float *shi = sh + (size_t)i * nsh * 3;
      float shv[nsh * 3];
#pragma unroll
      for (int k = 0; k < nsh * 3; ++k) shv[k] = shi[k];
      float acc[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
      for (int k = 0; k < nsh; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = fmaf(Y[k], shv[3 * k + c], acc[c]);
      float ga[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) ga[c] = acc[c] > 0.0f ? drgb[3 * i + c] : 0.0f;
      float gd[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < nsh; ++k) {
        float sk = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          dsh[(size_t)i * nsh * 3 + 3 * k + c] = Y[k] * ga[c];
          sk = fmaf(shv[3 * k + c], ga[c], sk);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) gd[a] = fmaf(dY[k][a], sk, gd[a]);
      }
      // d = v / |v|: dL/dv = (gd - d (d . gd)) / |v|
      const double d[3] = {v0 * dn, v1 * dn, v2 * dn};
      const double dd = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
#pragma unroll
      for (int a = 0; a < 3; ++a) gmu[a] += (gd[a] - d[a] * dd) * dn;
    }

    // ---- geometry, recomputed as in the forward
    double qw = quats[4 * i], qx = quats[4 * i + 1], qy = quats[4 * i + 2], qz = quats[4 * i + 3];
    const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    const double w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
    const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    const double s[3] = {scales[3 * i], scales[3 * i + 1], scales[3 * i + 2]};
    double Sig[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Sig[a][b] = R[a][0] * s[0] * s[0] * R[b][0] + R[a][1] * s[1] * s[1] * R[b][1] +
                                              R[a][2] * s[2] * s[2] * R[b][2];
    const double tz = t[2], iz = 1.0 / tz;
    const double rx = t[0] * iz, ry = t[1] * iz;
    const bool inx = rx > -cam.limx && rx < cam.limx, iny = ry > -cam.limy && ry < cam.limy;
    const double txz = fmin(fmax(rx, -cam.limx), cam.limx), tyz = fmin(fmax(ry, -cam.limy), cam.limy);
    const double J[2][3] = {{cam.fx * iz, 0.0, -cam.fx * txz * iz}, {0.0, cam.fy * iz, -cam.fy * tyz * iz}};
    double T2[2][3];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 3; ++b) T2[a][b] = J[a][0] * cam.R[b] + J[a][1] * cam.R[3 + b] + J[a][2] * cam.R[6 + b];
    double TS_[2][3];  // T2 Sigma
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 3; ++b) TS_[a][b] = T2[a][0] * Sig[0][b] + T2[a][1] * Sig[1][b] + T2[a][2] * Sig[2][b];
    const double Sxx = TS_[0][0] * T2[0][0] + TS_[0][1] * T2[0][1] + TS_[0][2] * T2[0][2];
    const double Sxy = TS_[0][0] * T2[1][0] + TS_[0][1] * T2[1][1] + TS_[0][2] * T2[1][2];
    const double Syy = TS_[1][0] * T2[1][0] + TS_[1][1] * T2[1][1] + TS_[1][2] * T2[1][2];
    // |S'| as the forward evaluates it (a sum of squares, accurate for thin
    // footprints); its derivatives below are the cofactors of S'
    const double det0 = proj_cov_det(T2, R, s[0], s[1], s[2]);
    const double Axx = Sxx + p.aa_v, Ayy = Syy + p.aa_v;
    const double deta = Axx * Ayy - Sxy * Sxy;
    const double ratio = det0 / deta;
    const double sr = ratio > 0.0 ? sqrt(ratio) : 0.0;

    // ---- opacity: o' = o sqrt(det0 / deta)
    const double go2 = dconic[4 * i + 3];
    gop = go2 * sr;
    double gSxx = 0.0, gSxy = 0.0, gSyy = 0.0;
    if (ratio > 0.0) {
      const double gr = go2 * (double)opac[i] * 0.5 / sr;  // dL/dratio
      const double gdet0 = gr / deta, gdeta = -gr * det0 / (deta * deta);
      gSxx += gdet0 * Syy + gdeta * Ayy;
      gSyy += gdet0 * Sxx + gdeta * Axx;
      gSxy += -2.0 * Sxy * (gdet0 + gdeta);
    }
    // ---- conic = S_a^-1: dL/dS_a = -conic G conic, G the symmetric gradient matrix
    {
      const double ca = Ayy / deta, cb = -Sxy / deta, cc = Axx / deta;
      const double Ga = dconic[4 * i], Gb = 0.5 * (double)dconic[4 * i + 1], Gc = dconic[4 * i + 2];
      // M = conic * G
      const double M00 = ca * Ga + cb * Gb, M01 = ca * Gb + cb * Gc, M10 = cb * Ga + cc * Gb, M11 = cb * Gb + cc * Gc;
      // N = M * conic
      const double N00 = M00 * ca + M01 * cb, N01 = M00 * cb + M01 * cc, N11 = M10 * cb + M11 * cc;
      gSxx -= N00;
      gSyy -= N11;
      gSxy -= 2.0 * N01;
    }
    // ---- EWA: S' = T2 Sigma T2^T with G' = [[gSxx, gSxy/2], [gSxy/2, gSyy]]
    const double G2[2][2] = {{gSxx, 0.5 * gSxy}, {0.5 * gSxy, gSyy}};
    double gSig[3][3];  // T2^T G' T2
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
        for (int u = 0; u < 2; ++u)
          for (int v = 0; v < 2; ++v) acc += T2[u][a] * G2[u][v] * T2[v][b];
        gSig[a][b] = acc;
      }
    double gT2[2][3];  // 2 G' T2 Sigma
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 3; ++b) gT2[a][b] = 2.0 * (G2[a][0] * TS_[0][b] + G2[a][1] * TS_[1][b]);
    double gJ[2][3];  // dL/dT2 W^T
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 3; ++b) gJ[a][b] = gT2[a][0] * cam.R[3 * b] + gT2[a][1] * cam.R[3 * b + 1] +
                                            gT2[a][2] * cam.R[3 * b + 2];
    // J entries: J00 = fx iz, J02 = -fx txz iz, J11 = fy iz, J12 = -fy tyz iz
    double giz = gJ[0][0] * cam.fx + gJ[1][1] * cam.fy - gJ[0][2] * cam.fx * txz - gJ[1][2] * cam.fy * tyz;
    double gtxz = -gJ[0][2] * cam.fx * iz, gtyz = -gJ[1][2] * cam.fy * iz;
    double gt[3] = {0.0, 0.0, 0.0};
    // means2d: u = fx t.x iz + cx, v = fy t.y iz + cy
    const double gu = dmeans2d[2 * i], gv = dmeans2d[2 * i + 1];
    gt[0] += gu * cam.fx * iz;
    gt[1] += gv * cam.fy * iz;
    giz += gu * cam.fx * t[0] + gv * cam.fy * t[1];
    // txz = clamp(t.x iz), tyz = clamp(t.y iz)
    if (inx) {
      gt[0] += gtxz * iz;
      giz += gtxz * t[0];
    }
    if (iny) {
      gt[1] += gtyz * iz;
      giz += gtyz * t[1];
    }
    gt[2] += -giz * iz * iz;
    // t = W mu + tw
    for (int a = 0; a < 3; ++a) gmu[a] += cam.R[a] * gt[0] + cam.R[3 + a] * gt[1] + cam.R[6 + a] * gt[2];

    // ---- Sigma = M M^T with M = R diag(s): dL/dM = 2 gSig M
    double gR[3][3];
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 3; ++k) {
        double gM = 0.0;
        for (int b = 0; b < 3; ++b) gM += 2.0 * gSig[a][b] * R[b][k] * s[k];
        gR[a][k] = gM * s[k];
        gs3[k] += gM * R[a][k];
      }
    // ---- R(q) with q normalised
    const double gw = 2.0 * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
    const double gx = 2.0 * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2 * x * gR[1][1] - w * gR[1][2] +
                             z * gR[2][0] + w * gR[2][1] - 2 * x * gR[2][2]);
    const double gy = 2.0 * (-2 * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] -
                             w * gR[2][0] + z * gR[2][1] - 2 * y * gR[2][2]);
    const double gz = 2.0 * (-2 * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] - 2 * z * gR[1][1] +
                             y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
    const double dotq = w * gw + x * gx + y * gy + z * gz;
    gq[0] = (gw - w * dotq) / qn;
    gq[1] = (gx - x * dotq) / qn;
    gq[2] = (gy - y * dotq) / qn;
    gq[3] = (gz - z * dotq) / qn;
  }
  for (int a = 0; a < 3; ++a) {
    dmeans3d[3 * i + a] = (float)gmu[a];
    dscales[3 * i + a] = (float)gs3[a];
  }
  for (int a = 0; a < 4; ++a) dquats[4 * i + a] = (float)gq[a];
  dopac[i] = (float)gop;
}

}  // namespace

hipError_t launch_blend_bwd(const BlendParams &p, int64_t n, const float *means2d, const float *conic_opacity,
                            const float *rgb, const uint32_t *vals, const uint32_t *ranges,
                            const uint32_t *tile_order, const float *final_T,
                            const uint32_t *last_contrib, const float *dL_dimage, float *dmeans2d,
                            float *dconic_opacity, float *drgb, hipStream_t s) {
  if (n > 0) {
    hipLaunchKernelGGL(zero_f32, dim3(ceil_div(2 * n, 256)), dim3(256), 0, s, dmeans2d, 2 * n);
    hipLaunchKernelGGL(zero_f32, dim3(ceil_div(4 * n, 256)), dim3(256), 0, s, dconic_opacity, 4 * n);
    hipLaunchKernelGGL(zero_f32, dim3(ceil_div(3 * n, 256)), dim3(256), 0, s, drgb, 3 * n);
  }
  const dim3 grid(p.gx * p.gy), block(BT);
  switch (p.blend) {
    case BLEND_EXP:
      hipLaunchKernelGGL(blend_bwd<BLEND_EXP>, grid, block, 0, s, p, means2d, conic_opacity, rgb, vals, ranges,
                         tile_order, final_T, last_contrib, dL_dimage, dmeans2d, dconic_opacity, drgb);
      break;
    case BLEND_POLY1:
      hipLaunchKernelGGL(blend_bwd<BLEND_POLY1>, grid, block, 0, s, p, means2d, conic_opacity, rgb, vals, ranges,
                         tile_order, final_T, last_contrib, dL_dimage, dmeans2d, dconic_opacity, drgb);
      break;
    case BLEND_POLY2:
      hipLaunchKernelGGL(blend_bwd<BLEND_POLY2>, grid, block, 0, s, p, means2d, conic_opacity, rgb, vals, ranges,
                         tile_order, final_T, last_contrib, dL_dimage, dmeans2d, dconic_opacity, drgb);
      break;
    default:
      hipLaunchKernelGGL(blend_bwd<BLEND_POLY3>, grid, block, 0, s, p, means2d, conic_opacity, rgb, vals, ranges,
                         tile_order, final_T, last_contrib, dL_dimage, dmeans2d, dconic_opacity, drgb);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const PreParams &p, int64_t n, const float *means3d, const float *scales,
                                 const float *quats, const float *opac, const float *sh, const uint32_t *tiles,
                                 const float *dmeans2d, const float *dconic_opacity, const float *drgb,
                                 float *dmeans3d, float *dscales, float *dquats, float *dopac, float *dsh,
                                 hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 grid(ceil_div(n, 128)), block(128);
#define GS_PRE_BWD(D)                                                                                           \
  hipLaunchKernelGGL(preprocess_bwd_kernel<D>, grid, block, 0, s, p, n, means3d, scales, quats, opac, sh, tiles, \
                     dmeans2d, dconic_opacity, drgb, dmeans3d, dscales, dquats, dopac, dsh)
  switch (p.sh_degree) {
    case 0: GS_PRE_BWD(0); break;
    case 1: GS_PRE_BWD(1); break;
    case 2: GS_PRE_BWD(2); break;
    default: GS_PRE_BWD(3); break;
  }
#undef GS_PRE_BWD
  return hipGetLastError();
}

}  // namespace gs
