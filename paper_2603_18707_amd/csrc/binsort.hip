// Tile binning: duplication of splats per covered tile, a stable LSD radix
// sort of the 64-bit keys (tile_id << 32) | bits(depth), and per-tile ranges.
//
// The sort is organised around the key's structure. An LSD radix sort
// processes the low digits first, and the 32 low bits (the depth) are the
// same for every copy of a splat. So the depth passes run once per splat
// (N items) instead of once per copy (K items, K ~ 3N at 1080p): splats are
// sorted by depth stably in index order, copies are emitted in that order
// (row-major tiles within each splat), and the remaining tile digits are
// sorted stably over the copies. The result is exactly the stable sort of
// the copies emitted in splat-index order, because within one tile each
// splat has at most one copy.
//
// Every kernel sized by the key count reads it from device memory, and grids
// are sized by the key capacity, so the whole stage runs without a host
// round trip (and can be captured in a graph).
#include "gs_internal.h"

namespace gs {

namespace {

constexpr int BS = 256;           // threads per block
constexpr int IPT = 16;           // items per thread (scans)
constexpr int TILE = BS * IPT;    // items per block (scans)
constexpr int RIPT = 4;           // items per thread (radix passes): more, smaller blocks fill the CUs
constexpr int RTILE = BS * RIPT;  // items per block (radix passes)
constexpr int RADIX = 256;        // max buckets per pass (8-bit digits)
constexpr uint32_t BIG = 64;      // splats with more copies are expanded block-wide

// ---------------------------------------------------------------------------
// scans
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T wave_inclusive(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  return v;
}

// exclusive scan over the 256 threads of a block; also returns the block total
template <typename T>
__device__ inline T block_exclusive(T v, T &total) {
  __shared__ T wsum[BS / 64];
  const T inc = wave_inclusive(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) wsum[w] = inc;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < BS / 64; ++k) {
    const T s = wsum[k];
    if (k < w) off += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return off + inc - v;
}

template <typename TIn, typename TOut>
__global__ __launch_bounds__(BS) void scan_reduce(const TIn *__restrict__ in, int64_t m, TOut *partials) {
  const int64_t base = (int64_t)blockIdx.x * TILE + (int64_t)threadIdx.x * IPT;
  TOut s = 0;
#pragma unroll
  for (int j = 0; j < IPT; ++j)
    if (base + j < m) s += (TOut)in[base + j];
  TOut tot;
  block_exclusive(s, tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// single block: exclusive scan of nb partials in place; *total = their sum
template <typename T>
__global__ __launch_bounds__(BS) void scan_partials(T *partials, int64_t nb, T *total) {
  T carry = 0;
  for (int64_t base = 0; base < nb; base += (int64_t)BS * IPT) {
    const int64_t b0 = base + (int64_t)threadIdx.x * IPT;
    T loc[IPT];
    T s = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      loc[j] = (b0 + j < nb) ? partials[b0 + j] : (T)0;
      s += loc[j];
    }
    T tot;
    T off = block_exclusive(s, tot) + carry;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      if (b0 + j < nb) partials[b0 + j] = off;
      off += loc[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

template <typename TIn, typename TOut>
__global__ __launch_bounds__(BS) void scan_down(const TIn *__restrict__ in, int64_t m,
                                                const TOut *__restrict__ partials, TOut *__restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * TILE + (int64_t)threadIdx.x * IPT;
  TOut loc[IPT];
  TOut s = 0;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    loc[j] = (base + j < m) ? (TOut)in[base + j] : (TOut)0;
    s += loc[j];
  }
  TOut tot;
  TOut off = block_exclusive(s, tot) + partials[blockIdx.x];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    if (base + j < m) out[base + j] = off;
    off += loc[j];
  }
}

// exclusive scan of m items; out[m] receives the total when write_total
template <typename TIn, typename TOut>
hipError_t exclusive_scan(const TIn *in, int64_t m, TOut *out, TOut *partials, bool write_total, hipStream_t s) {
  if (m == 0) return hipSuccess;  // callers only scan non-empty arrays
  const unsigned nb = ceil_div(m, TILE);
  hipLaunchKernelGGL((scan_reduce<TIn, TOut>), dim3(nb), dim3(BS), 0, s, in, m, partials);
  hipLaunchKernelGGL((scan_partials<TOut>), dim3(1), dim3(BS), 0, s, partials, (int64_t)nb,
                     write_total ? out + m : (TOut *)nullptr);
  hipLaunchKernelGGL((scan_down<TIn, TOut>), dim3(nb), dim3(BS), 0, s, in, m, partials, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// radix sort passes over (uint32 key, uint32 value)
// ---------------------------------------------------------------------------
__device__ inline uint32_t item_count(uint32_t kh, const uint32_t *kd) { return kd ? *kd : kh; }

__global__ __launch_bounds__(BS) void radix_upsweep(const uint32_t *__restrict__ keys, uint32_t kh,
                                                    const uint32_t *kd, int shift, int nbits,
                                                    uint32_t *__restrict__ hist, uint32_t nb) {
  __shared__ uint32_t h[BS / 64][RADIX];
  const uint32_t K = item_count(kh, kd);
  const uint32_t R = 1u << nbits, mask = R - 1u;
  for (int d = threadIdx.x; d < (BS / 64) * RADIX; d += BS) (&h[0][0])[d] = 0u;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * RTILE;
  const int w = threadIdx.x >> 6;
  if (base < K) {
#pragma unroll
    for (int it = 0; it < RIPT; ++it) {
      const uint64_t idx = base + (uint64_t)it * BS + threadIdx.x;
      if (idx < K) atomicAdd(&h[w][(keys[idx] >> shift) & mask], 1u);
    }
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < R; d += BS)
    hist[(size_t)d * nb + blockIdx.x] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

// Stable scatter: within a block, items are ranked in index order (rounds of
// 256 consecutive items; inside a round, wave by wave and lane by lane). The
// per-wave rank among equal digits comes from matching the digit bit by bit
// with ballots. FINAL writes the 64-bit output key (key << 32 | depth bits of
// the value's splat) instead of the 32-bit key.
template <bool FINAL>
__global__ __launch_bounds__(BS) void radix_downsweep(const uint32_t *__restrict__ kin,
                                                      const uint32_t *__restrict__ vin, uint32_t kh,
                                                      const uint32_t *kd, int shift, int nbits,
                                                      const uint32_t *__restrict__ hist, uint32_t nb,
                                                      uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                      uint64_t *__restrict__ k64out,
                                                      const uint32_t *__restrict__ depth_bits) {
  __shared__ uint32_t run[RADIX];
  __shared__ uint32_t wcnt[BS / 64][RADIX];
  __shared__ uint32_t woff[BS / 64][RADIX];
  const uint32_t K = item_count(kh, kd);
  const uint64_t base = (uint64_t)blockIdx.x * RTILE;
  if (base >= K) return;
  const uint32_t R = 1u << nbits, mask = R - 1u;
  for (uint32_t d = threadIdx.x; d < R; d += BS) {
    run[d] = hist[(size_t)d * nb + blockIdx.x];
#pragma unroll
    for (int w = 0; w < BS / 64; ++w) wcnt[w][d] = 0u;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int it = 0; it < RIPT; ++it) {
    const uint64_t idx = base + (uint64_t)it * BS + threadIdx.x;
    const bool valid = idx < K;
    const uint32_t key = valid ? kin[idx] : 0u;
    const uint32_t val = valid ? vin[idx] : 0u;
    const uint32_t d = (key >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && (peers & lt) == 0ull) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    for (uint32_t dd = threadIdx.x; dd < R; dd += BS) {
      uint32_t r = run[dd];
#pragma unroll
      for (int ww = 0; ww < BS / 64; ++ww) {
        const uint32_t c = wcnt[ww][dd];
        woff[ww][dd] = r;
        r += c;
        wcnt[ww][dd] = 0u;
      }
      run[dd] = r;
    }
    __syncthreads();
    const uint32_t pos = woff[w][d] + rank;
    if (valid && pos < K) {  // pos < K always holds for a correct ranking
      if (FINAL) {
        k64out[pos] = ((uint64_t)key << 32) | (uint64_t)depth_bits[val];
      } else {
        kout[pos] = key;
      }
      vout[pos] = val;
    }
  }
}

// ---------------------------------------------------------------------------
// stage kernels
// ---------------------------------------------------------------------------
__global__ void fill_u32(uint32_t *p, int64_t m, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) p[i] = v;
}

__global__ void depth_keys(int64_t n, const float *__restrict__ depth, const uint32_t *__restrict__ tiles,
                           uint32_t *__restrict__ key, uint32_t *__restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // visible splats have depth >= near_z > 0, where float bits order like the values
  key[i] = tiles[i] ? __float_as_uint(depth[i]) : 0xFFFFFFFFu;
  idx[i] = (uint32_t)i;
}

__global__ void gather_counts(int64_t n, const uint32_t *__restrict__ order, const uint32_t *__restrict__ tiles,
                              uint32_t *__restrict__ cnt) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint32_t i = order[s];
  cnt[s] = (int64_t)i < n ? tiles[i] : 0u;
}

// ctr[0] = effective key count (0 on overflow), ctr[1] = big-splat count
__global__ void finalize_count(int64_t n, const uint64_t *off, int64_t capacity, int64_t *num_keys,
                               int32_t *overflow, uint32_t *ctr) {
  const uint64_t K = n > 0 ? off[n] : 0ull;
  const bool over = K > (uint64_t)capacity;
  *num_keys = (int64_t)K;
  *overflow = over ? 1 : 0;
  ctr[0] = over ? 0u : (uint32_t)K;
  ctr[1] = 0u;
}

__global__ __launch_bounds__(BS) void duplicate(int64_t n, const uint32_t *__restrict__ order,
                                                const uint64_t *__restrict__ off, const int32_t *__restrict__ rect,
                                                int grid_w, uint64_t capacity, const int32_t *__restrict__ overflow,
                                                uint32_t *__restrict__ tkey, uint32_t *__restrict__ tval,
                                                uint32_t *__restrict__ big, uint32_t *__restrict__ ctr) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n || *overflow) return;
  const uint64_t o = off[s];
  const uint32_t cnt = (uint32_t)(off[s + 1] - o);
  if (cnt == 0 || o + cnt > capacity) return;
  if (cnt > BIG) {
    big[atomicAdd(&ctr[1], 1u)] = (uint32_t)s;
    return;
  }
  const uint32_t i = order[s];
  if ((int64_t)i >= n) return;
  const int4 r = reinterpret_cast<const int4 *>(rect)[i];
  uint64_t p = o;
  for (int ty = r.y; ty <= r.w; ++ty)
    for (int tx = r.x; tx <= r.z; ++tx) {
      tkey[p] = (uint32_t)(ty * grid_w + tx);
      tval[p] = i;
      ++p;
    }
}

__global__ __launch_bounds__(BS) void duplicate_big(int64_t n, const uint32_t *__restrict__ order,
                                                    const uint64_t *__restrict__ off,
                                                    const int32_t *__restrict__ rect, int grid_w, uint64_t capacity,
                                                    const uint32_t *__restrict__ big, const uint32_t *__restrict__ ctr,
                                                    uint32_t *__restrict__ tkey, uint32_t *__restrict__ tval) {
  const uint32_t nbig = ctr[1];
  for (uint32_t e = blockIdx.x; e < nbig; e += gridDim.x) {
    const uint32_t s = big[e];
    if ((int64_t)s >= n) continue;
    const uint32_t i = order[s];
    const uint64_t o = off[s];
    const uint32_t cnt = (uint32_t)(off[s + 1] - o);
    if ((int64_t)i >= n || o + cnt > capacity) continue;
    const int4 r = reinterpret_cast<const int4 *>(rect)[i];
    const uint32_t w = (uint32_t)(r.z - r.x + 1);
    for (uint32_t j = threadIdx.x; j < cnt; j += BS) {
      const uint32_t ty = r.y + j / w, tx = r.x + j % w;
      tkey[o + j] = ty * (uint32_t)grid_w + tx;
      tval[o + j] = i;
    }
  }
}

__global__ void tile_ranges(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ ctr, int64_t ntiles,
                            uint32_t *__restrict__ ranges) {
  const uint32_t K = ctr[0];
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const uint32_t t = (uint32_t)(keys[k] >> 32);
  if ((int64_t)t >= ntiles) return;
  if (k == 0 || (uint32_t)(keys[k - 1] >> 32) != t) ranges[2 * (size_t)t] = (uint32_t)k;
  if (k + 1 == K || (uint32_t)(keys[k + 1] >> 32) != t) ranges[2 * (size_t)t + 1] = (uint32_t)(k + 1);
}

// Longest-list-first dispatch order of the tiles: tiles bucketed by their list
// length (256 linear buckets up to the longest list), heaviest bucket first.
// A workgroup's time grows with its tile's list, so starting the long lists
// first keeps them off the tail of the blend launch. One workgroup.
__global__ __launch_bounds__(1024) void tile_order_kernel(const uint32_t *__restrict__ ranges, int64_t ntiles,
                                                          uint32_t *__restrict__ order) {
  constexpr int NB = 256;
  __shared__ uint32_t hist[NB];
  __shared__ uint32_t s_max;
  if (threadIdx.x == 0) s_max = 0u;
  for (int b = threadIdx.x; b < NB; b += blockDim.x) hist[b] = 0u;
  __syncthreads();
  uint32_t mx = 0;
  for (int64_t t = threadIdx.x; t < ntiles; t += blockDim.x) mx = max(mx, ranges[2 * t + 1] - ranges[2 * t]);
  atomicMax(&s_max, mx);
  __syncthreads();
  const uint64_t span = (uint64_t)s_max + 1ull;
  for (int64_t t = threadIdx.x; t < ntiles; t += blockDim.x) {
    const uint64_t len = ranges[2 * t + 1] - ranges[2 * t];
    atomicAdd(&hist[NB - 1 - (int)(len * NB / span)], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int b = 0; b < NB; ++b) {
      const uint32_t c = hist[b];
      hist[b] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int64_t t = threadIdx.x; t < ntiles; t += blockDim.x) {
    const uint64_t len = ranges[2 * t + 1] - ranges[2 * t];
    const uint32_t pos = atomicAdd(&hist[NB - 1 - (int)(len * NB / span)], 1u);
    if ((int64_t)pos < ntiles) order[pos] = (uint32_t)t;
  }
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
struct Workspace {
  uint32_t *dk0, *di0, *dk1, *di1;   // depth sort ping-pong [n]
  uint32_t *cnt;                     // copies per splat in depth order [n]
  uint64_t *off;                     // their exclusive scan [n + 1]
  uint32_t *hist;                    // digit histograms [RADIX * max blocks]
  uint64_t *part64;                  // scan partials
  uint32_t *part32;
  uint32_t *tk0, *tv0, *tk1, *tv1;   // tile sort ping-pong [capacity]
  uint32_t *big;                     // splats expanded block-wide [n]
  uint32_t *ctr;                     // counters
};

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

size_t carve(void *base, int64_t n, int64_t cap, Workspace *w) {
  const size_t N = (size_t)(n > 0 ? n : 1), C = (size_t)(cap > 0 ? cap : 1);
  const size_t nbn = ceil_div((int64_t)N, RTILE), nbk = ceil_div((int64_t)C, RTILE);
  const size_t nbmax = nbn > nbk ? nbn : nbk;
  const size_t hist_items = (size_t)RADIX * nbmax;
  const size_t parts = ceil_div((int64_t)(hist_items > N + 1 ? hist_items : N + 1), TILE) + 1;
  char *p = (char *)base;
  size_t o = 0;
  auto take = [&](size_t bytes) -> void * {
    void *r = p ? (void *)(p + o) : nullptr;
    o += align_up(bytes);
    return r;
  };
  Workspace t;
  t.dk0 = (uint32_t *)take(4 * N);
  t.di0 = (uint32_t *)take(4 * N);
  t.dk1 = (uint32_t *)take(4 * N);
  t.di1 = (uint32_t *)take(4 * N);
  t.cnt = (uint32_t *)take(4 * N);
  t.off = (uint64_t *)take(8 * (N + 1));
  t.hist = (uint32_t *)take(4 * hist_items);
  t.part64 = (uint64_t *)take(8 * parts);
  t.part32 = (uint32_t *)take(4 * parts);
  t.tk0 = (uint32_t *)take(4 * C);
  t.tv0 = (uint32_t *)take(4 * C);
  t.tk1 = (uint32_t *)take(4 * C);
  t.tv1 = (uint32_t *)take(4 * C);
  t.big = (uint32_t *)take(4 * N);
  t.ctr = (uint32_t *)take(4 * 16);
  if (w) *w = t;
  return o;
}

hipError_t radix_pass(const uint32_t *kin, const uint32_t *vin, uint32_t kh, const uint32_t *kd, uint32_t nb,
                      int shift, int nbits, uint32_t *hist, uint32_t *part32, uint32_t *kout, uint32_t *vout,
                      uint64_t *k64out, const uint32_t *depth_bits, bool final, hipStream_t s) {
  hipLaunchKernelGGL(radix_upsweep, dim3(nb), dim3(BS), 0, s, kin, kh, kd, shift, nbits, hist, nb);
  hipError_t e = exclusive_scan<uint32_t, uint32_t>(hist, (int64_t)(1u << nbits) * nb, hist, part32, false, s);
  if (e != hipSuccess) return e;
  if (final)
    hipLaunchKernelGGL(radix_downsweep<true>, dim3(nb), dim3(BS), 0, s, kin, vin, kh, kd, shift, nbits, hist, nb,
                       kout, vout, k64out, depth_bits);
  else
    hipLaunchKernelGGL(radix_downsweep<false>, dim3(nb), dim3(BS), 0, s, kin, vin, kh, kd, shift, nbits, hist,
                       nb, kout, vout, k64out, depth_bits);
  return hipGetLastError();
}

}  // namespace

size_t binsort_workspace_bytes(int64_t n, int64_t capacity, int32_t) { return carve(nullptr, n, capacity, nullptr); }

hipError_t launch_binsort(int64_t n, const float *depth, const int32_t *rect, const uint32_t *tiles, int grid_w,
                          int grid_h, int64_t capacity, void *ws, size_t, uint64_t *keys, uint32_t *vals,
                          uint32_t *ranges, uint32_t *tile_order, int64_t *num_keys, int32_t *overflow,
                          hipStream_t s) {
  Workspace w;
  carve(ws, n, capacity, &w);
  const int64_t ntiles = (int64_t)grid_w * grid_h;
  hipLaunchKernelGGL(fill_u32, dim3(ceil_div(2 * ntiles, 256)), dim3(256), 0, s, ranges, 2 * ntiles, 0u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;

  const uint32_t nbn = n > 0 ? ceil_div(n, RTILE) : 0;
  if (n > 0) {
    // 1. splats by depth (stable, index order on ties): four 8-bit passes
    hipLaunchKernelGGL(depth_keys, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, depth, tiles, w.dk0, w.di0);
    uint32_t *ka = w.dk0, *va = w.di0, *kb = w.dk1, *vb = w.di1;
    for (int pass = 0; pass < 4; ++pass) {
      e = radix_pass(ka, va, (uint32_t)n, nullptr, nbn, 8 * pass, 8, w.hist, w.part32, kb, vb, nullptr, nullptr,
                     false, s);
      if (e != hipSuccess) return e;
      uint32_t *tk = ka, *tv = va;
      ka = kb; va = vb; kb = tk; vb = tv;
    }
    // 2. copies per splat in depth order and their offsets
    hipLaunchKernelGGL(gather_counts, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, va, tiles, w.cnt);
    e = exclusive_scan<uint32_t, uint64_t>(w.cnt, n, w.off, w.part64, true, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_count, dim3(1), dim3(1), 0, s, n, w.off, capacity, num_keys, overflow, w.ctr);
    // 3. emit (tile, splat) copies in depth order
    hipLaunchKernelGGL(duplicate, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, va, w.off, rect, grid_w,
                       (uint64_t)capacity, overflow, w.tk0, w.tv0, w.big, w.ctr);
    hipLaunchKernelGGL(duplicate_big, dim3(1024), dim3(BS), 0, s, n, va, w.off, rect, grid_w, (uint64_t)capacity,
                       w.big, w.ctr, w.tk0, w.tv0);
  } else {
    hipLaunchKernelGGL(finalize_count, dim3(1), dim3(1), 0, s, (int64_t)0, w.off, capacity, num_keys, overflow,
                       w.ctr);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (capacity == 0) {
    if (tile_order)
      hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(1024), 0, s, ranges, ntiles, tile_order);
    return hipGetLastError();
  }

  // 4. stable LSD passes over the tile digits; the last writes the 64-bit keys
  int tile_bits = 1;
  while ((1ll << tile_bits) < ntiles) ++tile_bits;
  const int passes = (tile_bits + 7) / 8;
  const int bits = (tile_bits + passes - 1) / passes;
  const uint32_t nbk = ceil_div(capacity, RTILE);
  const uint32_t *depth_bits = reinterpret_cast<const uint32_t *>(depth);
  uint32_t *ka = w.tk0, *va = w.tv0, *kb = w.tk1, *vb = w.tv1;
  for (int pass = 0; pass < passes; ++pass) {
    const bool last = pass == passes - 1;
    e = radix_pass(ka, va, 0u, w.ctr, nbk, bits * pass, bits, w.hist, w.part32, last ? nullptr : kb,
                   last ? vals : vb, last ? keys : nullptr, depth_bits, last, s);
    if (e != hipSuccess) return e;
    uint32_t *tk = ka, *tv = va;
    ka = kb; va = vb; kb = tk; vb = tv;
  }
  // 5. per-tile ranges
  hipLaunchKernelGGL(tile_ranges, dim3(ceil_div(capacity, 256)), dim3(256), 0, s, keys, w.ctr, ntiles, ranges);
  // 6. longest-first dispatch order for the blend
  if (tile_order) hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(1024), 0, s, ranges, ntiles, tile_order);
  return hipGetLastError();
}

}  // namespace gs
