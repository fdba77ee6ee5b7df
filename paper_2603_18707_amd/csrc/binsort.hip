// Tile binning: duplication of splats per covered tile, a stable LSD radix
// sort of the 64-bit keys (tile_id << 32) | bits(depth), and per-tile ranges.
//
// The sort is organised around the key's structure. An LSD radix sort
// processes the low digits first, and the 32 low bits (the depth) are the
// same for every copy of a splat. So the depth passes run once per splat
// (N items) instead of once per copy (K items, K ~ 2-3 N at 1080p): splats
// are sorted by depth stably in index order, copies are emitted in that
// order (row-major tiles within each splat), and the remaining tile digits
// are sorted stably over the copies. The result is exactly the stable sort
// of the copies emitted in splat-index order, because within one tile each
// splat has at most one copy.
//
// A radix pass is three kernels and no workgroup ever waits on another (a
// hand-off between workgroups costs ~0.5 us through memory, and device
// atomics on scattered addresses cost more than the pass itself):
//  * count_pass: the key array is cut into partitions of SPART items;
//    C[d][p] = items of digit d in partition p (LDS histogram, plain stores).
//  * scan_rows: one workgroup per digit turns its row into output offsets:
//    the items of smaller digits (from digit totals known in advance) plus
//    the row's exclusive prefix.
//  * scatter_pass: each partition ranks its items stably (per-wave ballot
//    matching of the digit, waves in index order) and writes them at
//    C[d][p] + rank.
// Digit totals do not depend on the order, so one read of the depths gives
// them for all four depth passes (with the first pass's counts), and the
// emission kernel gives them for the tile passes; they are accumulated in 8
// striped copies (by workgroup) so no address sees more than an eighth of the
// workgroups. The tile passes carry each copy's depth bits with it, so the
// last one writes the 64-bit keys without gathering the depths.
//
// Every kernel sized by the key count reads it from device memory and grids
// are sized by the key capacity, so the stage runs without a host round trip
// (and can be captured in a graph).
#include "gs_internal.h"

namespace gs {

namespace {

constexpr int BS = 256;                 // threads per workgroup
constexpr int SIPT = 4;                 // items per thread in a sort partition
constexpr int SPART = BS * SIPT;        // items per sort partition
constexpr int EIPT = 4;                 // splats per thread in an emission partition
constexpr int EPART = BS * EIPT;        // splats per emission partition
static_assert(EPART == 1024, "the emission's binary search takes 10 steps");
constexpr int RADIX = 256;              // max buckets per pass (8-bit digits)
constexpr int DEPTH_PASSES = 4;
constexpr int MAX_TILE_PASSES = 4;      // tile ids < 2^30 need at most four digits of <= 8 bits
constexpr int STRIPES = 8;              // copies of the digit totals

enum : int { CTR_KEYS = 0, CTR_SLOTS = 16 };

// totals[stripe][pass][digit]
__device__ inline uint32_t *total_at(uint32_t *tot, int stripe, int pass, int d) {
  return tot + ((size_t)stripe * MAX_TILE_PASSES + pass) * RADIX + d;
}

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

// exclusive scan over the 256 threads of a workgroup; also returns the total
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

// visible splats have depth >= near_z > 0, where float bits order like the
// values; splats without tiles sort last (they emit nothing)
__device__ inline uint32_t depth_key(const float *depth, const uint32_t *tiles, uint32_t i) {
  return tiles[i] ? __float_as_uint(depth[i]) : 0xFFFFFFFFu;
}

// Workgroup b of a G-workgroup launch runs on XCD b % 8 (round-robin
// dispatch). Handing each XCD a contiguous run of partitions keeps the
// neighbouring partitions, whose outputs share cache lines at every digit
// boundary, in one L2 instead of writing the same lines from several. A
// bijection on [0, G).
__device__ inline uint32_t xcd_partition(uint32_t b, uint32_t G) {
  const uint32_t q = G / 8, r = G % 8, x = b % 8;
  return x * q + (x < r ? x : r) + b / 8;
}

__device__ inline uint32_t item_count(const uint32_t *count_dev, uint32_t count) {
  return count_dev ? *count_dev : count;
}

// ---------------------------------------------------------------------------
// state reset: totals, counters, ranges, outputs
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BS) void clear_state(uint4 *__restrict__ z, size_t nz16, uint32_t *__restrict__ ranges,
                                                  size_t nr, int64_t *num_keys, int32_t *overflow) {
  const size_t i = (size_t)blockIdx.x * BS + threadIdx.x, stride = (size_t)gridDim.x * BS;
  for (size_t j = i; j < nz16; j += stride) z[j] = make_uint4(0u, 0u, 0u, 0u);
  for (size_t j = i; j < nr; j += stride) ranges[j] = 0u;
  if (i == 0) {
    *num_keys = 0;
    *overflow = 0;
  }
}

// ---------------------------------------------------------------------------
// depth keys: counts of the first pass per partition, totals of all passes
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BS) void depth_count(uint32_t n, const float *__restrict__ depth,
                                                  const uint32_t *__restrict__ tiles, uint32_t *__restrict__ c0,
                                                  size_t c_stride, uint32_t *__restrict__ tot) {
  __shared__ uint32_t h[BS / 64][DEPTH_PASSES * RADIX];
  for (int j = threadIdx.x; j < (BS / 64) * DEPTH_PASSES * RADIX; j += BS) (&h[0][0])[j] = 0u;
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const uint64_t base = (uint64_t)blockIdx.x * SPART + threadIdx.x;
#pragma unroll
  for (int r = 0; r < SIPT; ++r) {
    const uint64_t i = base + (uint64_t)r * BS;
    if (i < n) {
      const uint32_t k = depth_key(depth, tiles, (uint32_t)i);
#pragma unroll
      for (int p = 0; p < DEPTH_PASSES; ++p) atomicAdd(&h[w][p * RADIX + ((k >> (8 * p)) & 255u)], 1u);
    }
  }
  __syncthreads();
  const int stripe = blockIdx.x % STRIPES;
  for (int j = threadIdx.x; j < DEPTH_PASSES * RADIX; j += BS) {
    uint32_t v = 0;
#pragma unroll
    for (int ww = 0; ww < BS / 64; ++ww) v += h[ww][j];
    const int p = j / RADIX, d = j % RADIX;
    if (p == 0) c0[(size_t)d * c_stride + blockIdx.x] = v;
    if (v) atomicAdd(total_at(tot, stripe, p, d), v);
  }
}

// ---------------------------------------------------------------------------
// one row per digit: C[d][p] <- items of smaller digits + items of digit d in
// partitions before p
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BS) void scan_rows(uint32_t *__restrict__ C, size_t c_stride,
                                                const uint32_t *count_dev, uint32_t count,
                                                const uint32_t *__restrict__ tot, int pass) {
  const uint32_t K = item_count(count_dev, count);
  const uint32_t P = (uint32_t)(((uint64_t)K + SPART - 1) / SPART);
  const int d = blockIdx.x;
  uint32_t mine = 0;
  if ((int)threadIdx.x < d) {
#pragma unroll
    for (int s = 0; s < STRIPES; ++s) mine += tot[((size_t)s * MAX_TILE_PASSES + pass) * RADIX + threadIdx.x];
  }
  uint32_t base;
  block_exclusive<uint32_t>(mine, base);
  uint32_t *row = C + (size_t)d * c_stride;
  uint32_t carry = base;
  for (uint32_t c0 = 0; c0 < P; c0 += BS * 4) {
    const uint32_t b = c0 + threadIdx.x * 4;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[j] = b + j < P ? row[b + j] : 0u;
      s += v[j];
    }
    uint32_t chunk;
    uint32_t off = block_exclusive<uint32_t>(s, chunk) + carry;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (b + j < P) row[b + j] = off;
      off += v[j];
    }
    carry += chunk;
  }
}

// ---------------------------------------------------------------------------
// C[d][p]: items of digit d in partition p
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BS) void count_pass(const uint32_t *__restrict__ keys, const uint32_t *count_dev,
                                                 uint32_t count, int shift, int nbits, uint32_t *__restrict__ C,
                                                 size_t c_stride) {
  __shared__ uint32_t h[BS / 64][RADIX];
  const uint32_t K = item_count(count_dev, count);
  const uint32_t nparts = (uint32_t)(((uint64_t)K + SPART - 1) / SPART);
  if (blockIdx.x >= nparts) return;  // capacity-sized grids
  for (int j = threadIdx.x; j < (BS / 64) * RADIX; j += BS) (&h[0][0])[j] = 0u;
  __syncthreads();
  const uint32_t R = 1u << nbits, mask = R - 1u;
  const int w = threadIdx.x >> 6;
  const uint64_t base = (uint64_t)blockIdx.x * SPART + threadIdx.x;
#pragma unroll
  for (int r = 0; r < SIPT; ++r) {
    const uint64_t i = base + (uint64_t)r * BS;
    if (i < K) atomicAdd(&h[w][(keys[i] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < R; d += BS) {
    uint32_t v = 0;
#pragma unroll
    for (int ww = 0; ww < BS / 64; ++ww) v += h[ww][d];
    C[(size_t)d * c_stride + blockIdx.x] = v;
  }
}

// ---------------------------------------------------------------------------
// one stable radix pass (uint32 key, uint32 value)
// ---------------------------------------------------------------------------
enum { SRC_KV = 0, SRC_DEPTH = 1 };                  // where the items come from
enum { DST_KV = 0, DST_ORDER = 1, DST_KEYS = 2 };    // what the pass writes

struct Pass {
  const uint32_t *kin, *vin;             // SRC_KV
  const float *depth;                    // SRC_DEPTH keys; DST_KEYS low key words
  const uint32_t *tiles;                 // SRC_DEPTH keys; DST_ORDER copy counts
  uint32_t n;                            // splat count (bound of the values)
  const uint32_t *count_dev;             // item count in device memory, or NULL ...
  uint32_t count;                        // ... for this host value
  int shift, nbits;                      // this pass's digit
  const uint32_t *C;                     // [digit][partition] output offsets (scan_rows)
  size_t c_stride;
  const uint32_t *bin;                   // depth bits carried with each item (tile passes), or NULL
  uint32_t *kout, *vout, *bout;          // DST_KV; DST_ORDER / DST_KEYS write vout
  uint32_t *cnt_out;                     // DST_ORDER: tiles[value] at the output position
  uint64_t *k64out;                      // DST_KEYS: (key << 32) | the carried depth bits
};

// Items of a partition are ranked in index order: wave w owns a contiguous
// run of 64 * SIPT items, taken 64 at a time; inside a wave the rank among
// equal digits comes from matching the digit bit by bit with ballots, plus a
// per-wave running count per digit in LDS.
template <int SRC, int DST>
__global__ __launch_bounds__(BS) void scatter_pass(Pass a) {
  __shared__ uint32_t wc[BS / 64][RADIX];
  const uint32_t K = item_count(a.count_dev, a.count);
  const uint32_t nparts = (uint32_t)(((uint64_t)K + SPART - 1) / SPART);
  if (blockIdx.x >= nparts) return;  // capacity-sized grids
  const uint32_t part = xcd_partition(blockIdx.x, nparts);
  const uint32_t R = 1u << a.nbits, mask = R - 1u;
  for (int j = threadIdx.x; j < (BS / 64) * RADIX; j += BS) (&wc[0][0])[j] = 0u;
  __syncthreads();

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint64_t base = (uint64_t)part * SPART + (uint64_t)w * (64 * SIPT) + lane;
  uint32_t key[SIPT], val[SIPT], bits[SIPT], rk[SIPT];
#pragma unroll
  for (int r = 0; r < SIPT; ++r) {
    const uint64_t idx = base + (uint64_t)r * 64;
    const bool valid = idx < K;
    if (SRC == SRC_DEPTH) {
      key[r] = valid ? depth_key(a.depth, a.tiles, (uint32_t)idx) : 0u;
      val[r] = (uint32_t)idx;
    } else {
      key[r] = valid ? a.kin[idx] : 0u;
      val[r] = valid ? a.vin[idx] : 0u;
    }
    bits[r] = (a.bin && valid) ? a.bin[idx] : 0u;
  }
#pragma unroll
  for (int r = 0; r < SIPT; ++r) {
    const bool valid = base + (uint64_t)r * 64 < K;
    const uint32_t d = (key[r] >> a.shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < a.nbits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t before = wc[w][d];
    rk[r] = before + (uint32_t)__popcll(peers & lt);
    __builtin_amdgcn_wave_barrier();
    if (valid && (peers & lt) == 0ull) wc[w][d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // per digit: where each wave's items start in the output
  if (threadIdx.x < R) {
    const uint32_t d = threadIdx.x;
    uint32_t run = a.C[(size_t)d * a.c_stride + part];
#pragma unroll
    for (int ww = 0; ww < BS / 64; ++ww) {
      const uint32_t c = wc[ww][d];
      wc[ww][d] = run;
      run += c;
    }
  }
  __syncthreads();

#pragma unroll
  for (int r = 0; r < SIPT; ++r) {
    const uint64_t idx = base + (uint64_t)r * 64;
    if (idx >= K) break;
    const uint32_t d = (key[r] >> a.shift) & mask;
    const uint32_t pos = wc[w][d] + rk[r];
    if (pos >= K) continue;  // unreachable when the counts are consistent
    if (DST == DST_KV) {
      a.kout[pos] = key[r];
      a.vout[pos] = val[r];
      if (a.bout) a.bout[pos] = bits[r];
    } else if (DST == DST_ORDER) {
      a.vout[pos] = val[r];
      a.cnt_out[pos] = val[r] < a.n ? a.tiles[val[r]] : 0u;
    } else {
      a.k64out[pos] = ((uint64_t)key[r] << 32) | bits[r];
      a.vout[pos] = val[r];
    }
  }
}

// ---------------------------------------------------------------------------
// copies of the splats
// ---------------------------------------------------------------------------
// copies per emission partition (plain stores; no inter-workgroup traffic)
__global__ __launch_bounds__(BS) void emit_sums(uint32_t n, const uint32_t *__restrict__ cnt,
                                                uint64_t *__restrict__ esum) {
  const uint64_t s0 = (uint64_t)blockIdx.x * EPART + threadIdx.x;
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < EIPT; ++j)
    if (s0 + (uint64_t)j * BS < n) s += cnt[s0 + (uint64_t)j * BS];
  uint64_t total;
  block_exclusive<uint64_t>(s, total);
  if (threadIdx.x == 0) esum[blockIdx.x] = total;
}

struct Emit {
  uint32_t n;
  const uint32_t *order, *cnt;           // splats in depth order and their copy counts
  const uint64_t *esum;                  // copies per partition
  const int32_t *rect;
  int grid_w;
  uint64_t capacity;
  uint32_t *ctr;
  const float *depth;
  uint32_t *tkey, *tval, *tbits;         // [capacity]: tile id, splat, depth bits
  uint32_t *tot;                         // tile digit totals [stripe][pass][digit]
  int tile_passes, tile_bits;            // digits per key and bits per digit
  int64_t *num_keys;
  int32_t *overflow;
};

// Offsets from the partition sums before this one, then every copy of the
// partition written by the whole workgroup (consecutive threads write
// consecutive keys), counting the tile digits as they are written.
__global__ __launch_bounds__(BS) void emit_copies(Emit a) {
  __shared__ uint32_t loff[EPART + 1];   // local exclusive offsets of the partition's splats
  __shared__ uint32_t sidx[EPART], sbits[EPART];
  __shared__ int32_t sx[EPART], sy[EPART], sw[EPART];
  __shared__ uint32_t th[MAX_TILE_PASSES * RADIX];
  const uint32_t nparts = (uint32_t)(((uint64_t)a.n + EPART - 1) / EPART);
  const uint32_t part = blockIdx.x;
  for (int j = threadIdx.x; j < MAX_TILE_PASSES * RADIX; j += BS) th[j] = 0u;
  // copies before this partition
  uint64_t part_sum = 0, pre;
  for (uint32_t q = threadIdx.x; q < part; q += BS) part_sum += a.esum[q];
  block_exclusive<uint64_t>(part_sum, pre);
  const uint64_t s0 = (uint64_t)part * EPART + (uint64_t)threadIdx.x * EIPT;
  uint32_t c[EIPT];
  uint64_t sum = 0;
#pragma unroll
  for (int j = 0; j < EIPT; ++j) {
    c[j] = s0 + j < a.n ? a.cnt[s0 + j] : 0u;
    sum += c[j];
  }
  uint64_t total;
  uint64_t off = block_exclusive<uint64_t>(sum, total);
  if (threadIdx.x == 0 && part == nparts - 1) {
    const uint64_t K = pre + total;
    const bool over = K > a.capacity;
    *a.num_keys = (int64_t)K;
    *a.overflow = over ? 1 : 0;
    a.ctr[CTR_KEYS] = over ? 0u : (uint32_t)K;
  }
#pragma unroll
  for (int j = 0; j < EIPT; ++j) {
    const int ls = threadIdx.x * EIPT + j;
    loff[ls] = (uint32_t)off;  // only used when the partition fits the capacity (< 2^32)
    off += c[j];
    if (c[j]) {
      const uint32_t i = a.order[s0 + j];
      const int4 r = i < a.n ? reinterpret_cast<const int4 *>(a.rect)[i] : make_int4(0, 0, -1, -1);
      sidx[ls] = i;
      sbits[ls] = i < a.n ? __float_as_uint(a.depth[i]) : 0u;
      sx[ls] = r.x;
      sy[ls] = r.y;
      sw[ls] = r.z - r.x + 1;
    }
  }
  if (threadIdx.x == BS - 1) loff[EPART] = (uint32_t)off;
  __syncthreads();
  if (pre + total > a.capacity || total == 0) return;  // an overflowing call writes no key
  const uint32_t T = (uint32_t)total;
  const uint32_t dmask = (1u << a.tile_bits) - 1u;
  for (uint32_t k = threadIdx.x; k < T; k += BS) {
    uint32_t lo = 0, hi = EPART;  // loff[lo] <= k < loff[hi]
#pragma unroll
    for (int it = 0; it < 10; ++it) {
      const uint32_t mid = (lo + hi) >> 1;
      if (loff[mid] <= k) lo = mid; else hi = mid;
    }
    const uint32_t r = k - loff[lo];
    const int32_t wdt = sw[lo];
    if (wdt <= 0) continue;  // counts that disagree with the rectangle
    const uint32_t q = r / (uint32_t)wdt;
    const uint32_t tile = (uint32_t)(sy[lo] + (int32_t)q) * (uint32_t)a.grid_w +
                          (uint32_t)(sx[lo] + (int32_t)(r - q * (uint32_t)wdt));
    const uint64_t pos = pre + k;
    a.tkey[pos] = tile;
    a.tval[pos] = sidx[lo];
    a.tbits[pos] = sbits[lo];
    for (int p = 0; p < a.tile_passes; ++p) atomicAdd(&th[p * RADIX + ((tile >> (p * a.tile_bits)) & dmask)], 1u);
  }
  __syncthreads();
  const int stripe = blockIdx.x % STRIPES;
  for (int j = threadIdx.x; j < a.tile_passes * RADIX; j += BS) {
    const uint32_t v = th[j];
    if (v) atomicAdd(total_at(a.tot, stripe, j / RADIX, j % RADIX), v);
  }
}

// ranges from the sorted keys
__global__ void tile_ranges(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ ctr, int64_t ntiles,
                            uint32_t *__restrict__ ranges) {
  const uint32_t K = ctr[CTR_KEYS];
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const uint32_t t = (uint32_t)(keys[k] >> 32);
  if ((int64_t)t >= ntiles) return;
  if (k == 0 || (uint32_t)(keys[k - 1] >> 32) != t) ranges[2 * (size_t)t] = (uint32_t)k;
  if (k + 1 == K || (uint32_t)(keys[k + 1] >> 32) != t) ranges[2 * (size_t)t + 1] = (uint32_t)(k + 1);
}

// Longest-list-first dispatch order of the tiles: tiles bucketed by list
// length on a log scale (16 buckets per doubling, so lengths within ~4% share
// a bucket), heaviest bucket first. A workgroup's time grows with its tile's
// list, so starting the long lists first keeps them off the tail of the blend
// launch. The order inside a bucket is unspecified. One workgroup.
__device__ inline int length_bucket(const uint32_t *ranges, int64_t t) {
  const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
  const int b = (int)(log2f((float)len + 1.0f) * 16.0f);
  return 255 - (b < 255 ? b : 255);
}

__global__ __launch_bounds__(1024) void tile_order_kernel(const uint32_t *__restrict__ ranges, int64_t ntiles,
                                                          uint32_t *__restrict__ order) {
  constexpr int NB = 256;
  __shared__ uint32_t hist[NB];
  __shared__ uint32_t wsum[NB / 64];
  if (threadIdx.x < NB) hist[threadIdx.x] = 0u;
  __syncthreads();
  for (int64_t t = threadIdx.x; t < ntiles; t += blockDim.x) atomicAdd(&hist[length_bucket(ranges, t)], 1u);
  __syncthreads();
  uint32_t v = 0, inc = 0;
  if (threadIdx.x < NB) {
    v = hist[threadIdx.x];
    inc = wave_inclusive(v);
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = inc;
  }
  __syncthreads();
  if (threadIdx.x < NB) {
    uint32_t off = inc - v;
    for (int k = 0; k < (int)(threadIdx.x >> 6); ++k) off += wsum[k];
    hist[threadIdx.x] = off;
  }
  __syncthreads();
  for (int64_t t = threadIdx.x; t < ntiles; t += blockDim.x) {
    const uint32_t pos = atomicAdd(&hist[length_bucket(ranges, t)], 1u);
    if ((int64_t)pos < ntiles) order[pos] = (uint32_t)t;
  }
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
struct TilePlan {
  int passes, bits;
};

TilePlan tile_plan(int64_t ntiles) {
  int tile_bits = 1;
  while ((1ll << tile_bits) < ntiles) ++tile_bits;
  TilePlan p;
  p.passes = (tile_bits + 7) / 8;
  p.bits = (tile_bits + p.passes - 1) / p.passes;
  return p;
}

struct Workspace {
  uint32_t *dk0, *dv0, *dk1, *dv1;       // depth sort ping-pong [n]
  uint32_t *order, *cnt;                 // splats in depth order, their copy counts [n]
  uint64_t *esum;                        // copies per emission partition
  uint32_t *tk0, *tv0, *tb0, *tk1, *tv1, *tb1;   // tile sort ping-pong [capacity]
  uint32_t *dC;                          // depth passes' counts [pass][256][depth partitions]
  uint32_t *tC;                          // tile passes' counts [pass][1 << bits][key partitions]
  // zeroed at the start of every call, contiguous:
  uint32_t *ctr;                         // counters
  uint32_t *dtot, *ttot;                 // digit totals [stripe][pass][256]
  void *zero_begin;
  size_t zero_bytes;
  size_t dstride, tstride;               // partitions per row
};

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

size_t carve(void *base, int64_t n, int64_t cap, int64_t ntiles, Workspace *w) {
  const size_t N = (size_t)(n > 0 ? n : 1), C = (size_t)(cap > 0 ? cap : 1);
  const TilePlan tp = tile_plan(ntiles > 0 ? ntiles : 1);
  char *p = (char *)base;
  size_t o = 0;
  auto take = [&](size_t bytes) -> void * {
    void *r = p ? (void *)(p + o) : nullptr;
    o += align_up(bytes);
    return r;
  };
  Workspace t;
  t.dk0 = (uint32_t *)take(4 * N);
  t.dv0 = (uint32_t *)take(4 * N);
  t.dk1 = (uint32_t *)take(4 * N);
  t.dv1 = (uint32_t *)take(4 * N);
  t.order = (uint32_t *)take(4 * N);
  t.cnt = (uint32_t *)take(4 * N);
  t.esum = (uint64_t *)take(8 * (size_t)ceil_div((int64_t)N, EPART));
  t.tk0 = (uint32_t *)take(4 * C);
  t.tv0 = (uint32_t *)take(4 * C);
  t.tb0 = (uint32_t *)take(4 * C);
  t.tk1 = (uint32_t *)take(4 * C);
  t.tv1 = (uint32_t *)take(4 * C);
  t.tb1 = (uint32_t *)take(4 * C);
  t.dstride = (size_t)ceil_div((int64_t)N, SPART);
  t.dC = (uint32_t *)take(4 * (size_t)DEPTH_PASSES * RADIX * t.dstride);
  t.tstride = (size_t)ceil_div((int64_t)C, SPART);
  t.tC = (uint32_t *)take(4 * ((size_t)tp.passes << tp.bits) * t.tstride);
  const size_t z0 = o;
  t.ctr = (uint32_t *)take(4 * CTR_SLOTS);
  t.dtot = (uint32_t *)take(4 * (size_t)STRIPES * MAX_TILE_PASSES * RADIX);
  t.ttot = (uint32_t *)take(4 * (size_t)STRIPES * MAX_TILE_PASSES * RADIX);
  t.zero_begin = p ? (void *)(p + z0) : nullptr;
  t.zero_bytes = o - z0;
  if (w) *w = t;
  return o;
}

}  // namespace

size_t binsort_workspace_bytes(int64_t n, int64_t capacity, int32_t num_tiles) {
  return carve(nullptr, n, capacity, num_tiles, nullptr);
}

hipError_t launch_binsort(int64_t n, const float *depth, const int32_t *rect, const uint32_t *tiles, int grid_w,
                          int grid_h, int64_t capacity, void *ws, size_t, uint64_t *keys, uint32_t *vals,
                          uint32_t *ranges, uint32_t *tile_order, int64_t *num_keys, int32_t *overflow,
                          hipStream_t s) {
  const int64_t ntiles = (int64_t)grid_w * grid_h;
  Workspace w;
  carve(ws, n, capacity, ntiles, &w);
  const TilePlan tp = tile_plan(ntiles);
  const size_t dpass = (size_t)RADIX * w.dstride;             // one depth pass's counts
  const size_t tpass = ((size_t)1 << tp.bits) * w.tstride;    // one tile pass's counts

  // 0. zero totals, counters and ranges; num_keys = overflow = 0
  {
    const size_t nz16 = w.zero_bytes / 16, nr = 2 * (size_t)ntiles;
    const size_t m = nz16 > nr ? nz16 : nr;
    const unsigned grid = (unsigned)(m / BS + 1 < 2048 ? m / BS + 1 : 2048);
    hipLaunchKernelGGL(clear_state, dim3(grid), dim3(BS), 0, s, (uint4 *)w.zero_begin, nz16, ranges, nr, num_keys,
                       overflow);
  }

  if (n > 0) {
    // 1. depth keys: first pass's counts, all passes' totals
    const unsigned dgrid = ceil_div(n, SPART);
    hipLaunchKernelGGL(depth_count, dim3(dgrid), dim3(BS), 0, s, (uint32_t)n, depth, tiles, w.dC, w.dstride,
                       w.dtot);
    // 2. splats by depth (stable, index order on ties): four 8-bit passes; the
    //    last writes the order and each splat's copy count
    Pass a{};
    a.depth = depth;
    a.tiles = tiles;
    a.n = (uint32_t)n;
    a.count = (uint32_t)n;
    a.nbits = 8;
    a.c_stride = w.dstride;
    a.cnt_out = w.cnt;
    uint32_t *kin = nullptr, *vin = nullptr, *kb = w.dk0, *vb = w.dv0, *ka = w.dk1, *va = w.dv1;
    for (int pass = 0; pass < DEPTH_PASSES; ++pass) {
      uint32_t *Cp = w.dC + pass * dpass;
      if (pass > 0)
        hipLaunchKernelGGL(count_pass, dim3(dgrid), dim3(BS), 0, s, (const uint32_t *)kin, (const uint32_t *)nullptr,
                           (uint32_t)n, 8 * pass, 8, Cp, w.dstride);
      hipLaunchKernelGGL(scan_rows, dim3(RADIX), dim3(BS), 0, s, Cp, w.dstride, (const uint32_t *)nullptr,
                         (uint32_t)n, (const uint32_t *)w.dtot, pass);
      a.kin = kin;
      a.vin = vin;
      a.shift = 8 * pass;
      a.C = Cp;
      a.kout = kb;
      a.vout = pass == DEPTH_PASSES - 1 ? w.order : vb;
      if (pass == 0)
        hipLaunchKernelGGL((scatter_pass<SRC_DEPTH, DST_KV>), dim3(dgrid), dim3(BS), 0, s, a);
      else if (pass < DEPTH_PASSES - 1)
        hipLaunchKernelGGL((scatter_pass<SRC_KV, DST_KV>), dim3(dgrid), dim3(BS), 0, s, a);
      else
        hipLaunchKernelGGL((scatter_pass<SRC_KV, DST_ORDER>), dim3(dgrid), dim3(BS), 0, s, a);
      kin = kb;
      vin = vb;
      uint32_t *tk = ka, *tv = va;
      ka = kb; va = vb; kb = tk; vb = tv;
    }
    // 3. copies in depth order with their depth bits, the tile passes' totals, K
    const unsigned egrid = ceil_div(n, EPART);
    hipLaunchKernelGGL(emit_sums, dim3(egrid), dim3(BS), 0, s, (uint32_t)n, (const uint32_t *)w.cnt, w.esum);
    Emit e{};
    e.n = (uint32_t)n;
    e.order = w.order;
    e.cnt = w.cnt;
    e.esum = w.esum;
    e.rect = rect;
    e.grid_w = grid_w;
    e.capacity = (uint64_t)capacity;
    e.ctr = w.ctr;
    e.depth = depth;
    e.tkey = w.tk0;
    e.tval = w.tv0;
    e.tbits = w.tb0;
    e.tot = w.ttot;
    e.tile_passes = tp.passes;
    e.tile_bits = tp.bits;
    e.num_keys = num_keys;
    e.overflow = overflow;
    hipLaunchKernelGGL(emit_copies, dim3(egrid), dim3(BS), 0, s, e);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;

  if (capacity > 0 && n > 0) {
    // 4. stable passes over the tile digits; the last writes the 64-bit keys
    const unsigned kgrid = ceil_div(capacity, SPART);
    Pass a{};
    a.depth = depth;
    a.n = (uint32_t)n;
    a.count_dev = w.ctr + CTR_KEYS;
    a.nbits = tp.bits;
    a.c_stride = w.tstride;
    uint32_t *ka = w.tk0, *va = w.tv0, *ba = w.tb0, *kb = w.tk1, *vb = w.tv1, *bb = w.tb1;
    for (int pass = 0; pass < tp.passes; ++pass) {
      const bool last = pass == tp.passes - 1;
      uint32_t *Cp = w.tC + pass * tpass;
      hipLaunchKernelGGL(count_pass, dim3(kgrid), dim3(BS), 0, s, (const uint32_t *)ka, a.count_dev, 0u,
                         tp.bits * pass, tp.bits, Cp, w.tstride);
      hipLaunchKernelGGL(scan_rows, dim3(1u << tp.bits), dim3(BS), 0, s, Cp, w.tstride, a.count_dev, 0u,
                         (const uint32_t *)w.ttot, pass);
      a.kin = ka;
      a.vin = va;
      a.bin = ba;
      a.shift = tp.bits * pass;
      a.C = Cp;
      a.kout = kb;
      a.vout = last ? vals : vb;
      a.bout = bb;
      a.k64out = keys;
      if (last)
        hipLaunchKernelGGL((scatter_pass<SRC_KV, DST_KEYS>), dim3(kgrid), dim3(BS), 0, s, a);
      else
        hipLaunchKernelGGL((scatter_pass<SRC_KV, DST_KV>), dim3(kgrid), dim3(BS), 0, s, a);
      uint32_t *tk = ka, *tv = va, *tb = ba;
      ka = kb; va = vb; ba = bb; kb = tk; vb = tv; bb = tb;
    }
    // 5. per-tile ranges
    hipLaunchKernelGGL(tile_ranges, dim3(ceil_div(capacity, 256)), dim3(256), 0, s, keys, w.ctr, ntiles, ranges);
  }
  // 6. longest-first dispatch order for the blend
  if (tile_order) hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(1024), 0, s, ranges, ntiles, tile_order);
  return hipGetLastError();
}

}  // namespace gs
