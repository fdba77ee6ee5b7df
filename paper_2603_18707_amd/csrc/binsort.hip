// Tile binning: duplication of splats per covered tile, a stable sort of the
// 64-bit keys (tile_id << 32) | bits(depth), and per-tile ranges.
//
// The sorted order is (tile, depth, splat index): a stable sort of the copies
// emitted in splat-index order (tiles row-major inside each splat). It is
// reached in two steps that each sort only what varies:
//  1. the copies, emitted in splat-index order, are grouped by tile with a
//     stable LSD radix sort on the ceil(log2 tiles) tile bits only (two 7-bit
//     passes at 1080p), so inside a tile they stay in index order;
//  2. each tile's list is sorted stably by depth bits: by one wave when it
//     holds at most 510 copies, by a workgroup in LDS up to 2048 copies and
//     in chunks of that size through global memory beyond, all in one
//     kernel (longest lists dispatched first, so they overlap the rest).
//     Keys are offset by the tile's smallest depth, so only the bits that
//     vary inside the tile are sorted (usually 3 of 4 bytes).
// With a capacity of 2048 or more copies per tile, the splats are instead
// sorted by depth first and their copies emitted in that order, so the tile
// passes alone give the final order. With per-tile culling, the copies come
// from the culling kernels (cull_count, sums_scan, cull_emit) and then take
// the same route.
// A radix pass of step 1 is three kernels and no workgroup ever waits on
// another (a hand-off between workgroups costs ~0.5 us through memory, and
// device atomics on scattered addresses cost more than the pass itself):
//  * count_pass: the key array is cut into partitions of SPART items;
//    C[d][p] = items of digit d in partition p (LDS histogram, plain stores).
//  * scan_rows: one workgroup per digit turns its row into output offsets:
//    the items of smaller digits (from digit totals known in advance) plus
//    the row's exclusive prefix.
//  * scatter_pass: each partition ranks its items stably (per-wave ballot
//    matching of the digit, waves in index order) and writes them at
//    C[d][p] + rank.
// Digit totals do not depend on the order: the emission kernel counts them
// as it writes the copies, in 8 striped copies (by workgroup) so no address
// sees more than an eighth of the workgroups. Each copy carries its depth
// bits, so no pass gathers depths.
//
// Every kernel sized by the key count reads it from device memory and grids
// are sized by the key capacity, so the stage runs without a host round trip
// (and can be captured in a graph).
#include "blend_common.h"
#include "gs_internal.h"

namespace gs {

namespace {

constexpr int BS = 256;                 // threads per workgroup
constexpr int SIPT = 4;                 // items per thread in a sort partition
constexpr int SPART = BS * SIPT;        // items per sort partition
constexpr int LONG_SIPT = 8;            // the same on the long lists' route
constexpr int EIPT = 4;                 // splats per thread in an emission partition
constexpr int EPART = BS * EIPT;        // splats per emission partition
constexpr int RADIX = 256;              // max buckets per pass (8-bit digits)
static_assert(BS == RADIX, "per-digit steps give one digit to each thread");
constexpr int MAX_TILE_PASSES = 4;      // tile ids < 2^30 need at most four digits of <= 8 bits
constexpr int STRIPES = 8;              // copies of the digit totals
constexpr int SEG_IPT = 8;              // copies per thread of a workgroup's list sort (2048 in LDS)
// Average list length (capacity per tile) from which the tile passes take
// partitions of BS * LONG_SIPT keys, so each digit leaves a partition in
// longer runs
constexpr int64_t LONG_SEG_MIN_AVG = 512;
constexpr int DEPTH_PASSES = 4;         // 8-bit digits of a float's bits
// Average list length from which the splats are sorted by depth before the
// emission (no per-tile sort): lists this long are sorted by the per-tile
// kernel in chunks through global memory, at a fraction of the HBM rate.
constexpr int64_t PRESORT_MIN_AVG = 2048;
static_assert(DEPTH_PASSES <= MAX_TILE_PASSES, "the depth totals share the tile totals' layout");

enum : int { CTR_KEYS = 0, CTR_SPLIT = 1, CTR_SLOTS = 16 };

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

// The lanes of the wave whose digit d (its low `nbits` bits) equals this
// lane's, among the lanes where `valid` holds: a ballot per bit, and from it
// the lanes that agree with this lane's bit, peers & ~(ballot ^ s) with s
// this lane's bit spread over the word, one three-input logic op per word
// (v_bitop3_b32; its truth table is indexed by the operand bits as
// 4 src0 + 2 src1 + src2, so f(a, b, c) = a & ~(b ^ c) is 0x90).
constexpr int MATCH_LUT = 0x90;
__device__ inline uint64_t match_digit(uint32_t d, int nbits, bool valid) {
  const uint64_t v = __ballot(valid);
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  for (int b = 0; b < nbits; ++b) {
    const uint32_t s = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d, b, 1);  // all ones where bit b is set
    const uint64_t bb = __builtin_amdgcn_uicmp(s, 0u, 33);  // ballot of s != 0 (33: not equal)
    lo = __builtin_amdgcn_bitop3_b32(lo, (uint32_t)bb, s, MATCH_LUT);
    hi = __builtin_amdgcn_bitop3_b32(hi, (uint32_t)(bb >> 32), s, MATCH_LUT);
  }
  return ((uint64_t)hi << 32) | lo;
}

// set bits of m below this lane: the lane's rank among the lanes of m
__device__ inline uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
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
// one row per digit: C[d][p] <- items of smaller digits + items of digit d in
// partitions before p
// ---------------------------------------------------------------------------
template <int IPT>
__global__ __launch_bounds__(BS) void scan_rows(uint32_t *__restrict__ C, size_t c_stride,
                                                const uint32_t *count_dev, uint32_t count,
                                                const uint32_t *__restrict__ tot, int pass) {
  constexpr int PART = BS * IPT;
  const uint32_t K = item_count(count_dev, count);
  const uint32_t P = (uint32_t)(((uint64_t)K + PART - 1) / PART);
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
template <int IPT>
__global__ __launch_bounds__(BS) void count_pass(const uint32_t *__restrict__ keys, const uint32_t *count_dev,
                                                 uint32_t count, int shift, int nbits, uint32_t *__restrict__ C,
                                                 size_t c_stride) {
  constexpr int PART = BS * IPT;
  __shared__ uint32_t h[BS / 64][RADIX];
  const uint32_t K = item_count(count_dev, count);
  const uint32_t nparts = (uint32_t)(((uint64_t)K + PART - 1) / PART);
  if (blockIdx.x >= nparts) return;  // capacity-sized grids
  for (int j = threadIdx.x; j < (BS / 64) * RADIX; j += BS) (&h[0][0])[j] = 0u;
  __syncthreads();
  const uint32_t R = 1u << nbits, mask = R - 1u;
  const int w = threadIdx.x >> 6;
  // consecutive partitions on one XCD: the column stores of neighbouring
  // partitions share cache lines, which then merge in that XCD's L2
  const uint32_t part = xcd_partition(blockIdx.x, nparts);
  const uint64_t base = (uint64_t)part * PART + threadIdx.x;
  uint32_t d[IPT];
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint64_t i = base + (uint64_t)r * BS;
    d[r] = i < K ? (keys[i] >> shift) & mask : 0u;
  }
  // keys often arrive in runs of equal digits (grouped by the lower digits):
  // a wave whose digits are all equal adds its count once instead of
  // serializing 64 atomics on one word (valid lanes are a prefix of the wave)
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const bool valid = base + (uint64_t)r * BS < K;
    const uint32_t first = __builtin_amdgcn_readfirstlane(d[r]);
    const uint64_t vm = __ballot(valid);
    if (vm != 0ull && __ballot(valid && d[r] == first) == vm) {  // uniform
      if ((threadIdx.x & 63) == 0) atomicAdd(&h[w][first], (uint32_t)__popcll(vm));
    } else if (valid) {
      atomicAdd(&h[w][d[r]], 1u);
    }
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < R; d += BS) {
    uint32_t v = 0;
#pragma unroll
    for (int ww = 0; ww < BS / 64; ++ww) v += h[ww][d];
    C[(size_t)d * c_stride + part] = v;
  }
}

// ---------------------------------------------------------------------------
// one stable radix pass over (tile id, splat, depth bits)
// ---------------------------------------------------------------------------
struct Pass {
  const uint32_t *kin, *vin, *bin;       // keys (tile ids or depth bits), splats, depth bits;
                                         // vin NULL: the value is the item's index; bin may be NULL
  const uint32_t *count_dev;             // item count in device memory, or NULL for `count`
  uint32_t count;
  int shift, nbits;                      // this pass's digit
  const uint32_t *C;                     // [digit][partition] output offsets (scan_rows)
  size_t c_stride;
  uint32_t *kout, *vout, *bout;          // bout may be NULL
  uint64_t *keys_final;                  // non-NULL: write (key << 32 | bits) and the value here instead
  uint32_t *vals_final;
};

// Items of a partition (BS * IPT of them) are ranked in index order: wave w
// owns a contiguous run of 64 * IPT items, taken 64 at a time; inside a wave the rank among
// equal digits comes from matching the digit bit by bit with ballots, plus a
// per-wave running count per digit in LDS.
template <int IPT>
__global__ __launch_bounds__(BS) void scatter_pass(Pass a) {
  constexpr int PART = BS * IPT;
  __shared__ uint32_t wc[BS / 64][RADIX];
  __shared__ uint32_t goff[RADIX];
  __shared__ uint32_t Ks[PART], Vs[PART], Bs[PART];
  const uint32_t K = item_count(a.count_dev, a.count);
  const uint32_t nparts = (uint32_t)(((uint64_t)K + PART - 1) / PART);
  if (blockIdx.x >= nparts) return;  // capacity-sized grids
  const uint32_t part = xcd_partition(blockIdx.x, nparts);
  const uint32_t R = 1u << a.nbits, mask = R - 1u;
  for (int j = threadIdx.x; j < (BS / 64) * RADIX; j += BS) (&wc[0][0])[j] = 0u;
  __syncthreads();

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t base = (uint64_t)part * PART + (uint64_t)w * (64 * IPT) + lane;
  uint32_t key[IPT], val[IPT], bits[IPT], rk[IPT];
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint64_t idx = base + (uint64_t)r * 64;
    const bool valid = idx < K;
    key[r] = valid ? a.kin[idx] : 0u;
    val[r] = valid ? (a.vin ? a.vin[idx] : (uint32_t)idx) : 0u;
    bits[r] = valid && a.bin ? a.bin[idx] : 0u;
  }
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const bool valid = base + (uint64_t)r * 64 < K;
    const uint32_t d = (key[r] >> a.shift) & mask;
    const uint64_t peers = match_digit(d, a.nbits, valid);
    const uint32_t before = wc[w][d];
    const uint32_t below = lanes_below(peers);
    rk[r] = before + below;
    __builtin_amdgcn_wave_barrier();
    if (valid && below == 0u) wc[w][d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // The partition's items are first placed in digit order in LDS, then
  // written out by consecutive threads: item i of the staged order goes to
  // goff[d] + i, so every digit run leaves as one contiguous burst instead of
  // one scattered 4-byte store per item.
  {
    const uint32_t d = threadIdx.x;  // BS == RADIX: one digit per thread
    uint32_t tot = 0;
    if (d < R) {
#pragma unroll
      for (int ww = 0; ww < BS / 64; ++ww) tot += wc[ww][d];
    }
    uint32_t unused;
    uint32_t run = block_exclusive<uint32_t>(tot, unused);
    if (d < R) {
      goff[d] = a.C[(size_t)d * a.c_stride + part] - run;
#pragma unroll
      for (int ww = 0; ww < BS / 64; ++ww) {
        const uint32_t c = wc[ww][d];
        wc[ww][d] = run;
        run += c;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    if (base + (uint64_t)r * 64 < K) {
      const uint32_t local = wc[w][(key[r] >> a.shift) & mask] + rk[r];
      if (local < PART) {  // always, when the counts are consistent
        Ks[local] = key[r];
        Vs[local] = val[r];
        Bs[local] = bits[r];
      }
    }
  }
  __syncthreads();
  const uint64_t p0 = (uint64_t)part * PART;
  const uint32_t m = K - p0 < (uint64_t)PART ? (uint32_t)(K - p0) : (uint32_t)PART;
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint32_t i = threadIdx.x + (uint32_t)r * BS;
    if (i < m) {
      const uint32_t k = Ks[i];
      const uint32_t pos = goff[(k >> a.shift) & mask] + i;
      if (pos < K) {  // always, when the counts are consistent
        if (a.keys_final) {
          a.keys_final[pos] = ((uint64_t)k << 32) | (uint64_t)Bs[i];
          a.vals_final[pos] = Vs[i];
        } else {
          a.kout[pos] = k;
          a.vout[pos] = Vs[i];
          if (a.bout) a.bout[pos] = Bs[i];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// copies of the splats, in splat-index order
// ---------------------------------------------------------------------------
// copies per emission partition (plain stores; no inter-workgroup traffic);
// also resets the call's state (what clear_state does when n = 0) unless z
// is NULL (it was reset before). The emission order is perm[0..n) when perm
// is given (splats sorted by depth), else splat-index order.
__global__ __launch_bounds__(BS) void emit_sums(uint32_t n, const uint32_t *__restrict__ tiles,
                                                const uint32_t *__restrict__ perm, uint64_t *__restrict__ esum,
                                                uint4 *__restrict__ z, size_t nz16, uint32_t *__restrict__ ranges,
                                                size_t nr, int64_t *num_keys, int32_t *overflow) {
  if (z) {
    const size_t i = (size_t)blockIdx.x * BS + threadIdx.x, stride = (size_t)gridDim.x * BS;
    for (size_t j = i; j < nz16; j += stride) z[j] = make_uint4(0u, 0u, 0u, 0u);
    for (size_t j = i; j < nr; j += stride) ranges[j] = 0u;
    if (i == 0) {
      *num_keys = 0;
      *overflow = 0;
    }
  }
  const uint64_t s0 = (uint64_t)blockIdx.x * EPART + threadIdx.x;
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < EIPT; ++j) {
    const uint64_t i = s0 + (uint64_t)j * BS;
    if (i < n) s += tiles[perm ? perm[i] : i];
  }
  uint64_t total;
  block_exclusive<uint64_t>(s, total);
  if (threadIdx.x == 0) esum[blockIdx.x] = total;
}

struct Emit {
  uint32_t n;
  const uint32_t *perm;                  // emission order (NULL: splat-index order)
  const uint32_t *tiles;                 // copies per splat (rectangle areas)
  const uint64_t *esum;                  // copies per partition
  const int32_t *rect;
  const float *depth;
  int grid_w;
  uint64_t capacity;
  uint32_t *ctr;
  uint32_t *tkey, *tval, *tbits;         // [capacity]: tile id, splat, depth bits
  uint32_t *tot;                         // tile digit totals [stripe][pass][digit]
  int tile_passes, tile_bits;            // digits per key and bits per digit
  int64_t *num_keys;
  int32_t *overflow;
  bool scanned;                          // esum holds exclusive prefixes and K is set (sums_scan ran)
  bool row_digits;                       // count the tile digits per rectangle row, not per copy
};

// From this many emission partitions the partition sums are scanned once
// (sums_scan) instead of each workgroup adding up the sums before its own,
// which costs O(partitions^2) loads (3 ms at the 84k partitions of the
// 96-view batch, a few us below this).
constexpr uint32_t EMIT_SCAN_MIN_PARTS = 4096;

// Tile digits of a run of len consecutive tile ids from t0, counted per run:
// the lowest digit takes len >> bits copies in every bin (all0) and one more
// in the len & mask bins from t0's on (a range, possibly wrapping, kept in the
// difference array d0); each higher digit takes the overlap of the run with
// every value of t >> (p bits) it spans, a few per run. Counting per copy
// instead puts a run's equal high digits, from consecutive threads, on one
// LDS word.
__device__ inline void count_run_digits(uint32_t t0, uint32_t len, int bits, int passes, uint32_t *th, uint32_t *d0,
                                        uint32_t *all0) {
  const uint32_t R0 = 1u << bits, dmask = R0 - 1u, t1 = t0 + len - 1u;
  if (len >> bits) atomicAdd(all0, len >> bits);
  const uint32_t rem = len & dmask, s0 = t0 & dmask, e0 = s0 + rem;
  if (rem) {
    atomicAdd(&d0[s0], 1u);
    if (e0 <= R0) {
      atomicSub(&d0[e0], 1u);
    } else {
      atomicSub(&d0[R0], 1u);
      atomicAdd(&d0[0], 1u);
      atomicSub(&d0[e0 - R0], 1u);
    }
  }
  for (int pp = 1; pp < passes; ++pp) {
    const int sh = pp * bits;
    for (uint32_t v = t0 >> sh; v <= (t1 >> sh); ++v) {
      const uint32_t lo = max(t0, v << sh), hi = min(t1, ((v + 1u) << sh) - 1u);
      atomicAdd(&th[pp * RADIX + (v & dmask)], hi - lo + 1u);
    }
  }
}

// adds the lowest digit's counts (prefix of d0 plus all0) into th[0..R0);
// every thread of the workgroup calls it after the last count
__device__ inline void flush_lowest_digit(uint32_t *th, const uint32_t *d0, const uint32_t *all0, int bits) {
  __syncthreads();
  const uint32_t d = threadIdx.x, dmask = (1u << bits) - 1u;  // BS == RADIX
  uint32_t unused;
  const uint32_t v = d <= dmask ? d0[d] : 0u;
  const uint32_t inc = block_exclusive<uint32_t>(v, unused) + v;
  if (d <= dmask) th[d] += inc + *all0;
  __syncthreads();
}

// Offsets from the partition sums before this one, then every copy of the
// partition written by the whole workgroup (consecutive threads write
// consecutive keys), counting the tile digits as they are written. The
// copies are taken EWIN at a time: each splat marks the window position of
// its first copy with its local index, and an inclusive max-scan over the
// window gives every position its splat (splats in order, so the last mark
// at or before a position is its splat), one LDS read per copy instead of a
// binary search.
constexpr int EWIN = BS * 8;            // copies per window
static_assert(EPART <= 65536, "local splat indices are 16-bit");

// inclusive max-scan over m[0..EWIN) (8 consecutive entries per thread),
// starting from `carry`; returns the window's last value
__device__ inline uint32_t window_max_scan(uint16_t *m, uint32_t carry, uint32_t *wmax) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint4 raw = reinterpret_cast<uint4 *>(m)[threadIdx.x];
  uint32_t v[8] = {raw.x & 0xFFFFu, raw.x >> 16, raw.y & 0xFFFFu, raw.y >> 16,
                   raw.z & 0xFFFFu, raw.z >> 16, raw.w & 0xFFFFu, raw.w >> 16};
#pragma unroll
  for (int i = 1; i < 8; ++i) v[i] = max(v[i], v[i - 1]);
  uint32_t inc = v[7];
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)inc, o, 64);
    if (lane >= o) inc = max(inc, y);
  }
  if (lane == 63) wmax[w] = inc;
  uint32_t before = (uint32_t)__shfl_up((int)inc, 1, 64);
  if (lane == 0) before = 0u;
  __syncthreads();
  uint32_t pre = carry;
#pragma unroll
  for (int k = 0; k < BS / 64; ++k)
    if (k < w) pre = max(pre, wmax[k]);
  pre = max(pre, before);
  uint32_t last = carry;
#pragma unroll
  for (int k = 0; k < BS / 64; ++k) last = max(last, wmax[k]);
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = max(v[i], pre);
  raw.x = v[0] | (v[1] << 16);
  raw.y = v[2] | (v[3] << 16);
  raw.z = v[4] | (v[5] << 16);
  raw.w = v[6] | (v[7] << 16);
  reinterpret_cast<uint4 *>(m)[threadIdx.x] = raw;
  return last;
}

__global__ __launch_bounds__(BS) void emit_copies(Emit a) {
  __shared__ uint32_t loff[EPART];       // local exclusive offsets of the partition's splats
  __shared__ uint32_t sbits[EPART];
  __shared__ int32_t sx[EPART], sy[EPART], sw[EPART];
  __shared__ float sinv[EPART];          // 1 / width
  __shared__ uint32_t ssp[EPART];        // splat of each emission position
  __shared__ uint32_t th[MAX_TILE_PASSES * RADIX];
  __shared__ uint32_t d0[RADIX + 1], all0;  // lowest digit, counted per run (count_run_digits)
  __shared__ __align__(16) uint16_t owner[EWIN];
  __shared__ uint32_t wmax[BS / 64];
  const uint32_t nparts = (uint32_t)(((uint64_t)a.n + EPART - 1) / EPART);
  const uint32_t part = blockIdx.x;
  for (int j = threadIdx.x; j < MAX_TILE_PASSES * RADIX; j += BS) th[j] = 0u;
  for (int j = threadIdx.x; j <= RADIX; j += BS) d0[j] = 0u;
  if (threadIdx.x == 0) all0 = 0u;
  // copies before this partition
  uint64_t pre;
  if (a.scanned) {  // uniform
    pre = a.esum[part];
  } else {
    uint64_t part_sum = 0;
    for (uint32_t q = threadIdx.x; q < part; q += BS) part_sum += a.esum[q];
    block_exclusive<uint64_t>(part_sum, pre);
  }
  const uint64_t s0 = (uint64_t)part * EPART + (uint64_t)threadIdx.x * EIPT;
  uint32_t c[EIPT];
  uint64_t sum = 0;
  uint32_t sp[EIPT];  // the splats at these emission positions
#pragma unroll
  for (int j = 0; j < EIPT; ++j) {
    sp[j] = s0 + j < a.n ? (a.perm ? a.perm[s0 + j] : (uint32_t)(s0 + j)) : 0u;
    c[j] = s0 + j < a.n ? a.tiles[sp[j]] : 0u;
    sum += c[j];
  }
  uint64_t total;
  uint64_t off = block_exclusive<uint64_t>(sum, total);
  if (!a.scanned && threadIdx.x == 0 && part == nparts - 1) {
    const uint64_t K = pre + total;
    const bool over = K > a.capacity;
    *a.num_keys = (int64_t)K;
    *a.overflow = over ? 1 : 0;
    a.ctr[CTR_KEYS] = over ? 0u : (uint32_t)K;
  }
  uint32_t first[EIPT];  // local offset of each of this thread's splats
#pragma unroll
  for (int j = 0; j < EIPT; ++j) {
    const int ls = threadIdx.x * EIPT + j;
    first[j] = (uint32_t)off;  // only used when the partition fits the capacity (< 2^32)
    loff[ls] = (uint32_t)off;
    off += c[j];
    if (c[j]) {
      const int4 r = reinterpret_cast<const int4 *>(a.rect)[sp[j]];
      sbits[ls] = __float_as_uint(a.depth[sp[j]]);
      ssp[ls] = sp[j];
      sx[ls] = r.x;
      sy[ls] = r.y;
      sw[ls] = r.z - r.x + 1;
      sinv[ls] = r.z >= r.x ? 1.0f / (float)(r.z - r.x + 1) : 0.0f;
    }
  }
  if (pre + total > a.capacity || total == 0) return;  // an overflowing call writes no key (uniform)
  const uint32_t T = (uint32_t)total;
  const uint32_t dmask = (1u << a.tile_bits) - 1u;
  __syncthreads();  // the resets above before the counts
  // With long rows (the depth-first route's large splats) the tile digits of
  // this thread's splats are counted once per rectangle row (the copies below
  // take the rows in the same way: copy r of a splat is column r % w of row
  // r / w); with short ones, per copy as the copies are written (per row,
  // each thread walks its splats' rows alone: 14.5 -> 22 us at 1M splats).
#pragma unroll
  for (int j = 0; j < EIPT; ++j) {
    const int ls = threadIdx.x * EIPT + j;
    if (!a.row_digits || !c[j] || sw[ls] <= 0) continue;
    const uint32_t wdt = (uint32_t)sw[ls], rows = c[j] / wdt, rest = c[j] - rows * wdt;
    for (uint32_t q = 0; q <= rows; ++q) {
      const uint32_t len = q < rows ? wdt : rest;
      if (len)
        count_run_digits((uint32_t)(sy[ls] + (int32_t)q) * (uint32_t)a.grid_w + (uint32_t)sx[ls], len, a.tile_bits,
                         a.tile_passes, th, d0, &all0);
    }
  }
  uint32_t carry = 0;
  for (uint32_t k0 = 0; k0 < T; k0 += EWIN) {  // uniform trip count
    reinterpret_cast<uint4 *>(owner)[threadIdx.x] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();  // also orders the staging above before its readers
#pragma unroll
    for (int j = 0; j < EIPT; ++j)
      if (c[j] && first[j] >= k0 && first[j] - k0 < (uint32_t)EWIN)
        owner[first[j] - k0] = (uint16_t)(threadIdx.x * EIPT + j);
    __syncthreads();
    carry = window_max_scan(owner, carry, wmax);
    __syncthreads();
    const uint32_t m = T - k0 < (uint32_t)EWIN ? T - k0 : (uint32_t)EWIN;
    for (uint32_t i = threadIdx.x; i < m; i += BS) {
      const uint32_t ls = owner[i];
      const uint32_t r = k0 + i - loff[ls];
      const int32_t wdt = sw[ls];
      if (wdt <= 0) continue;  // counts that disagree with the rectangle
      // r / wdt: below 2^22 the float product is within 1/2 of the quotient,
      // so one correction step makes it exact
      uint32_t q;
      if (r < (1u << 22)) {
        q = (uint32_t)((float)r * sinv[ls]);
        if (q * (uint32_t)wdt > r) --q;
        else if ((q + 1u) * (uint32_t)wdt <= r) ++q;
      } else {
        q = r / (uint32_t)wdt;
      }
      const uint32_t tile = (uint32_t)(sy[ls] + (int32_t)q) * (uint32_t)a.grid_w +
                            (uint32_t)(sx[ls] + (int32_t)(r - q * (uint32_t)wdt));
      const uint64_t pos = pre + k0 + i;
      a.tkey[pos] = tile;
      a.tval[pos] = ssp[ls];
      a.tbits[pos] = sbits[ls];
      if (!a.row_digits)
        for (int p = 0; p < a.tile_passes; ++p) atomicAdd(&th[p * RADIX + ((tile >> (p * a.tile_bits)) & dmask)], 1u);
    }
    __syncthreads();  // the window's readers are done before it is cleared
  }
  if (a.row_digits) flush_lowest_digit(th, d0, &all0, a.tile_bits);  // uniform
  const int stripe = blockIdx.x % STRIPES;
  for (int j = threadIdx.x; j < a.tile_passes * RADIX; j += BS) {
    const uint32_t v = th[j];
    if (v) atomicAdd(total_at(a.tot, stripe, j / RADIX, j % RADIX), v);
  }
}

// ---------------------------------------------------------------------------
// tile culling: copies only for the tiles a splat can reach
// ---------------------------------------------------------------------------
struct Cull {
  const float *means2d, *conic_opacity;  // the projected records
  BlendParams p;                         // kernel and eps, for cull_cut (tiles are TS pixels wide)
  // each row's kept run [a, b], saved by cull_count for cull_emit: workgroup
  // g owns rcap slots at seg[g / per_seg] + (g % per_seg) * rcap (buffers the
  // tile passes use later), 16-bit slots a | b << 8 when the grid is at most
  // 256 tiles wide, else 32-bit a | b << 16; a workgroup with more rows than
  // rcap saves none
  uint32_t *seg[3];
  uint32_t rcap, per_seg;
  bool narrow;
};

struct SpanSlots {
  void *p;
  bool narrow;
  __device__ void put(uint32_t k, int a, int b) const {
    if (narrow)
      static_cast<uint16_t *>(p)[k] = (uint16_t)((uint32_t)(a & 0xFF) | ((uint32_t)(b & 0xFF) << 8));
    else
      static_cast<uint32_t *>(p)[k] = (uint32_t)a | ((uint32_t)b << 16);
  }
  __device__ void get(uint32_t k, int &a, int &b) const {
    if (narrow) {
      const uint32_t w = static_cast<const uint16_t *>(p)[k];
      a = (int)(w & 0xFFu);
      b = (int)(w >> 8);
    } else {
      const uint32_t w = static_cast<const uint32_t *>(p)[k];
      a = (int)(w & 0xFFFFu);
      b = (int)(w >> 16);
    }
  }
};

__device__ inline SpanSlots span_slots(const Cull &cu, uint32_t g) {
  const size_t off = (size_t)(g % cu.per_seg) * cu.rcap;
  uint32_t *base = cu.seg[g / cu.per_seg];
  return SpanSlots{cu.narrow ? (void *)(reinterpret_cast<uint16_t *>(base) + off) : (void *)(base + off), cu.narrow};
}

// One workgroup of the culled binning takes BS splats (in emission order)
// and walks their rectangle rows, BS rows at a time: rows, not tiles, are
// the unit of work, so a splat covering thousands of tiles costs a few dozen
// row items and the workgroup's lanes stay evenly loaded. Per splat it keeps
// what the tile test needs, in double: the conic (a, b, c) with b/a, b/c,
// det/a, det/c and 1/a precomputed, the cut, and the half extents
// X = sqrt(cut c / det), Y = sqrt(cut a / det) of the region Q <= cut.
struct CullLds {
  uint32_t roff[BS + 1];  // row items of the workgroup's splats before each splat
  float u[BS], v[BS], A[BS], C[BS];
  double iA[BS], bA[BS], bC[BS], dA[BS], dC[BS], cut[BS], X[BS], Y[BS];
  int32_t x0[BS], x1[BS], y0[BS];
  uint32_t sp[BS], bits[BS];
};

// Stages the workgroup's splats; returns its row items. A splat without
// tiles or with an empty rectangle has no row; otherwise its rows are those
// of its rectangle (with cut < 0 all of them empty), counted from the
// rectangle alone, so `full` = false stages only what writing saved runs
// needs (splat, depth bits, first row) and gives the same row items.
__device__ inline uint32_t cull_stage(uint32_t n, const uint32_t *perm, const uint32_t *tiles, const int32_t *rect,
                                      const float *depth, const Cull &cu, CullLds &L, bool full = true) {
#pragma clang fp contract(off)
  const uint64_t pos = (uint64_t)blockIdx.x * BS + threadIdx.x;
  const int j = threadIdx.x;
  uint32_t rows = 0;
  if (pos < n) {
    const uint32_t s = perm ? perm[pos] : (uint32_t)pos;
    const int4 r = tiles[s] != 0u ? reinterpret_cast<const int4 *>(rect)[s] : make_int4(0, 0, -1, -1);
    if (r.z >= r.x && r.w >= r.y) {
      rows = (uint32_t)(r.w - r.y + 1);
      L.y0[j] = r.y;
      L.sp[j] = s;
      L.bits[j] = depth ? __float_as_uint(depth[s]) : 0u;
      L.cut[j] = -1.0;
    }
    if (full && rows) {
      const float2 m = reinterpret_cast<const float2 *>(cu.means2d)[s];
      const float4 co = reinterpret_cast<const float4 *>(cu.conic_opacity)[s];
      const double cut = cull_cut(cu.p, co.w, co.x, co.y, co.z);
      if (cut >= 0.0) {
        const double A = co.x, B = co.y, C = co.z, det = A * C - B * B;
        const double iA = 1.0 / A, iC = 1.0 / C, cd = cut / det;
        L.u[j] = m.x;
        L.v[j] = m.y;
        L.A[j] = co.x;
        L.C[j] = co.z;
        L.iA[j] = iA;
        L.bA[j] = B * iA;
        L.bC[j] = B * iC;
        L.dA[j] = det * iA;
        L.dC[j] = det * iC;
        L.cut[j] = cut;
        L.X[j] = sqrt(cd * C);
        L.Y[j] = sqrt(cd * A);
        L.x0[j] = r.x;
        L.x1[j] = r.z;
      }
    }
  }
  uint32_t total;
  L.roff[j] = block_exclusive<uint32_t>(rows, total);
  if (j == BS - 1) L.roff[BS] = total;
  __syncthreads();
  return total;
}

// row item k of the workgroup: its splat j (roff[j] <= k < roff[j + 1]) and tile row
__device__ inline void row_item(const CullLds &L, uint32_t k, int &j, int &ty) {
  uint32_t lo = 0, hi = BS;
#pragma unroll
  for (int it = 0; it < 8; ++it) {
    const uint32_t mid = (lo + hi) >> 1;
    if (L.roff[mid] <= k) lo = mid; else hi = mid;
  }
  j = (int)lo;
  ty = L.y0[lo] + (int)(k - L.roff[lo]);
}

// The tile test: whether the least Q over the pixel-centre rectangle of
// tile (tx, ty) is at most cut. Zero when the mean is inside; otherwise the
// least value over the four edges, where Q restricted to an edge is a
// quadratic minimised at its vertex clamped to the edge, written as a
// completed square (two non-negative terms, no cancellation):
//   along dy = y: Q = a (dx - xs)^2 + (det / a) y^2, xs = -(b / a) y;
//   along dx = x: Q = c (dy - ys)^2 + (det / c) x^2, ys = -(b / c) x.
// Its relative error is a few ulps of double, so only minima within ~1e-15
// of cut can be decided differently by another double evaluation.
__device__ inline bool tile_kept(const CullLds &L, int j, int tx, int ty) {
#pragma clang fp contract(off)
  constexpr int T = TS;
  const double u = L.u[j], v = L.v[j];
  const double x0 = ((double)(tx * T) + 0.5) - u, x1 = ((double)(tx * T + T) - 0.5) - u;
  const double y0 = ((double)(ty * T) + 0.5) - v, y1 = ((double)(ty * T + T) - 0.5) - v;
  if (x0 <= 0.0 && x1 >= 0.0 && y0 <= 0.0 && y1 >= 0.0) return true;
  const double A = L.A[j], C = L.C[j], bA = L.bA[j], bC = L.bC[j], dA = L.dA[j], dC = L.dC[j], cut = L.cut[j];
  double q = cut + 1.0;
  const double ya[2] = {y0, y1}, xa[2] = {x0, x1};
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const double y = ya[e], xs = -(bA * y);
    const double dx = fmin(fmax(xs, x0), x1) - xs;
    q = fmin(q, A * (dx * dx) + dA * (y * y));
    const double x = xa[e], ys = -(bC * x);
    const double dy = fmin(fmax(ys, y0), y1) - ys;
    q = fmin(q, C * (dy * dy) + dC * (x * x));
  }
  return q <= cut;
}

// The kept tiles of row ty of splat j, [a, b] (a > b: none). The region
// Q <= cut is convex, so its tiles in a row are contiguous: the row's strip
// of pixel-centre offsets meets the ellipse in an x-interval, found in
// closed form (the ellipse's right side x_r(y) = -(b/a) y +
// sqrt((cut - (det/a) y^2) / a) is concave with its apex at y = -(b/c) X, so
// its largest value over the strip is at that apex clamped to the strip;
// the left side likewise), widened by 1e-3 px + 1e-6 (X + Y) so that it
// holds every tile the test can keep. From both ends of that candidate
// range tiles are put to the test until one is kept; those between are kept
// untested (they hold points of the ellipse's interior). Only ties within
// rounding of cut on two or more tiles of one row could make a per-tile
// evaluation differ.
__device__ inline void row_span(const CullLds &L, int j, int ty, int &a, int &b) {
#pragma clang fp contract(off)
  constexpr int T = TS;
  a = 1;
  b = 0;
  const double cut = L.cut[j];
  if (!(cut >= 0.0)) return;  // no pixel passes
  const double v = L.v[j], X = L.X[j], Y = L.Y[j];
  const double y0 = ((double)(ty * T) + 0.5) - v, y1 = ((double)(ty * T + T) - 0.5) - v;
  const double m = 1e-3 + 1e-6 * (X + Y);
  if (y0 > Y + m || y1 < -Y - m) return;
  double lo = fmax(y0, -Y), hi = fmin(y1, Y);
  if (lo > hi) lo = hi = (y0 > 0.0 ? Y : -Y);  // the strip passes within m of a tip
  const double bA = L.bA[j], dA = L.dA[j], iA = L.iA[j];
  const double yr = -(L.bC[j] * X);           // apex of the right side; the left one's is at -yr
  const double ya = fmin(fmax(yr, lo), hi), yb = fmin(fmax(-yr, lo), hi);
  const double ra = cut - dA * (ya * ya), rb = cut - dA * (yb * yb);
  const double u = L.u[j];
  const double xmax = -(bA * ya) + (ra > 0.0 ? sqrt(ra * iA) : 0.0) + m;
  const double xmin = -(bA * yb) - (rb > 0.0 ? sqrt(rb * iA) : 0.0) - m;
  // tiles whose pixel-centre span [T tx + 0.5 - u, T tx + T - 0.5 - u] meets [xmin, xmax]
  const double ca = fmax(ceil(((xmin + u) - ((double)T - 0.5)) * (1.0 / T)), (double)L.x0[j]);
  const double cb = fmin(floor(((xmax + u) - 0.5) * (1.0 / T)), (double)L.x1[j]);
  if (!(ca <= cb)) return;
  int ia = (int)ca, ib = (int)cb;
  while (ia <= ib && !tile_kept(L, j, ia, ty)) ++ia;
  if (ia > ib) return;
  while (ib > ia && !tile_kept(L, j, ib, ty)) --ib;
  a = ia;
  b = ib;
}

// kept copies per workgroup of BS emission positions (esum)
__global__ __launch_bounds__(BS) void cull_count(uint32_t n, const uint32_t *__restrict__ perm,
                                                 const uint32_t *__restrict__ tiles, const int32_t *__restrict__ rect,
                                                 Cull cu, uint64_t *__restrict__ esum) {
  __shared__ CullLds L;
  const uint32_t R = cull_stage(n, perm, tiles, rect, nullptr, cu, L);
  const bool save = R <= cu.rcap;
  const SpanSlots saved = span_slots(cu, blockIdx.x);
  uint64_t kept = 0;
  for (uint32_t k = threadIdx.x; k < R; k += BS) {
    int j, ty, a, b;
    row_item(L, k, j, ty);
    row_span(L, j, ty, a, b);
    if (a <= b) {
      kept += (uint64_t)(b - a + 1);
    } else {
      a = 1;  // one encoding for every empty run
      b = 0;
    }
    if (save) saved.put(k, a, b);  // tile columns < 2^15 (< 2^8 for narrow slots)
  }
  uint64_t total;
  block_exclusive<uint64_t>(kept, total);
  if (threadIdx.x == 0) esum[blockIdx.x] = total;
}

// esum -> exclusive prefix in place; K, overflow and the key counter from
// the total. One workgroup of CS_THREADS scans the partition sums in tiles of
// CS_THREADS x CS_ITEMS consecutive sums, all of a tile's loads in flight
// together, carrying the running total from tile to tile. The culled
// emission's sums always take it, the plain emission's from
// EMIT_SCAN_MIN_PARTS partitions on.
constexpr int CS_THREADS = 1024, CS_ITEMS = 4;

__global__ __launch_bounds__(CS_THREADS) void sums_scan(uint64_t *__restrict__ esum, uint32_t parts,
                                                        uint64_t capacity, uint32_t *__restrict__ ctr,
                                                        int64_t *num_keys, int32_t *overflow) {
  __shared__ uint64_t wsum[CS_THREADS / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t carry = 0;
  for (uint32_t t0 = 0; t0 < parts; t0 += CS_THREADS * CS_ITEMS) {
    const uint32_t b = t0 + threadIdx.x * CS_ITEMS;
    uint64_t v[CS_ITEMS], sum = 0;
#pragma unroll
    for (int j = 0; j < CS_ITEMS; ++j) {
      v[j] = b + j < parts ? esum[b + j] : 0ull;
      sum += v[j];
    }
    const uint64_t inc = wave_inclusive<uint64_t>(sum);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint64_t off = carry + inc - sum, tot = 0;
#pragma unroll
    for (int k = 0; k < CS_THREADS / 64; ++k) {
      const uint64_t x = wsum[k];
      if (k < w) off += x;
      tot += x;
    }
    __syncthreads();  // wsum is reused by the next tile
#pragma unroll
    for (int j = 0; j < CS_ITEMS; ++j) {
      if (b + j < parts) esum[b + j] = off;
      off += v[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    const bool over = carry > capacity;
    *num_keys = (int64_t)carry;
    *overflow = over ? 1 : 0;
    ctr[CTR_KEYS] = over ? 0u : (uint32_t)carry;
  }
}

// The kept copies of the workgroup's splats, in emission order (splats in
// order, each one's tiles row-major), nothing when the call overflows. Row
// items BS at a time: each takes its row's run of tiles and its place from a
// workgroup scan of the runs' lengths, and counts the run's tile digits (the
// lowest digit as a range of bins, in a difference array, the higher ones
// per value, a few per run); then the round's copies are written by
// consecutive threads to consecutive keys, each copy finding its row by a
// max-scan over window marks (as in emit_copies). Per-copy stores from one
// thread per run would scatter every store instruction over 64 runs, and
// per-copy digit atomics would put a run's equal high digits on one LDS word.
__global__ __launch_bounds__(BS) void cull_emit(Emit a, Cull cu) {
  __shared__ CullLds L;
  __shared__ uint32_t th[MAX_TILE_PASSES * RADIX];
  __shared__ uint32_t d0[RADIX + 1];  // lowest digit: difference array of the runs' bin ranges
  __shared__ uint32_t all0;           // whole cycles of the lowest digit (one copy in every bin)
  __shared__ uint32_t rloc[BS], rtile[BS], rsp[BS], rbits[BS];  // the round's rows: place, first tile, splat, bits
  __shared__ __align__(16) uint16_t owner[EWIN];
  __shared__ uint32_t wmax[BS / 64];
  for (int j = threadIdx.x; j < MAX_TILE_PASSES * RADIX; j += BS) th[j] = 0u;
  for (int j = threadIdx.x; j <= RADIX; j += BS) d0[j] = 0u;
  if (threadIdx.x == 0) all0 = 0u;
  // the row items of the rectangles alone first: whether cull_count saved the runs
  uint32_t R = cull_stage(a.n, a.perm, a.tiles, a.rect, a.depth, cu, L, false);  // orders the resets too
  if (*a.overflow) return;  // uniform: written before this launch
  const bool save = R <= cu.rcap;
  const SpanSlots saved = span_slots(cu, blockIdx.x);
  if (!save) R = cull_stage(a.n, a.perm, a.tiles, a.rect, a.depth, cu, L);  // recompute the runs
  uint64_t carry = a.esum[blockIdx.x];
  for (uint32_t base = 0; base < R; base += BS) {  // uniform trip count
    const uint32_t k = base + threadIdx.x;
    int j = 0, ty = 0, ta = 1, tb = 0;
    if (k < R) {
      row_item(L, k, j, ty);
      if (save) {
        saved.get(k, ta, tb);
      } else {
        row_span(L, j, ty, ta, tb);
      }
    }
    const uint32_t len = ta <= tb ? (uint32_t)(tb - ta + 1) : 0u;
    uint32_t chunk;
    const uint32_t loc = block_exclusive<uint32_t>(len, chunk);  // ends with a barrier
    if (len) {
      const uint32_t t0 = (uint32_t)ty * (uint32_t)a.grid_w + (uint32_t)ta;
      rloc[threadIdx.x] = loc;
      rtile[threadIdx.x] = t0;
      rsp[threadIdx.x] = L.sp[j];
      rbits[threadIdx.x] = L.bits[j];
      count_run_digits(t0, len, a.tile_bits, a.tile_passes, th, d0, &all0);
    }
    // the round's copies, consecutive threads on consecutive keys
    uint32_t wcarry = 0;
    for (uint32_t k0 = 0; k0 < chunk; k0 += EWIN) {  // uniform trip count
      reinterpret_cast<uint4 *>(owner)[threadIdx.x] = make_uint4(0u, 0u, 0u, 0u);
      __syncthreads();  // also orders the round's row table before its readers
      if (len && loc >= k0 && loc - k0 < (uint32_t)EWIN) owner[loc - k0] = (uint16_t)threadIdx.x;
      __syncthreads();
      wcarry = window_max_scan(owner, wcarry, wmax);
      __syncthreads();
      const uint32_t m = chunk - k0 < (uint32_t)EWIN ? chunk - k0 : (uint32_t)EWIN;
      for (uint32_t i = threadIdx.x; i < m; i += BS) {
        const uint32_t r = owner[i], c = k0 + i;
        const uint64_t o = carry + c;
        if (o < a.capacity) {  // always, when the counts are consistent
          a.tkey[o] = rtile[r] + (c - rloc[r]);
          a.tval[o] = rsp[r];
          a.tbits[o] = rbits[r];
        }
      }
      __syncthreads();  // the window and the row table are reused
    }
    carry += chunk;
  }
  flush_lowest_digit(th, d0, &all0, a.tile_bits);
  const int stripe = blockIdx.x % STRIPES;
  for (int j = threadIdx.x; j < a.tile_passes * RADIX; j += BS) {
    const uint32_t v = th[j];
    if (v) atomicAdd(total_at(a.tot, stripe, j / RADIX, j % RADIX), v);
  }
}

// per-byte histograms of the splats' depth bits: the digit totals of the
// depth passes, in striped copies like the tile digit totals
__global__ __launch_bounds__(BS) void depth_hist(const float *__restrict__ depth, uint32_t n, uint32_t *__restrict__ tot) {
  __shared__ uint32_t h[DEPTH_PASSES * RADIX];
  for (int j = threadIdx.x; j < DEPTH_PASSES * RADIX; j += BS) h[j] = 0u;
  __syncthreads();
  for (uint64_t i = (uint64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (uint64_t)gridDim.x * BS) {
    const uint32_t b = __float_as_uint(depth[i]);
#pragma unroll
    for (int p = 0; p < DEPTH_PASSES; ++p) atomicAdd(&h[p * RADIX + ((b >> (8 * p)) & 255u)], 1u);
  }
  __syncthreads();
  const int stripe = blockIdx.x % STRIPES;
  for (int j = threadIdx.x; j < DEPTH_PASSES * RADIX; j += BS) {
    const uint32_t v = h[j];
    if (v) atomicAdd(total_at(tot, stripe, j / RADIX, j % RADIX), v);
  }
}

// ranges from the tile-grouped copies: tile ids in 32-bit keys, or in the
// high half of the final 64-bit keys (WIDE)
// each thread takes RIPT consecutive keys (and their neighbours), all
// loaded at once
constexpr int RIPT = 4;

template <bool WIDE>
__global__ __launch_bounds__(BS) void tile_ranges(const void *__restrict__ tkey, const uint32_t *__restrict__ ctr,
                                                  int64_t ntiles, uint32_t *__restrict__ ranges) {
  const uint32_t K = ctr[CTR_KEYS];
  const uint64_t k0 = ((uint64_t)blockIdx.x * BS + threadIdx.x) * RIPT;
  if (k0 >= K) return;
  auto at = [&](uint64_t i) -> uint32_t {
    return WIDE ? (uint32_t)(reinterpret_cast<const uint64_t *>(tkey)[i] >> 32) : reinterpret_cast<const uint32_t *>(tkey)[i];
  };
  uint32_t t[RIPT + 2];  // keys k0 - 1 .. k0 + RIPT (0xFFFFFFFF outside [0, K))
#pragma unroll
  for (int j = 0; j < RIPT + 2; ++j) {
    const int64_t i = (int64_t)k0 - 1 + j;
    t[j] = i >= 0 && i < (int64_t)K ? at((uint64_t)i) : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int j = 1; j <= RIPT; ++j) {
    const uint64_t k = k0 - 1 + j;
    if (k >= K || (int64_t)t[j] >= ntiles) continue;
    if (t[j - 1] != t[j]) ranges[2 * (size_t)t[j]] = (uint32_t)k;
    if (t[j + 1] != t[j]) ranges[2 * (size_t)t[j] + 1] = (uint32_t)(k + 1);
  }
}

// Lists of at most WAVE_MAX copies are sorted by one wave alone (four
// copies per lane up to WAVE_SHORT, else eight). Length buckets are
// floor(16 log2(len + 1)): 510 copies fall in bucket 143 and 511 in bucket
// 144, so in the longest-first order every longer list comes before every
// such one, and the order kernel records where they start.
constexpr uint32_t WAVE_MAX = 510;
constexpr int WAVE_BUCKET = 143;
constexpr uint32_t WAVE_SHORT = 256;

__device__ inline int bucket_of_length(uint32_t len) {
  const int b = (int)(log2f((float)len + 1.0f) * 16.0f);
  return 255 - (b < 255 ? b : 255);
}

// One workgroup; each thread takes tiles tid + 1024 k in groups of ORD_ITEMS,
// all of a group's range loads in flight together (the kernel is a few
// dependent round trips to memory, so their number sets its time), and keeps
// the ranges and buckets of the first group for the scatter.
constexpr int ORD_THREADS = 1024, ORD_ITEMS = 8;

__global__ __launch_bounds__(ORD_THREADS) void tile_order_kernel(const uint32_t *__restrict__ ranges, int64_t ntiles,
                                                                 uint32_t *__restrict__ order,
                                                                 uint32_t *__restrict__ split) {
  constexpr int NB = 256;
  __shared__ uint32_t hist[NB];
  __shared__ uint32_t wsum[NB / 64];
  if (threadIdx.x < NB) hist[threadIdx.x] = 0u;
  __syncthreads();
  constexpr int64_t GROUP = (int64_t)ORD_THREADS * ORD_ITEMS;
  int first[ORD_ITEMS];
  uint2 frng[ORD_ITEMS];
  for (int64_t g0 = 0; g0 < ntiles; g0 += GROUP) {
    uint2 rg[ORD_ITEMS];
#pragma unroll
    for (int k = 0; k < ORD_ITEMS; ++k) {
      const int64_t t = g0 + threadIdx.x + (int64_t)k * ORD_THREADS;
      rg[k] = t < ntiles ? make_uint2(ranges[2 * t], ranges[2 * t + 1]) : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int k = 0; k < ORD_ITEMS; ++k) {
      const int64_t t = g0 + threadIdx.x + (int64_t)k * ORD_THREADS;
      const int b = t < ntiles ? bucket_of_length(rg[k].y - rg[k].x) : -1;
      if (b >= 0) atomicAdd(&hist[b], 1u);
      if (g0 == 0) {
        first[k] = b;
        frng[k] = rg[k];
      }
    }
  }
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
    if (split && threadIdx.x == 255 - WAVE_BUCKET) *split = off;  // first position of a list <= WAVE_MAX
  }
  __syncthreads();
  for (int64_t g0 = 0; g0 < ntiles; g0 += GROUP) {
    int b[ORD_ITEMS];
    uint2 rg[ORD_ITEMS];
#pragma unroll
    for (int k = 0; k < ORD_ITEMS; ++k) {
      const int64_t t = g0 + threadIdx.x + (int64_t)k * ORD_THREADS;
      if (g0 == 0) {
        b[k] = first[k];
        rg[k] = frng[k];
      } else {
        rg[k] = t < ntiles ? make_uint2(ranges[2 * t], ranges[2 * t + 1]) : make_uint2(0u, 0u);
        b[k] = t < ntiles ? bucket_of_length(rg[k].y - rg[k].x) : -1;
      }
    }
#pragma unroll
    for (int k = 0; k < ORD_ITEMS; ++k) {
      if (b[k] >= 0) {
        const uint32_t pos = atomicAdd(&hist[b[k]], 1u);
        if ((int64_t)pos < ntiles) order[pos] = (uint32_t)(g0 + threadIdx.x + (int64_t)k * ORD_THREADS);
      }
    }
  }
}

// The same order for large grids (the stacked views of a batch): a bucket
// histogram per chunk of ORD_CHUNK tiles, an exclusive scan over the
// bucket-major [bucket][chunk] counts, and a scatter through per-chunk bucket
// cursors in LDS; one workgroup would take hundreds of microseconds.
constexpr int64_t ORD_MULTI_MIN = 65536;  // tiles from which the order takes these three kernels
constexpr int ORD_CHUNK = BS * 8;         // tiles per workgroup there

inline uint32_t order_chunks(int64_t ntiles) { return (uint32_t)((ntiles + ORD_CHUNK - 1) / ORD_CHUNK); }

__global__ __launch_bounds__(BS) void order_hist(const uint32_t *__restrict__ ranges, int64_t ntiles,
                                                 uint32_t *__restrict__ H, uint32_t G) {
  __shared__ uint32_t h[RADIX];
  h[threadIdx.x] = 0u;  // BS == RADIX
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * ORD_CHUNK + threadIdx.x;
  uint32_t len[ORD_CHUNK / BS];
#pragma unroll
  for (int j = 0; j < ORD_CHUNK / BS; ++j) {
    const int64_t t = t0 + (int64_t)j * BS;
    len[j] = t < ntiles ? ranges[2 * t + 1] - ranges[2 * t] : 0u;
  }
#pragma unroll
  for (int j = 0; j < ORD_CHUNK / BS; ++j)
    if (t0 + (int64_t)j * BS < ntiles) atomicAdd(&h[bucket_of_length(len[j])], 1u);
  __syncthreads();
  H[(size_t)threadIdx.x * G + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of H[0..m) in place, one workgroup, CS_THREADS x 4 entries per step with a carry
__global__ __launch_bounds__(1024) void order_offsets(uint32_t *__restrict__ H, uint32_t m) {
  constexpr int NT = 1024, IT = 4;
  __shared__ uint32_t wsum[NT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (uint32_t t0 = 0; t0 < m; t0 += NT * IT) {
    const uint32_t b = t0 + threadIdx.x * IT;
    uint32_t v[IT], sum = 0;
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      v[j] = b + j < m ? H[b + j] : 0u;
      sum += v[j];
    }
    const uint32_t inc = wave_inclusive<uint32_t>(sum);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = carry + inc - sum, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) {
      const uint32_t x = wsum[k];
      if (k < w) off += x;
      tot += x;
    }
    __syncthreads();  // wsum is reused by the next step
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      if (b + j < m) H[b + j] = off;
      off += v[j];
    }
    carry += tot;
  }
}

__global__ __launch_bounds__(BS) void order_scatter(const uint32_t *__restrict__ ranges, int64_t ntiles,
                                                    const uint32_t *__restrict__ H, uint32_t G,
                                                    uint32_t *__restrict__ order, uint32_t *__restrict__ split) {
  __shared__ uint32_t cur[RADIX];
  cur[threadIdx.x] = H[(size_t)threadIdx.x * G + blockIdx.x];
  // first position of a list <= WAVE_MAX: where that bucket starts, in chunk 0
  if (split && blockIdx.x == 0 && threadIdx.x == 255 - WAVE_BUCKET) *split = cur[threadIdx.x];
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * ORD_CHUNK + threadIdx.x;
#pragma unroll
  for (int j = 0; j < ORD_CHUNK / BS; ++j) {
    const int64_t t = t0 + (int64_t)j * BS;
    if (t < ntiles) {
      const uint32_t pos = atomicAdd(&cur[bucket_of_length(ranges[2 * t + 1] - ranges[2 * t])], 1u);
      if ((int64_t)pos < ntiles) order[pos] = (uint32_t)t;
    }
  }
}

// ---------------------------------------------------------------------------
// per-tile stable sort by depth bits
// ---------------------------------------------------------------------------
// Stable ranking of a chunk of m <= BS * IPT items held wave-contiguously in
// registers (item i = w * 64 * R + r * 64 + lane, R = ceil(m / 256) rounds,
// so every wave holds a share) by the 8-bit digit at `shift`: rk[r] = number
// of the wave's earlier items with the same digit, wc[w][d] += the wave's
// count of digit d (wc zeroed by the caller).
__device__ inline uint32_t chunk_rounds(uint32_t m) { return (m + BS - 1) / BS; }

template <int IPT>
__device__ inline void rank_chunk(const uint32_t (&key)[IPT], uint32_t (&rk)[IPT], uint32_t m, int shift,
                                  uint32_t (*wc)[RADIX]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t R = chunk_rounds(m);
  const uint32_t wbase = (uint32_t)w * 64u * R;
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    if ((uint32_t)r < R && wbase + (uint32_t)r * 64u < m) {  // uniform over the wave
      const bool valid = wbase + (uint32_t)r * 64u + (uint32_t)lane < m;
      const uint32_t d = (key[r] >> shift) & 255u;
      const uint64_t peers = match_digit(d, 8, valid);
      const uint32_t before = wc[w][d];
      const uint32_t below = lanes_below(peers);
      rk[r] = before + below;
      __builtin_amdgcn_wave_barrier();
      if (valid && below == 0u) wc[w][d] = before + (uint32_t)__popcll(peers);
      __builtin_amdgcn_wave_barrier();
    }
  }
}

struct Seg {
  const uint32_t *ranges, *order;        // order may be NULL (row-major dispatch)
  int64_t ntiles;
  const uint32_t *bits, *vals;           // tile-grouped copies: depth bits, splat (index order in a tile)
  uint32_t *sbits, *svals;               // scratch with the same indexing (lists longer than 4096)
  uint64_t *keys;                        // outputs
  uint32_t *vout;
  const uint32_t *split;                 // with an order: first position of a list <= WAVE_MAX
};

// A stable LSD radix sort of one tile's list by depth bits, by a workgroup.
// The keys are the depth bits minus the tile's smallest one (same order,
// same ties), and only the bytes that vary are sorted, low byte first, with
// the list spread over all four waves (ceil(n / 256) rounds of 64 per wave).
// Up to BS * IPT copies are sorted in LDS; a longer list is sorted chunk by
// chunk through global memory (per pass a digit count over the whole list,
// then the chunks in order, ranked in registers and written to the other
// buffer). Returns with the workgroup converged.
template <int IPT>
struct SortLds {
  uint32_t Kb[BS * IPT], Vb[BS * IPT];
  uint32_t wc[BS / 64][RADIX];
  uint32_t run[RADIX];
  uint32_t s_mn[BS / 64], s_mx[BS / 64];
};

template <int IPT>
__device__ __forceinline__ void sort_list(const Seg &a, uint32_t t, uint32_t start, uint32_t n, SortLds<IPT> &sl) {
  constexpr int SEG_IPT = IPT;
  constexpr int SEG_CAP = BS * IPT;
  uint32_t *Kb = sl.Kb, *Vb = sl.Vb, *run = sl.run, *s_mn = sl.s_mn, *s_mx = sl.s_mx;
  uint32_t (*wc)[RADIX] = sl.wc;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t tkey = (uint64_t)t << 32;
  uint32_t key[SEG_IPT], val[SEG_IPT], rk[SEG_IPT];
  const bool in_lds = n <= SEG_CAP;
  const uint32_t R0 = chunk_rounds(in_lds ? n : (uint32_t)SEG_CAP);
  const uint32_t wbase0 = (uint32_t)w * 64u * R0 + (uint32_t)lane;

  // the tile's depth range; a list that fits in LDS is loaded into registers
  // here (every load in flight at once), a longer one is scanned 8 loads at a time
  uint32_t mn = 0xFFFFFFFFu, mx = 0u;
  if (in_lds) {
#pragma unroll
    for (int r = 0; r < SEG_IPT; ++r) {
      const uint32_t i = wbase0 + (uint32_t)r * 64u;
      const bool mine = (uint32_t)r < R0 && i < n;
      key[r] = mine ? a.bits[start + i] : 0u;
      val[r] = mine ? a.vals[start + i] : 0u;
      if (mine) {
        mn = min(mn, key[r]);
        mx = max(mx, key[r]);
      }
    }
  } else {
    for (uint32_t i0 = threadIdx.x; i0 < n; i0 += 8 * BS) {
      uint32_t k8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) k8[u] = i0 + u * BS < n ? a.bits[start + i0 + u * BS] : 0u;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (i0 + u * BS < n) {
          mn = min(mn, k8[u]);
          mx = max(mx, k8[u]);
        }
      }
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    mn = min(mn, (uint32_t)__shfl_xor((int)mn, o, 64));
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
  }
  if (lane == 0) {
    s_mn[w] = mn;
    s_mx[w] = mx;
  }
  __syncthreads();
  mn = s_mn[0];
  mx = s_mx[0];
#pragma unroll
  for (int k = 1; k < BS / 64; ++k) {
    mn = min(mn, s_mn[k]);
    mx = max(mx, s_mx[k]);
  }
  const uint32_t span = mx - mn;
  const int passes = span ? (32 - __clz(span) + 7) / 8 : 0;

  if (in_lds) {
    const uint32_t R = R0;
    const uint32_t wbase = wbase0;
#pragma unroll
    for (int r = 0; r < SEG_IPT; ++r) key[r] -= mn;  // unused slots are never read
    for (int p = 0; p < passes; ++p) {
      for (int j = threadIdx.x; j < (BS / 64) * RADIX; j += BS) (&wc[0][0])[j] = 0u;
      __syncthreads();
      rank_chunk<IPT>(key, rk, n, 8 * p, wc);
      __syncthreads();
      {
        const uint32_t d = threadIdx.x;  // BS == RADIX: one digit per thread
        uint32_t tot = 0;
#pragma unroll
        for (int ww = 0; ww < BS / 64; ++ww) tot += wc[ww][d];
        uint32_t unused;
        uint32_t r0 = block_exclusive<uint32_t>(tot, unused);
#pragma unroll
        for (int ww = 0; ww < BS / 64; ++ww) {
          const uint32_t c = wc[ww][d];
          wc[ww][d] = r0;
          r0 += c;
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < SEG_IPT; ++r) {
        if ((uint32_t)r < R && wbase + (uint32_t)r * 64u < n) {
          const uint32_t pos = wc[w][(key[r] >> (8 * p)) & 255u] + rk[r];
          if (pos < n) {  // always, when the counts are consistent
            Kb[pos] = key[r];
            Vb[pos] = val[r];
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < SEG_IPT; ++r) {
        const uint32_t i = wbase + (uint32_t)r * 64u;
        if ((uint32_t)r < R && i < n) {
          key[r] = Kb[i];
          val[r] = Vb[i];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < SEG_IPT; ++r) {
      const uint32_t i = wbase + (uint32_t)r * 64u;
      if ((uint32_t)r < R && i < n) {
        a.keys[start + i] = tkey | (uint64_t)(key[r] + mn);
        a.vout[start + i] = val[r];
      }
    }
    return;
  }

  // long list: each pass is a digit count over the whole list, then the list
  // in order, SEG_CAP at a time, ranked in registers and written to the other
  // buffer (the last pass writes the outputs)
  if (passes == 0) {
    for (uint32_t i = threadIdx.x; i < n; i += BS) {
      a.keys[start + i] = tkey | (uint64_t)a.bits[start + i];
      a.vout[start + i] = a.vals[start + i];
    }
    return;
  }
  for (int p = 0; p < passes; ++p) {
    const bool first = p == 0, last = p == passes - 1;
    const uint32_t *kin = (p & 1) ? a.sbits : a.bits;  // pass 0 reads the raw bits
    const uint32_t *vin = (p & 1) ? a.svals : a.vals;
    uint32_t *kout = (p & 1) ? (uint32_t *)a.bits : a.sbits;
    uint32_t *vout = (p & 1) ? (uint32_t *)a.vals : a.svals;
    const uint32_t sub = first ? mn : 0u;
    if (threadIdx.x < RADIX) run[threadIdx.x] = 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += BS) atomicAdd(&run[((kin[start + i] - sub) >> (8 * p)) & 255u], 1u);
    __syncthreads();
    {
      uint32_t unused;
      const uint32_t excl = block_exclusive<uint32_t>(run[threadIdx.x], unused);
      __syncthreads();
      run[threadIdx.x] = excl;
    }
    __syncthreads();
    for (uint32_t c0 = 0; c0 < n; c0 += SEG_CAP) {
      const uint32_t m = min((uint32_t)SEG_CAP, n - c0);
      const uint32_t R = chunk_rounds(m);
      const uint32_t wbase = (uint32_t)w * 64u * R + (uint32_t)lane;
#pragma unroll
      for (int r = 0; r < SEG_IPT; ++r) {
        const uint32_t i = wbase + (uint32_t)r * 64u;
        const bool mine = (uint32_t)r < R && i < m;
        key[r] = mine ? kin[start + c0 + i] - sub : 0u;
        val[r] = mine ? vin[start + c0 + i] : 0u;
      }
      for (int j = threadIdx.x; j < (BS / 64) * RADIX; j += BS) (&wc[0][0])[j] = 0u;
      __syncthreads();
      rank_chunk<IPT>(key, rk, m, 8 * p, wc);
      __syncthreads();
      {
        const uint32_t d = threadIdx.x;
        uint32_t r0 = run[d];
#pragma unroll
        for (int ww = 0; ww < BS / 64; ++ww) {
          const uint32_t c = wc[ww][d];
          wc[ww][d] = r0;
          r0 += c;
        }
        run[d] = r0;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < SEG_IPT; ++r) {
        if ((uint32_t)r < R && wbase + (uint32_t)r * 64u < m) {
          const uint32_t pos = wc[w][(key[r] >> (8 * p)) & 255u] + rk[r];
          if (pos >= n) continue;  // unreachable when the counts are consistent
          if (last) {
            a.keys[start + pos] = tkey | (uint64_t)(key[r] + mn);
            a.vout[start + pos] = val[r];
          } else {
            kout[start + pos] = key[r];
            vout[start + pos] = val[r];
          }
        }
      }
      __syncthreads();
    }
  }
}

// LDS of one wave sorting a list of at most WAVE_MAX copies
struct WaveLds {
  uint32_t Kb[WAVE_MAX], Vb[WAVE_MAX], wc[RADIX];
};

// orders a wave's LDS writes before its later reads by other lanes
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same stable LSD sort as sort_list for a list of n <= 64 IPT copies,
// by one wave and without workgroup barriers: copy i = r * 64 + lane is held
// by lane `lane` in round r, rounds are ranked in order (earlier copies
// first, so equal keys keep their order), and the 256 digit counts are
// scanned by the wave, four per lane.
template <int IPT>
__device__ inline void sort_list_wave(const Seg &a, uint32_t t, uint32_t start, uint32_t n, WaveLds &wl) {
  const int lane = threadIdx.x & 63;
  const uint32_t R = (n + 63) / 64;
  uint32_t key[IPT], val[IPT], rk[IPT];
  uint32_t mn = 0xFFFFFFFFu, mx = 0u;
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint32_t i = (uint32_t)r * 64u + (uint32_t)lane;
    const bool mine = i < n;
    key[r] = mine ? a.bits[start + i] : 0u;
    val[r] = mine ? a.vals[start + i] : 0u;
    if (mine) {
      mn = min(mn, key[r]);
      mx = max(mx, key[r]);
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    mn = min(mn, (uint32_t)__shfl_xor((int)mn, o, 64));
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
  }
  const uint32_t span = mx - mn;
  const int passes = span ? (32 - __clz(span) + 7) / 8 : 0;
#pragma unroll
  for (int r = 0; r < IPT; ++r) key[r] -= mn;  // unused slots are never read
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
#pragma unroll
    for (int j = 0; j < RADIX / 64; ++j) wl.wc[j * 64 + lane] = 0u;
    wave_sync();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      if ((uint32_t)r < R) {  // uniform over the wave
        const bool valid = (uint32_t)r * 64u + (uint32_t)lane < n;
        const uint32_t d = (key[r] >> shift) & 255u;
        const uint64_t peers = match_digit(d, 8, valid);
        const uint32_t before = wl.wc[d];
        const uint32_t below = lanes_below(peers);
        rk[r] = before + below;
        wave_sync();
        if (valid && below == 0u) wl.wc[d] = before + (uint32_t)__popcll(peers);
        wave_sync();
      }
    }
    {  // exclusive offsets of the 256 digits: lane takes digits 4 lane .. 4 lane + 3
      uint32_t c[4], sum = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        c[j] = wl.wc[4 * lane + j];
        sum += c[j];
      }
      uint32_t off = wave_inclusive<uint32_t>(sum) - sum;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        wl.wc[4 * lane + j] = off;
        off += c[j];
      }
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      if ((uint32_t)r * 64u + (uint32_t)lane < n) {
        const uint32_t pos = wl.wc[(key[r] >> shift) & 255u] + rk[r];
        if (pos < n) {  // always, when the counts are consistent
          wl.Kb[pos] = key[r];
          wl.Vb[pos] = val[r];
        }
      }
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const uint32_t i = (uint32_t)r * 64u + (uint32_t)lane;
      if (i < n) {
        key[r] = wl.Kb[i];
        val[r] = wl.Vb[i];
      }
    }
    wave_sync();
  }
  const uint64_t tkey = (uint64_t)t << 32;
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint32_t i = (uint32_t)r * 64u + (uint32_t)lane;
    if (i < n) {
      a.keys[start + i] = tkey | (uint64_t)(key[r] + mn);
      a.vout[start + i] = val[r];
    }
  }
}

// Every tile's list. With a longest-first order, workgroup b < S (S = the
// first position of a list of at most WAVE_MAX copies) takes position b
// alone and sorts it with all its waves; the later workgroups take four
// consecutive positions from S on, one wave each, side by side. Without an
// order every workgroup takes one tile. Either way a list is sorted by the
// whole workgroup when it is longer than WAVE_MAX, else by one wave; the
// grid has one workgroup per tile and the spare ones exit.
template <int IPT>
// at most 80 VGPRs: six waves per SIMD instead of five (no spills)
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(6, 6))) void segment_sort(Seg a) {
  __shared__ union {
    SortLds<IPT> sl;
    WaveLds wl[BS / 64];
  } lds;
  constexpr int NQ = BS / 64;
  const int w = threadIdx.x >> 6;
  const int64_t S = a.split ? min((int64_t)*a.split, a.ntiles) : a.ntiles;
  const int64_t b = blockIdx.x;
  int64_t first;
  int cnt;
  if (b < S) {
    first = b;
    cnt = 1;
  } else {
    first = S + NQ * (b - S);
    cnt = NQ;
  }
  if (first >= a.ntiles) return;
  uint32_t tt[NQ], st[NQ], nn[NQ];
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    const int64_t pos = first + j;
    nn[j] = 0u;
    tt[j] = 0u;
    st[j] = 0u;
    if (j < cnt && pos < a.ntiles) {
      tt[j] = a.order ? min(a.order[pos], (uint32_t)(a.ntiles - 1)) : (uint32_t)pos;
      st[j] = a.ranges[2 * (size_t)tt[j]];
      const uint32_t e = a.ranges[2 * (size_t)tt[j] + 1];
      nn[j] = e > st[j] ? e - st[j] : 0u;
    }
  }
#pragma unroll
  for (int j = 0; j < NQ; ++j) {  // uniform over the workgroup
    if (nn[j] > WAVE_MAX) {
      sort_list<IPT>(a, tt[j], st[j], nn[j], lds.sl);
      __syncthreads();  // the LDS is reused
    }
  }
  if (nn[w] > 0u && nn[w] <= WAVE_SHORT)
    sort_list_wave<WAVE_SHORT / 64>(a, tt[w], st[w], nn[w], lds.wl[w]);
  else if (nn[w] > WAVE_SHORT && nn[w] <= WAVE_MAX)
    sort_list_wave<(WAVE_MAX + 63) / 64>(a, tt[w], st[w], nn[w], lds.wl[w]);
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
  uint64_t *esum;                        // copies per emission partition
  uint32_t *tk[2], *tv[2], *tb[2];       // tile passes ping-pong [capacity]: tile id, splat, depth bits
  uint32_t *tC;                          // tile passes' counts [pass][1 << bits][key partitions]
  uint32_t *dk[2], *dv[2];               // depth passes ping-pong [n]: depth bits, splat
  uint32_t *dC;                          // a depth pass's counts [256][splat partitions]
  uint32_t *oH;                          // large grids' tile order: [bucket][chunk] counts, then offsets
  // zeroed at the start of every call, contiguous:
  uint32_t *ctr;                         // counters
  uint32_t *ttot;                        // tile digit totals [stripe][pass][256]
  uint32_t *dtot;                        // depth digit totals [stripe][pass][256]
  void *zero_begin;
  size_t zero_bytes;
  size_t tstride;                        // partitions per row
  size_t dstride;                        // splat partitions per row of dC
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
  t.esum = (uint64_t *)take(8 * (size_t)ceil_div((int64_t)N, BS));  // per BS splats (culled route), else per EPART
  for (int b = 0; b < 2; ++b) {
    t.tk[b] = (uint32_t *)take(4 * C);
    t.tv[b] = (uint32_t *)take(4 * C);
    t.tb[b] = (uint32_t *)take(4 * C);
  }
  t.tstride = (size_t)ceil_div((int64_t)C, SPART);
  t.tC = (uint32_t *)take(4 * ((size_t)tp.passes << tp.bits) * t.tstride);
  for (int b = 0; b < 2; ++b) {
    t.dk[b] = (uint32_t *)take(4 * N);
    t.dv[b] = (uint32_t *)take(4 * N);
  }
  t.dstride = (size_t)ceil_div((int64_t)N, SPART);
  t.dC = (uint32_t *)take(4 * (size_t)RADIX * t.dstride);
  t.oH = ntiles >= ORD_MULTI_MIN ? (uint32_t *)take(4 * (size_t)RADIX * order_chunks(ntiles)) : nullptr;
  const size_t z0 = o;
  t.ctr = (uint32_t *)take(4 * CTR_SLOTS);
  t.ttot = (uint32_t *)take(4 * (size_t)STRIPES * MAX_TILE_PASSES * RADIX);
  t.dtot = (uint32_t *)take(4 * (size_t)STRIPES * MAX_TILE_PASSES * RADIX);
  t.zero_begin = p ? (void *)(p + z0) : nullptr;
  t.zero_bytes = o - z0;
  if (w) *w = t;
  return o;
}

}  // namespace

size_t binsort_workspace_bytes(int64_t n, int64_t capacity, int32_t num_tiles) {
  return carve(nullptr, n, capacity, num_tiles, nullptr);
}

namespace {
// the longest-first tile order (and the split) from the ranges
void launch_tile_order(const uint32_t *ranges, int64_t ntiles, uint32_t *order, uint32_t *split, const Workspace &w,
                       hipStream_t s) {
  if (ntiles >= ORD_MULTI_MIN && w.oH) {
    const uint32_t G = order_chunks(ntiles);
    hipLaunchKernelGGL(order_hist, dim3(G), dim3(BS), 0, s, ranges, ntiles, w.oH, G);
    hipLaunchKernelGGL(order_offsets, dim3(1), dim3(1024), 0, s, w.oH, (uint32_t)(RADIX * G));
    hipLaunchKernelGGL(order_scatter, dim3(G), dim3(BS), 0, s, ranges, ntiles, (const uint32_t *)w.oH, G, order,
                       split);
  } else {
    hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(ORD_THREADS), 0, s, ranges, ntiles, order, split);
  }
}

// count, scan and scatter of one stable digit pass over the keys of `a`
// (count in device memory), in partitions of BS * IPT items
template <int IPT>
void radix_pass(const Pass &a, int64_t capacity, const uint32_t *tot, int pass, hipStream_t s) {
  const unsigned grid = ceil_div(capacity, BS * IPT);
  hipLaunchKernelGGL(count_pass<IPT>, dim3(grid), dim3(BS), 0, s, a.kin, a.count_dev, 0u, a.shift, a.nbits,
                     (uint32_t *)a.C, a.c_stride);
  hipLaunchKernelGGL(scan_rows<IPT>, dim3(1u << a.nbits), dim3(BS), 0, s, (uint32_t *)a.C, a.c_stride, a.count_dev,
                     0u, tot, pass);
  hipLaunchKernelGGL(scatter_pass<IPT>, dim3(grid), dim3(BS), 0, s, a);
}
}  // namespace

namespace {
hipError_t binsort(int64_t n, const float *depth, const int32_t *rect, const uint32_t *tiles, int grid_w, int grid_h,
                   int64_t capacity, void *ws, uint64_t *keys, uint32_t *vals, uint32_t *ranges, uint32_t *tile_order,
                   int64_t *num_keys, int32_t *overflow, const Cull *cu, hipStream_t s) {
  const int64_t ntiles = (int64_t)grid_w * grid_h;
  Workspace w;
  carve(ws, n, capacity, ntiles, &w);
  const TilePlan tp = tile_plan(ntiles);
  const size_t tpass = ((size_t)1 << tp.bits) * w.tstride;    // one tile pass's counts

  // Long lists (a capacity of PRESORT_MIN_AVG copies per tile or more): the
  // splats are sorted by depth first and their copies emitted in that order,
  // so the stable tile passes leave every tile's list in (depth, splat) order
  // and no per-tile sort runs. Shorter lists: copies in splat-index order,
  // then each tile's list sorted by depth. Both give the same keys and values.
  const bool presort = n > 0 && capacity > 0 && capacity >= PRESORT_MIN_AVG * ntiles;

  // 0. zero totals, counters and ranges; num_keys = overflow = 0 (with step 1 when n > 0)
  const size_t nz16 = w.zero_bytes / 16, nr = 2 * (size_t)ntiles;
  if (n == 0 || presort || cu) {
    const size_t m = nz16 > nr ? nz16 : nr;
    const unsigned grid = (unsigned)(m / BS + 1 < 2048 ? m / BS + 1 : 2048);
    hipLaunchKernelGGL(clear_state, dim3(grid), dim3(BS), 0, s, (uint4 *)w.zero_begin, nz16, ranges, nr, num_keys,
                       overflow);
  }
  const uint32_t *perm = nullptr;
  if (presort) {
    // 0b. stable LSD sort of the splats by depth bits (four 8-bit passes over n)
    const unsigned hgrid = (unsigned)(ceil_div(n, BS * 16) < 1024 ? ceil_div(n, BS * 16) : 1024);
    hipLaunchKernelGGL(depth_hist, dim3(hgrid), dim3(BS), 0, s, depth, (uint32_t)n, w.dtot);
    const unsigned ngrid = ceil_div(n, SPART);
    int dc = 0;
    for (int pass = 0; pass < DEPTH_PASSES; ++pass) {
      const uint32_t *kin = pass == 0 ? reinterpret_cast<const uint32_t *>(depth) : w.dk[dc];
      hipLaunchKernelGGL(count_pass<SIPT>, dim3(ngrid), dim3(BS), 0, s, kin, (const uint32_t *)nullptr,
                         (uint32_t)n, 8 * pass, 8, w.dC, w.dstride);
      hipLaunchKernelGGL(scan_rows<SIPT>, dim3(RADIX), dim3(BS), 0, s, w.dC, w.dstride, (const uint32_t *)nullptr,
                         (uint32_t)n, (const uint32_t *)w.dtot, pass);
      Pass a{};
      a.kin = kin;
      a.vin = pass == 0 ? nullptr : w.dv[dc];  // splat index on the first pass
      a.count = (uint32_t)n;
      a.shift = 8 * pass;
      a.nbits = 8;
      a.C = w.dC;
      a.c_stride = w.dstride;
      a.kout = w.dk[dc ^ 1];
      a.vout = w.dv[dc ^ 1];
      hipLaunchKernelGGL(scatter_pass<SIPT>, dim3(ngrid), dim3(BS), 0, s, a);
      dc ^= 1;
    }
    perm = w.dv[dc];
  }
  if (n > 0) {
    // 1. copies (in splat-index or depth order) with their depth bits, the tile digit totals, K
    const unsigned egrid = ceil_div(n, EPART), cgrid = ceil_div(n, BS);
    if (cu) {
      hipLaunchKernelGGL(cull_count, dim3(cgrid), dim3(BS), 0, s, (uint32_t)n, perm, tiles, rect, *cu, w.esum);
      hipLaunchKernelGGL(sums_scan, dim3(1), dim3(CS_THREADS), 0, s, w.esum, cgrid, (uint64_t)capacity, w.ctr, num_keys,
                         overflow);
    } else {
      hipLaunchKernelGGL(emit_sums, dim3(egrid), dim3(BS), 0, s, (uint32_t)n, tiles, perm, w.esum,
                         presort ? (uint4 *)nullptr : (uint4 *)w.zero_begin, nz16, ranges, nr, num_keys, overflow);
      if (egrid >= EMIT_SCAN_MIN_PARTS)
        hipLaunchKernelGGL(sums_scan, dim3(1), dim3(CS_THREADS), 0, s, w.esum, egrid, (uint64_t)capacity, w.ctr,
                           num_keys, overflow);
    }
    Emit e{};
    e.n = (uint32_t)n;
    e.perm = perm;
    e.tiles = tiles;
    e.esum = w.esum;
    e.rect = rect;
    e.depth = depth;
    e.grid_w = grid_w;
    e.capacity = (uint64_t)capacity;
    e.ctr = w.ctr;
    e.tkey = w.tk[0];
    e.tval = w.tv[0];
    e.tbits = w.tb[0];
    e.tot = w.ttot;
    e.tile_passes = tp.passes;
    e.tile_bits = tp.bits;
    e.num_keys = num_keys;
    e.overflow = overflow;
    e.scanned = !cu && egrid >= EMIT_SCAN_MIN_PARTS;
    e.row_digits = presort;
    if (cu)
      hipLaunchKernelGGL(cull_emit, dim3(cgrid), dim3(BS), 0, s, e, *cu);
    else
      hipLaunchKernelGGL(emit_copies, dim3(egrid), dim3(BS), 0, s, e);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;

  if (capacity > 0 && n > 0) {
    // 2. stable passes over the tile digits (larger partitions for the long
    // lists' route, so each digit leaves a partition in longer runs)
    const uint32_t *count_dev = w.ctr + CTR_KEYS;
    int cur = 0;
    for (int pass = 0; pass < tp.passes; ++pass) {
      Pass a{};
      a.kin = w.tk[cur];
      a.vin = w.tv[cur];
      a.bin = w.tb[cur];
      a.count_dev = count_dev;
      a.shift = tp.bits * pass;
      a.nbits = tp.bits;
      a.C = w.tC + pass * tpass;
      a.c_stride = w.tstride;
      a.kout = w.tk[cur ^ 1];
      a.vout = w.tv[cur ^ 1];
      a.bout = w.tb[cur ^ 1];
      if (presort && pass == tp.passes - 1) {  // already in (tile, depth, splat) order: the outputs
        a.keys_final = keys;
        a.vals_final = vals;
      }
      if (presort || capacity >= LONG_SEG_MIN_AVG * ntiles)
        radix_pass<LONG_SIPT>(a, capacity, w.ttot, pass, s);
      else
        radix_pass<SIPT>(a, capacity, w.ttot, pass, s);
      cur ^= 1;
    }
    // 3. per-tile ranges, longest-first order, then (in index order) each tile's list by depth
    if (presort) {
      hipLaunchKernelGGL(tile_ranges<true>, dim3(ceil_div(capacity, BS * RIPT)), dim3(BS), 0, s, (const void *)keys,
                         count_dev, ntiles, ranges);
      if (tile_order)
        launch_tile_order(ranges, ntiles, tile_order, (uint32_t *)nullptr, w, s);
      return hipGetLastError();
    }
    hipLaunchKernelGGL(tile_ranges<false>, dim3(ceil_div(capacity, BS * RIPT)), dim3(BS), 0, s, (const void *)w.tk[cur],
                       count_dev, ntiles, ranges);
    if (tile_order)
      launch_tile_order(ranges, ntiles, tile_order, w.ctr + CTR_SPLIT, w, s);
    Seg g{};
    g.ranges = ranges;
    g.order = tile_order;
    g.ntiles = ntiles;
    g.bits = w.tb[cur];
    g.vals = w.tv[cur];
    g.sbits = w.tb[cur ^ 1];
    g.svals = w.tv[cur ^ 1];
    g.keys = keys;
    g.vout = vals;
    g.split = tile_order ? w.ctr + CTR_SPLIT : nullptr;
    hipLaunchKernelGGL(segment_sort<SEG_IPT>, dim3((unsigned)ntiles), dim3(BS), 0, s, g);
    return hipGetLastError();
  }
  // nothing emitted (or no room): ranges stay zero
  if (tile_order)
    launch_tile_order(ranges, ntiles, tile_order, (uint32_t *)nullptr, w, s);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_binsort(int64_t n, const float *depth, const int32_t *rect, const uint32_t *tiles, int grid_w,
                          int grid_h, int64_t capacity, void *ws, size_t, uint64_t *keys, uint32_t *vals,
                          uint32_t *ranges, uint32_t *tile_order, int64_t *num_keys, int32_t *overflow,
                          hipStream_t s) {
  return binsort(n, depth, rect, tiles, grid_w, grid_h, capacity, ws, keys, vals, ranges, tile_order, num_keys,
                 overflow, nullptr, s);
}

hipError_t launch_binsort_culled(int64_t n, const float *depth, const int32_t *rect, const uint32_t *tiles,
                                 const float *means2d, const float *conic_opacity, const BlendParams &bp,
                                 int grid_w, int grid_h, int64_t capacity, void *ws, size_t, uint64_t *keys,
                                 uint32_t *vals, uint32_t *ranges, uint32_t *tile_order, int64_t *num_keys,
                                 int32_t *overflow, hipStream_t s) {
  Cull cu{means2d, conic_opacity, bp, {nullptr, nullptr, nullptr}, 0u, 1u, grid_w <= 256};
  {
    // the second ping-pong buffers of the tile passes are free until the
    // first pass: three arrays of `capacity` words for the saved runs
    Workspace w;
    carve(ws, n, capacity, (int64_t)grid_w * grid_h, &w);
    const uint64_t groups = n > 0 ? (uint64_t)ceil_div(n, BS) : 1u;
    const uint64_t per_seg = (groups + 2) / 3;
    const uint64_t rcap = capacity > 0 ? (uint64_t)capacity * (cu.narrow ? 2u : 1u) / per_seg : 0u;
    cu.seg[0] = w.tk[1];
    cu.seg[1] = w.tv[1];
    cu.seg[2] = w.tb[1];
    cu.per_seg = (uint32_t)per_seg;
    cu.rcap = (uint32_t)(rcap < 0xFFFFFFFFull ? rcap : 0xFFFFFFFFull);
  }
  return binsort(n, depth, rect, tiles, grid_w, grid_h, capacity, ws, keys, vals, ranges, tile_order, num_keys,
                 overflow, &cu, s);
}

}  // namespace gs
