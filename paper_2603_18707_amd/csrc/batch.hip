// Batched rendering of many (scene, view) pairs with one sort and one
// persistent blend launch, every kernel enqueued without a host round trip so
// the whole frame can be captured once in a graph and replayed.
//
// Layout. View v renders scene s(v) (N splats) at W x H with a gx x gy tile
// grid. Its splats occupy the pair range [pair_off(v), pair_off(v) + N) of one
// concatenated record array (ranges padded to 64 so a preprocess workgroup
// never straddles two views). The views' tile grids are stacked vertically in
// one virtual grid of width max gx: view v's tile row ty is virtual row
// row_base(v) + ty. A rectangle stays a rectangle there, so the single-view
// binning (duplication, stable radix sort of (tile << 32 | depth), ranges)
// runs unchanged over all pairs, and inside every virtual tile the list is
// ordered by (depth, splat index) exactly as a per-view render orders it:
// batched images are bit-identical to per-view ones.
//
// The blend is persistent: a fixed number of workgroups take virtual tiles
// from an atomic counter until none is left (every workgroup reaches the end
// of the queue, so the grid always drains), in longest-list-first order over
// all views, blending each with the same tile code as gs_rasterize_fwd into
// that view's output planes.
#include <cstring>

#include "blend_common.h"
#include "gs_internal.h"
#include "project_common.h"

namespace gs {

namespace {

constexpr int MAX_SCENES = 16;

struct SceneTable {
  int64_t n[MAX_SCENES];
  const float *means3d[MAX_SCENES], *scales[MAX_SCENES], *quats[MAX_SCENES], *opac[MAX_SCENES],
      *sh[MAX_SCENES];
};

// per-view derived layout, written on the device from the caller's view table
struct ViewInfo {
  int64_t pair_off, block_off, n, image_offset, pixel_offset;
  int32_t row_base, gx, gy, W, H, scene;
};

// The projection's work order: per scene, its views' 64-splat blocks in
// groups, so that the views of a scene project the same block back to back on
// one XCD (workgroup x runs on XCD x mod 8) and all but the first read the
// splat's 236 bytes from that XCD's L2. Item j of scene s (from base) is
// block (j / 8 / nv) * 8 + j % 8 of the scene's view sview[off + (j / 8) % nv];
// a scene takes ceil(blocks / 8) * 8 * nv items.
struct SceneWork {
  int64_t base;
  int32_t nv, off;
};

// Derives the per-view layout from the view table on the device. Views whose
// entry fails the same bounds checks the host applied to its own copy (scene
// index, image size, output ranges) are dropped: they get no pairs and no
// tiles, so nothing is ever read or written out of range even if the device
// table differs from the validated host table.
__global__ void batch_setup(const gs_view *__restrict__ views, int nviews, SceneTable st, int nscenes, int tile,
                            int gh, int64_t pairs, int64_t images_len, int64_t planes_len, ViewInfo *__restrict__ info,
                            SceneWork *__restrict__ swork, int32_t *__restrict__ sview,
                            uint32_t *__restrict__ row_view, uint32_t *__restrict__ counter) {
  for (int r = threadIdx.x; r < gh; r += blockDim.x) row_view[r] = (uint32_t)nviews;  // sentinel: no view
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t blocks = 0;
    int32_t rows = 0;
    for (int v = 0; v < nviews; ++v) {
      const gs_view &w = views[v];
      const int64_t W = w.cam.width, H = w.cam.height;
      const bool ok = w.scene >= 0 && w.scene < nscenes && W >= 1 && H >= 1 && W <= 32768 && H <= 32768 &&
                      w.image_offset >= 0 && w.pixel_offset >= 0 && w.image_offset + 3 * W * H <= images_len &&
                      w.pixel_offset + W * H <= planes_len &&
                      (blocks + (st.n[w.scene] + 63) / 64) * 64 <= pairs;  // the pair arrays hold its range
      ViewInfo in;
      in.scene = ok ? w.scene : 0;
      in.n = ok ? st.n[w.scene] : 0;
      in.block_off = blocks;
      in.pair_off = blocks * 64;
      in.row_base = rows;
      in.W = ok ? (int32_t)W : 0;
      in.H = ok ? (int32_t)H : 0;
      in.gx = ok ? (int32_t)((W + tile - 1) / tile) : 0;
      in.gy = ok ? (int32_t)((H + tile - 1) / tile) : 0;
      in.image_offset = ok ? w.image_offset : 0;
      in.pixel_offset = ok ? w.pixel_offset : 0;
      info[v] = in;
      blocks += (in.n + 63) / 64;
      rows += in.gy;
    }
    ViewInfo end;
    end.scene = 0;
    end.n = 0;
    end.block_off = blocks;
    end.pair_off = blocks * 64;
    end.row_base = rows;
    end.W = end.H = end.gx = end.gy = 0;
    end.image_offset = end.pixel_offset = 0;
    info[nviews] = end;
    *counter = 0u;
    // the projection's work order (SceneWork): the views with pairs, grouped
    // by scene in view order (a counting sort over the scenes)
    int32_t nv[MAX_SCENES], at[MAX_SCENES];
    for (int sc = 0; sc < MAX_SCENES; ++sc) nv[sc] = 0;
    for (int v = 0; v < nviews; ++v)
      if (info[v].n > 0) ++nv[info[v].scene];
    int64_t base = 0;
    int32_t off = 0;
    for (int sc = 0; sc < nscenes; ++sc) {
      swork[sc].base = base;
      swork[sc].nv = nv[sc];
      swork[sc].off = off;
      at[sc] = off;
      base += nv[sc] > 0 ? (st.n[sc] + 511) / 512 * 8 * nv[sc] : 0;
      off += nv[sc];
    }
    swork[nscenes].base = base;
    swork[nscenes].nv = 0;
    swork[nscenes].off = off;
    for (int v = 0; v < nviews; ++v)
      if (info[v].n > 0) sview[at[info[v].scene]++] = v;
  }
  __syncthreads();
  // virtual tile row -> view
  for (int v = 0; v < nviews; ++v) {
    const int32_t r0 = info[v].row_base, r1 = info[v + 1].row_base;
    for (int32_t r = r0 + threadIdx.x; r < r1 && r < gh; r += blockDim.x) row_view[r] = (uint32_t)v;
  }
}

// One workgroup per work item (SceneWork); the grid may hold spare items,
// which return.
template <int DEG>
__global__ __launch_bounds__(64) void batch_preprocess(PreParams base, SceneTable st, const gs_view *__restrict__ views,
                                                       const ViewInfo *__restrict__ info,
                                                       const SceneWork *__restrict__ swork,
                                                       const int32_t *__restrict__ sview, int nscenes, PreOut out) {
  const int64_t x = blockIdx.x;
  int s = 0;
  while (s < nscenes && swork[s + 1].base <= x) ++s;
  if (s >= nscenes) return;
  const SceneWork sw = swork[s];
  const int64_t j = x - sw.base, y = j >> 3;
  const int v = sview[sw.off + (int32_t)(y % sw.nv)];
  const int64_t blk = y / sw.nv * 8 + (j & 7);
  const ViewInfo in = info[v];
  if (blk * 64 >= in.n) return;  // past the view's last block
  const int64_t i = blk * 64 + threadIdx.x;
  const int64_t o = in.pair_off + i;
  float Y[16];
  bool live = false;
  if (i < in.n) {
    PreParams p = base;
    const gs_camera cam = views[v].cam;
    make_cam(&cam, base.tile, &p.cam);
    live = project_one<DEG>(p, i, st.means3d[s], st.scales[s], st.quats[s], st.opac[s], o, in.row_base, out, Y);
  } else {  // padding pair: culled
    out.depth[o] = 0.0f;
    reinterpret_cast<float2 *>(out.means2d)[o] = make_float2(0.f, 0.f);
    reinterpret_cast<float4 *>(out.conic_opacity)[o] = make_float4(0.f, 0.f, 0.f, 0.f);
    reinterpret_cast<int4 *>(out.rect)[o] = make_int4(0, 0, -1, -1);
    out.tiles[o] = 0u;
  }
  const float3 c = sh_colour<DEG>(st.sh[s], i, live, Y);
  out.rgb[3 * o] = c.x;
  out.rgb[3 * o + 1] = c.y;
  out.rgb[3 * o + 2] = c.z;
}

template <int KIND, int NT, int SB>
__global__ __launch_bounds__(NT) void batch_blend(BlendParams base, const ViewInfo *__restrict__ info,
                                                  const uint32_t *__restrict__ row_view, int grid_w,
                                                  uint32_t nitems, const uint32_t *__restrict__ ranges,
                                                  const uint32_t *__restrict__ order,
                                                  const float *__restrict__ means2d,
                                                  const float *__restrict__ conic_opacity,
                                                  const float *__restrict__ rgb, const uint32_t *__restrict__ vals,
                                                  float *images, float *final_T, uint32_t *n_contrib,
                                                  uint32_t *last_contrib, uint32_t *counter) {
  __shared__ uint32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t item = s_item;
    __syncthreads();
    if (item >= nitems) break;  // the queue is empty: every workgroup ends here
    const uint32_t tile = min(order[item], nitems - 1u);  // longest lists first
    const uint32_t vrow = tile / (uint32_t)grid_w, tx = tile % (uint32_t)grid_w;
    const int v = (int)row_view[vrow];
    const ViewInfo in = info[v];
    if ((int)tx >= in.gx) continue;  // virtual tile outside this view's grid
    BlendParams p = base;
    p.W = in.W;
    p.H = in.H;
    p.gx = in.gx;
    p.gy = in.gy;
    const BlendOut out{images + in.image_offset, final_T + in.pixel_offset, n_contrib + in.pixel_offset,
                       last_contrib + in.pixel_offset, nullptr, nullptr};
    blend_tile<KIND, NT, false, SB>(p, (int)tx, (int)vrow - in.row_base, ranges[2 * (size_t)tile], ranges[2 * (size_t)tile + 1],
                         means2d, conic_opacity, rgb, vals, out);
  }
}

// Keys of each view: the copies in the view's block of virtual tiles (rows
// row_base .. row_base + gy - 1, columns 0 .. gx - 1), summed from the tile
// ranges. One workgroup per view.
__global__ __launch_bounds__(256) void batch_view_keys(const ViewInfo *__restrict__ info, int grid_w,
                                                       const uint32_t *__restrict__ ranges,
                                                       int64_t *__restrict__ view_keys) {
  __shared__ uint64_t part[256 / 64];
  const ViewInfo in = info[blockIdx.x];
  const int64_t ntile = (int64_t)in.gx * in.gy;
  uint64_t sum = 0;
  for (int64_t i = threadIdx.x; i < ntile; i += blockDim.x) {
    const size_t t = (size_t)(in.row_base + i / in.gx) * (size_t)grid_w + (size_t)(i % in.gx);
    sum += ranges[2 * t + 1] - ranges[2 * t];
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) view_keys[blockIdx.x] = (int64_t)(part[0] + part[1] + part[2] + part[3]);
}

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchWs {
  ViewInfo *info;
  SceneWork *swork;
  int32_t *sview;
  uint32_t *row_view;
  float *means2d, *conic_opacity, *rgb, *depth;
  int32_t *rect;
  uint32_t *tiles;
  uint64_t *keys;
  uint32_t *vals, *ranges, *order, *counter;
  void *sort_ws;
  size_t sort_bytes;
};

size_t carve_batch(void *base, int nviews, int64_t pairs, int gw, int gh, int64_t cap, BatchWs *w) {
  char *p = (char *)base;
  size_t o = 0;
  auto take = [&](size_t bytes) -> void * {
    void *r = p ? (void *)(p + o) : nullptr;
    o += align_up(bytes);
    return r;
  };
  BatchWs t;
  const size_t P = (size_t)(pairs > 0 ? pairs : 1);
  t.info = (ViewInfo *)take(sizeof(ViewInfo) * (nviews + 1));
  t.swork = (SceneWork *)take(sizeof(SceneWork) * (MAX_SCENES + 1));
  t.sview = (int32_t *)take(4 * (size_t)(nviews > 0 ? nviews : 1));
  t.row_view = (uint32_t *)take(4 * (size_t)gh);
  t.means2d = (float *)take(8 * P);
  t.conic_opacity = (float *)take(16 * P);
  t.rgb = (float *)take(12 * P);
  t.depth = (float *)take(4 * P);
  t.rect = (int32_t *)take(16 * P);
  t.tiles = (uint32_t *)take(4 * P);
  t.keys = (uint64_t *)take(8 * (size_t)(cap > 0 ? cap : 1));
  t.vals = (uint32_t *)take(4 * (size_t)(cap > 0 ? cap : 1));
  t.ranges = (uint32_t *)take(8 * (size_t)gw * gh);
  t.order = (uint32_t *)take(4 * (size_t)gw * gh);
  t.counter = (uint32_t *)take(256);
  t.sort_bytes = binsort_workspace_bytes(pairs, cap, gw * gh);
  t.sort_ws = take(t.sort_bytes);
  if (w) *w = t;
  return o;
}

template <int KIND, int SB>
void launch_batch_blend_stage(int nt, unsigned wgs, const BlendParams &b, const BatchWs &w, int gw, uint32_t nitems,
                              float *images, float *final_T, uint32_t *n_contrib, uint32_t *last_contrib,
                              hipStream_t s) {
  if (nt == 64)
    hipLaunchKernelGGL((batch_blend<KIND, 64, SB>), dim3(wgs), dim3(64), 0, s, b, w.info, w.row_view, gw, nitems,
                       w.ranges, w.order, w.means2d, w.conic_opacity, w.rgb, w.vals, images, final_T, n_contrib,
                       last_contrib, w.counter);
  else if (nt == 128)
    hipLaunchKernelGGL((batch_blend<KIND, 128, SB>), dim3(wgs), dim3(128), 0, s, b, w.info, w.row_view, gw, nitems,
                       w.ranges, w.order, w.means2d, w.conic_opacity, w.rgb, w.vals, images, final_T, n_contrib,
                       last_contrib, w.counter);
  else
    hipLaunchKernelGGL((batch_blend<KIND, 256, SB>), dim3(wgs), dim3(256), 0, s, b, w.info, w.row_view, gw, nitems,
                       w.ranges, w.order, w.means2d, w.conic_opacity, w.rgb, w.vals, images, final_T, n_contrib,
                       last_contrib, w.counter);
}

template <int KIND>
void launch_batch_blend(int nt, unsigned wgs, const BlendParams &b, const BatchWs &w, int gw, uint32_t nitems,
                        float *images, float *final_T, uint32_t *n_contrib, uint32_t *last_contrib, hipStream_t s) {
  if (b.stage == 1)
    launch_batch_blend_stage<KIND, 1>(nt, wgs, b, w, gw, nitems, images, final_T, n_contrib, last_contrib, s);
  else
    launch_batch_blend_stage<KIND, 2>(nt, wgs, b, w, gw, nitems, images, final_T, n_contrib, last_contrib, s);
}

}  // namespace

size_t batch_workspace_bytes(int nviews, int64_t pairs, int gw, int gh, int64_t capacity) {
  return carve_batch(nullptr, nviews, pairs, gw, gh, capacity, nullptr);
}

hipError_t launch_batch(const PreParams &pre, const BlendParams &blend, const gs_scene *scenes, int nscenes,
                        const gs_view *views_dev, int nviews, int64_t pairs, int gw, int gh, int64_t capacity,
                        int workgroups, void *ws, float *images, int64_t images_len, float *final_T,
                        uint32_t *n_contrib, uint32_t *last_contrib, int64_t planes_len, int64_t *num_keys,
                        int32_t *overflow, int64_t *view_keys, hipStream_t s) {
  BatchWs w;
  carve_batch(ws, nviews, pairs, gw, gh, capacity, &w);
  SceneTable st;
  std::memset(&st, 0, sizeof(st));
  for (int i = 0; i < nscenes; ++i) {
    st.n[i] = scenes[i].n;
    st.means3d[i] = scenes[i].means3d;
    st.scales[i] = scenes[i].scales;
    st.quats[i] = scenes[i].quats;
    st.opac[i] = scenes[i].opacities;
    st.sh[i] = scenes[i].sh;
  }
  hipLaunchKernelGGL(batch_setup, dim3(1), dim3(256), 0, s, views_dev, nviews, st, nscenes, pre.tile, gh, pairs,
                     images_len, planes_len, w.info, w.swork, w.sview, w.row_view, w.counter);
  PreOut out{w.means2d, w.conic_opacity, w.rgb, w.depth, w.rect, w.tiles};
  // the work items: pairs / 64 blocks plus at most 7 spare per view (a
  // scene's block count rounded up to a multiple of 8 for each of its views)
  const unsigned items = pairs > 0 ? (unsigned)(pairs / 64 + 7 * (int64_t)nviews) : 0u;
  if (items > 0) {
    switch (pre.sh_degree) {
      case 0:
        hipLaunchKernelGGL(batch_preprocess<0>, dim3(items), dim3(64), 0, s, pre, st, views_dev, w.info, w.swork,
                           w.sview, nscenes, out);
        break;
      case 1:
        hipLaunchKernelGGL(batch_preprocess<1>, dim3(items), dim3(64), 0, s, pre, st, views_dev, w.info, w.swork,
                           w.sview, nscenes, out);
        break;
      case 2:
        hipLaunchKernelGGL(batch_preprocess<2>, dim3(items), dim3(64), 0, s, pre, st, views_dev, w.info, w.swork,
                           w.sview, nscenes, out);
        break;
      default:
        hipLaunchKernelGGL(batch_preprocess<3>, dim3(items), dim3(64), 0, s, pre, st, views_dev, w.info, w.swork,
                           w.sview, nscenes, out);
        break;
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_binsort(pairs, w.depth, w.rect, w.tiles, gw, gh, capacity, w.sort_ws, w.sort_bytes, w.keys, w.vals,
                     w.ranges, w.order, num_keys, overflow, s);
  if (e != hipSuccess) return e;
  if (view_keys && nviews > 0)
    hipLaunchKernelGGL(batch_view_keys, dim3(nviews), dim3(256), 0, s, w.info, gw, w.ranges, view_keys);
  const uint32_t nitems = (uint32_t)((int64_t)gw * gh);
  const unsigned wgs = (unsigned)(workgroups > 0 ? workgroups : 2048);
  switch (blend.blend) {
    case BLEND_EXP:
      launch_batch_blend<BLEND_EXP>(blend.threads, wgs, blend, w, gw, nitems, images, final_T, n_contrib,
                                    last_contrib, s);
      break;
    case BLEND_POLY1:
      launch_batch_blend<BLEND_POLY1>(blend.threads, wgs, blend, w, gw, nitems, images, final_T, n_contrib,
                                      last_contrib, s);
      break;
    case BLEND_POLY2:
      launch_batch_blend<BLEND_POLY2>(blend.threads, wgs, blend, w, gw, nitems, images, final_T, n_contrib,
                                      last_contrib, s);
      break;
    default:
      launch_batch_blend<BLEND_POLY3>(blend.threads, wgs, blend, w, gw, nitems, images, final_T, n_contrib,
                                      last_contrib, s);
      break;
  }
  return hipGetLastError();
}

}  // namespace gs
