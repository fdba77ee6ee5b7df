/*
 * gs.h -- C ABI of libgs, a gfx950 (MI355X) rasterizer for 3D Gaussian
 * Splatting with the truncated exponential kernel g(x) = exp(-x/2) or the
 * ReLU-activated polynomial kernels f_N(x) = max(sum_i c_i x^i, 0), N = 1..3,
 * and the tighter culling radii they allow, after "From ex(p) to poly:
 * Gaussian Splatting with Polynomial Kernels" (Mueller, Winter, Steinberger).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers to caller-owned, contiguous buffers
 *    in the layouts stated below (row-major, float = IEEE binary32). The
 *    library never allocates, frees or retains them.
 *  - Struct arguments (gs_camera, gs_kernel, gs_params) are HOST pointers;
 *    they are read during the call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Entry
 *    points only enqueue work on it and return; results are valid once the
 *    stream reaches them. Nothing synchronises with the host.
 *  - Every argument is checked on the host before any HIP call. A bad argument
 *    returns GS_EINVAL (GS_EUNSUPPORTED for a valid but unsupported setting)
 *    and enqueues nothing. A failed launch returns GS_EHIP. gs_last_error()
 *    describes the last failure on the calling thread.
 *  - Inputs are never written. Outputs are written in full for every splat,
 *    pixel or tile in range, so they need no clearing beforehand.
 *  - Splat and key indices are 32-bit: n < 2^31 splats, key_capacity < 2^32.
 *  - Calls that share buffers must be ordered on one stream by the caller.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GS_OK = 0,
  GS_EINVAL = -1,        /* bad argument, nothing enqueued */
  GS_EUNSUPPORTED = -2,  /* valid but unsupported setting, nothing enqueued */
  GS_ECAPACITY = -3,     /* the call needs more scratch memory than the library holds (gs_bin_sort_noalloc) */
  GS_EHIP = -4           /* a HIP runtime call or launch failed */
} gs_status;

/* Kernel applied to the screen-space quadric Q(v) = (v - mu')^T S'^-1 (v - mu')
 * (Sec. 2, Eq. 1). EXP: g(Q) = exp(-Q/2) (Sec. 3). POLY: f_N(Q) =
 * max(sum_{i<=N} c_i Q^i, 0) (Sec. 3, Eq. 2); for N = 2 the polynomial is used
 * only for Q below its first positive root x_0 and is 0 beyond (Sec. 3.3,
 * Eq. 6), since the fitted parabola rises again. */
typedef enum { GS_KERNEL_EXP = 0, GS_KERNEL_POLY = 1 } gs_kernel_kind;

/* Bounding radius r = k * sqrt(lambda_max(S')) of a projected splat, with
 * lambda_max the larger eigenvalue of its anti-aliased 2D covariance
 * (Sec. 2.1). The multiplier k is
 *   SIGMA3:          3 (the 3DGS square bound, Sec. 2.1);
 *   POLY_UNIVERSAL:  sqrt(x_0), x_0 the first positive root of the polynomial,
 *                    the same for every splat (Sec. 3.2, Eq. 5; App. B with
 *                    eps = 0);
 *   POLY_OPACITY:    sqrt(x_e), x_e the first positive root of
 *                    o' p(x) = eps for the splat's opacity o' (Sec. 3.2, Eq. 4;
 *                    App. B); splats with o' c_0 < eps are culled;
 *   EXP_OPACITY:     sqrt(2 ln(o'/eps)), where o' exp(-x/2) falls to eps
 *                    (Sec. 3.2, Eq. 3); splats with o' < eps are culled.
 * POLY_* modes take the polynomial of the gs_kernel even when kind is EXP:
 * that pairs the exponential with the polynomial's tighter culling, the
 * setting the paper shows to produce blocky artefacts (Sec. 5.2, Fig. 3a). */
typedef enum {
  GS_RADIUS_SIGMA3 = 0,
  GS_RADIUS_POLY_UNIVERSAL = 1,
  GS_RADIUS_POLY_OPACITY = 2,
  GS_RADIUS_EXP_OPACITY = 3
} gs_radius_mode;

/* Tile rectangle of a splat (rect and tiles_touched of gs_preprocess).
 *   SQUARE:      the tiles met by the square of half side r = k sqrt(lambda_max)
 *                around the mean (the bounding square of Sec. 2.1).
 *   ELLIPSE_BOX: the tiles met by the axis-aligned bounding box of the
 *                ellipse Q = k^2, half sides k sqrt(S_a,xx) and k sqrt(S_a,yy)
 *                (times radius_pad), a subset of SQUARE's: the tighter
 *                rectangle of the bounds the paper surveys (Sec. 2.1). With
 *                the POLY_* and EXP_OPACITY radii, k^2 bounds where alpha >= eps,
 *                so images do not change, only the copies that cannot
 *                contribute are dropped. */
typedef enum { GS_RECT_SQUARE = 0, GS_RECT_ELLIPSE_BOX = 1 } gs_rect_mode;

typedef struct {
  int32_t kind;        /* gs_kernel_kind */
  int32_t order;       /* polynomial order N in 1..3 (read for POLY and for POLY_* radii) */
  int32_t radius_mode; /* gs_radius_mode */
  int32_t reserved;    /* must be 0 */
  double coeffs[4];    /* c_0..c_3; entries above `order` are ignored. The polynomial must
                          satisfy c_0 > 0 and decrease on [0, x_0] (true for the paper's
                          fits); otherwise GS_EUNSUPPORTED. */
} gs_kernel;

typedef struct {
  float eps;        /* contribution threshold: alpha < eps is skipped (1/255, Sec. 3.1) */
  float alpha_max;  /* alpha is clamped to this (0.99) */
  float t_min;      /* a pixel stops before the splat that takes T below this (1e-4) */
  float aa_v;       /* anti-aliasing: added to the diagonal of the 2D covariance, px^2 (0.3) */
  float near_z;     /* splats with camera z below this are culled (0.2) */
  float radius_pad; /* r is multiplied by this (>= 1; 1 + 2^-20 keeps rectangles conservative) */
  float bg[3];      /* background colour added as T * bg */
  int32_t tile;     /* tile edge in pixels; only 16 is supported */
  int32_t blend_threads; /* launch shape of the blend: threads per 16x16 tile, 64, 128 or 256
                            (4, 2 or 1 pixels per thread); 0 = the library's default. Results
                            do not depend on it. */
  int32_t rect_mode;     /* gs_rect_mode */
  int32_t blend_stage;   /* records each blend thread stages in LDS per batch, 1 or 2 (a batch holds
                            blend_threads x blend_stage records); 0 = the library's default (2).
                            Results do not depend on it. */
} gs_params;

typedef struct {
  float viewmat[16]; /* world -> camera, row-major 4x4; camera x right, y down, z forward.
                        The rotation block must be orthonormal; the last row is ignored. */
  float fx, fy;      /* focal lengths in pixels */
  float cx, cy;      /* principal point in pixels; pixel (i, j) has its centre at (i+0.5, j+0.5) */
  int32_t width, height; /* image size, 1..32768 each */
} gs_camera;

/* ---------------------------------------------------------------------- */
/* host-only helpers (no HIP calls)                                        */
/* ---------------------------------------------------------------------- */

const char *gs_version(void);

/* Message for the last non-GS_OK status returned on the calling thread. */
const char *gs_last_error(void);

/* Fills `out` with the library's coefficient table for (kind, order,
 * radius_mode). Order 1 uses Sec. 3.1's printed first-order pair (intercept
 * 0.773, root 4.386); orders 2 and 3 use the library's own L1 fit on
 * [0, 2 ln 255] (Sec. 3.1 fitting; Sec. 3.3). */
gs_status gs_kernel_default(int32_t kind, int32_t order, int32_t radius_mode, gs_kernel *out);

/* App. A: the order-2 polynomial kernel fitted (same L1 objective) over
 * [0, x_max], x_max = (sqrt(2) p_t / s_min + sqrt(-2 ln eps))^2 = 1992.8 for
 * 16-px tiles and s_min = sqrt(0.3), the smallest scale the 2-D
 * anti-aliasing leaves: every quadric value a renderer with exact per-tile
 * culling (gs_bin_sort_culled) can evaluate, for splats culled at their eps
 * cut-off. The fit stays monotone over that range, the alternative to the cut
 * at the first root of Eq. 6; on a range this wide it is all but the
 * order-1 line, as App. A expects for 16-px tiles. Fills `out` (kind POLY,
 * order 2, the given radius_mode). */
gs_status gs_kernel_order2_tile_range(int32_t radius_mode, gs_kernel *out);

/* First positive root x_0 of the kernel's polynomial (App. B closed forms:
 * linear, quadratic formula, Cardano), after the checks gs_preprocess makes. */
gs_status gs_kernel_root(const gs_kernel *kernel, double *x0_out);

/* eps 1/255, alpha_max 0.99, t_min 1e-4, aa_v 0.3, near_z 0.2,
 * radius_pad 1 + 2^-20, bg 0, tile 16, blend_threads 0, rect_mode SQUARE, blend_stage 0. */
gs_status gs_params_default(gs_params *out);

/* ---------------------------------------------------------------------- */
/* forward path                                                            */
/* ---------------------------------------------------------------------- */

/* Per-splat projection (Sec. 2 Eq. 1; Sec. 2.1; Sec. 3.2 Eqs. 3-5; Sec. 3.4;
 * App. B). For each splat i < n:
 *   camera-space mean t = W mu + tw; depth[i] = t.z rounded to float;
 *   culled when t.z < near_z;
 *   S = R(q) diag(s)^2 R(q)^T; S' = J W S W^T J^T with J the Jacobian of the
 *   perspective map at t (x/z and y/z clamped to 1.3 tan of the half field of
 *   view); anti-aliasing S_a = S' + aa_v I, o' = o sqrt(|S'| / |S_a|);
 *   conic = S_a^-1; mean2d = (fx t.x/t.z + cx, fy t.y/t.z + cy);
 *   r = k sqrt(lambda_max(S_a)) * radius_pad (k per gs_radius_mode);
 *   half sides (hx, hy) = (r, r) for GS_RECT_SQUARE, else
 *   k (sqrt(S_a,xx), sqrt(S_a,yy)) * radius_pad (gs_rect_mode);
 *   rect = inclusive tile rectangle (x_lo, y_lo, x_hi, y_hi) with
 *   x_lo = clamp(floor((u - hx)/tile), 0, gx), x_hi = clamp(floor((u + hx)/tile), -1, gx - 1)
 *   and likewise in y with hy, stored as (0, 0, -1, -1) when empty;
 *   tiles_touched = tiles in rect;
 *   rgb = max(sum_k Y_k(d) sh_k + 0.5, 0) with real SH of degree sh_degree at
 *   d = normalize(mu - camera centre).
 * Geometry up to the rectangle is computed in double precision, so depth and
 * rectangles are reproducible; the record is rounded to float on output.
 * Culled splats get zero means2d, conic_opacity and rgb, rect (0,0,-1,-1)
 * and tiles_touched 0 (depth is still written).
 *
 * in : means3d [n,3], scales [n,3] (standard deviations), quats [n,4]
 *      (w,x,y,z, need not be normalised), opacities [n] in [0,1],
 *      sh [n,(sh_degree+1)^2,3] (16-byte aligned), sh_degree in 0..3.
 * out: means2d [n,2], conic_opacity [n,4] = (a, b, c, o') with conic
 *      [[a, b], [b, c]], rgb [n,3], depth [n], rect [n,4] int32,
 *      tiles_touched [n] uint32.
 * n = 0 is a valid no-op. */
gs_status gs_preprocess(const gs_camera *cam, const gs_kernel *kernel, const gs_params *params, int64_t n,
                        const float *means3d, const float *scales, const float *quats, const float *opacities,
                        const float *sh, int32_t sh_degree, float *means2d, float *conic_opacity, float *rgb,
                        float *depth, int32_t *rect, uint32_t *tiles_touched, void *stream);

/* Bytes of device workspace gs_bin_sort needs for n splats, a key capacity
 * and a tile count. */
gs_status gs_bin_sort_workspace(int64_t n, int64_t key_capacity, int32_t num_tiles, size_t *bytes);

/* Tile binning (Sec. 2.1; the tile partitioning the paper's CUDA renderers
 * share, Sec. 4.2): every splat is duplicated once per tile of its rect with
 * the 64-bit key (tile_id << 32) | bits(depth) (tile_id = ty * grid_w + tx,
 * rows of the rect in order, depth's float bits, depths being positive for
 * every splat with tiles), the value being the splat index. The key list is
 * sorted stably, so equal keys keep splat-index order and the result is
 * unique; ranges[t] = (first, last + 1) of tile t's keys, (0, 0) if none.
 *
 * in : depth [n], rect [n,4], tiles_touched [n] (gs_preprocess outputs),
 *      grid_w x grid_h tiles, key_capacity = length of keys and vals.
 * out: keys [key_capacity] uint64 and vals [key_capacity] uint32 (first
 *      *num_keys entries valid), ranges [grid_w * grid_h, 2] uint32,
 *      num_keys (device int64) = K, the total number of copies,
 *      overflow (device int32) = 1 when K > key_capacity, else 0. On overflow
 *      keys and vals hold no valid entries and every range is (0, 0); the
 *      caller reads *num_keys and calls again with a larger capacity.
 *      tile_order [grid_w * grid_h] uint32 (may be NULL) = every tile id once,
 *      longest lists first (lists bucketed by length); passed to the blend
 *      entry points it makes the workgroups with the most work start first.
 * workspace: device buffer of at least gs_bin_sort_workspace() bytes,
 *      contents undefined before and after. */
gs_status gs_bin_sort(int64_t n, const float *depth, const int32_t *rect, const uint32_t *tiles_touched,
                      int32_t grid_w, int32_t grid_h, int64_t key_capacity, void *workspace,
                      size_t workspace_bytes, uint64_t *keys, uint32_t *vals, uint32_t *ranges,
                      uint32_t *tile_order, int64_t *num_keys, int32_t *overflow, void *stream);

/* Largest workspace gs_bin_sort_noalloc serves: 128 MiB, enough for 1M splats
 * with a key capacity of 4M at 1920x1080 (gs_bin_sort_workspace gives ~112 MiB). */
#define GS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): gs_bin_sort
 * with its workspace taken from a static device array of
 * GS_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends. Arguments, outputs and errors are those of
 * gs_bin_sort without the workspace; the stream must belong to the current
 * device. Returns GS_ECAPACITY, enqueueing nothing, when
 * gs_bin_sort_workspace(n, key_capacity, grid_w * grid_h) exceeds
 * GS_NOALLOC_SCRATCH_BYTES. Calls no hipMalloc, hipFree or allocating library
 * routine; the first call on a device looks the array's address up once
 * (hipGetSymbolAddress). Every call on one GPU shares that GPU's array, whose
 * contents are undefined between calls (the binning clears what must start
 * at zero itself): calls that may overlap in time on one GPU (other streams,
 * unordered host threads) race and give undefined results. */
gs_status gs_bin_sort_noalloc(int64_t n, const float *depth, const int32_t *rect, const uint32_t *tiles_touched,
                              int32_t grid_w, int32_t grid_h, int64_t key_capacity, uint64_t *keys, uint32_t *vals,
                              uint32_t *ranges, uint32_t *tile_order, int64_t *num_keys, int32_t *overflow,
                              void *stream);

/* Tile binning with per-tile culling (the tile test of StopThePop that the
 * paper adds to every renderer it evaluates, Sec. 2.1 and Sec. 4; App. A
 * looks at the tile bound it gives): as gs_bin_sort, but a splat's copy for
 * a tile of its rect is emitted only when the point of the tile's
 * pixel-centre rectangle [16 tx + 0.5, 16 tx + 15.5] x [16 ty + 0.5,
 * 16 ty + 15.5] where the splat contributes most, the minimum of
 * Q = d^T conic d over that rectangle (d = point - mean2d), has
 * Q <= cut(o, conic), evaluated in double (a minimum within double rounding
 * of cut may be decided either way). cut is the largest Q at which gs_rasterize_fwd can
 * include a pixel of the splat: the double threshold of alpha >= eps for the
 * kernel, widened by bounds on the blend's float rounding (2^-16 (|thr| + 16)
 * on the threshold thr, then 2^-19 times the rounding terms of its
 * tile-local evaluation; the formula is in the implementation). Splats whose
 * conic is not positive definite, or whose opacity reaches eps nowhere, get
 * no copy. Every pixel the blend includes lies in a kept tile, so images,
 * final_T, n_contrib and the blended set are those of gs_bin_sort's lists;
 * the lists hold fewer entries (n_eval and last_contrib count list
 * positions and shrink with them). K counts kept copies, so a key_capacity
 * below the sum of tiles_touched may suffice.
 *
 * in : as gs_bin_sort, plus kernel and params (kernel, eps, tile) and the
 *      projected records means2d [n,2] (8-byte aligned) and conic_opacity
 *      [n,4] (16-byte aligned); grid_w * grid_h < 2^22 and grid_w <= 32767.
 * out, workspace: as gs_bin_sort (the same workspace size). */
gs_status gs_bin_sort_culled(const gs_kernel *kernel, const gs_params *params, int64_t n, const float *depth,
                             const int32_t *rect, const uint32_t *tiles_touched, const float *means2d,
                             const float *conic_opacity, int32_t grid_w, int32_t grid_h, int64_t key_capacity,
                             void *workspace, size_t workspace_bytes, uint64_t *keys, uint32_t *vals,
                             uint32_t *ranges, uint32_t *tile_order, int64_t *num_keys, int32_t *overflow,
                             void *stream);

/* Front-to-back blending per pixel (Sec. 2, Eq. 1 and the alpha compositing
 * it feeds; the kernel of Sec. 3 Eq. 2 / Eq. 6 or exp). For each pixel, over
 * its tile's sorted list: Q = d^T conic d with d = pixel centre - mean2d;
 * alpha = min(alpha_max, o' k(Q)); skipped if alpha < eps; T' = T (1 - alpha);
 * the pixel stops, without blending, at the first splat with T' < t_min;
 * otherwise C += rgb alpha T and T = T'. image = C + T bg.
 *
 * in : means2d, conic_opacity, rgb (gs_preprocess), vals, ranges and
 *      tile_order (gs_bin_sort; tile_order may be NULL for row-major order,
 *      it only changes which workgroup renders which tile), n = number of
 *      splats the values index. A splat whose conic is not positive definite
 *      (a > 0, c > 0, a c > b^2; gs_preprocess culls the others) is never
 *      blended. Q is evaluated in float as c (dy + dx b/c)^2 + dx^2 (ac - b^2)/c,
 *      a sum of two non-negative terms, so its rounding stays a few ulps of Q
 *      however elongated the footprint.
 * out: image [3,H,W] planar, final_T [H,W], n_contrib [H,W] = splats
 *      blended, last_contrib [H,W] = 1 + list position (within the tile)
 *      of the last blended splat, 0 if none (the backward pass starts there),
 *      n_eval [H,W] (may be NULL) = list entries evaluated, including the one
 *      that stopped the pixel. */
gs_status gs_rasterize_fwd(const gs_camera *cam, const gs_kernel *kernel, const gs_params *params, int64_t n,
                           const float *means2d, const float *conic_opacity, const float *rgb,
                           const uint32_t *vals, const uint32_t *ranges, const uint32_t *tile_order, float *image,
                           float *final_T, uint32_t *n_contrib, uint32_t *last_contrib, uint32_t *n_eval,
                           void *stream);

/* gs_rasterize_fwd with the quadric on the matrix cores (Sec. 5.1: Q of a
 * block of pixels against a batch of splats is a matrix product of the
 * pixels' monomials (1, x, y, x^2, x y, y^2) and per-splat coefficient
 * vectors). Each splat's coefficients expand t = x_e - Q about the centre of
 * the 8x8 pixel block a wave shades, computed in double from the float record
 * and rounded once; v_mfma_f32_32x32x2_f32 forms t for 32 splats x 32 pixels.
 * Blending, early termination and the outputs are those of gs_rasterize_fwd
 * (same arguments; blend_threads is ignored: 256 threads per tile), up to
 * rounding: the quadric's rounding differs (a few 1e-5 in t where t is near
 * 0), and each 32-splat step composites its two halves of 16 separately and
 * combines them by the over operator's associativity, so images agree with
 * gs_rasterize_fwd's within float rounding except at inclusion and
 * termination decisions within that rounding of their thresholds. The lists
 * must come from gs_bin_sort (per-tile culling bounds the vector blend's
 * rounding, not this one's). */
gs_status gs_rasterize_fwd_mfma(const gs_camera *cam, const gs_kernel *kernel, const gs_params *params, int64_t n,
                                const float *means2d, const float *conic_opacity, const float *rgb,
                                const uint32_t *vals, const uint32_t *ranges, const uint32_t *tile_order,
                                float *image, float *final_T, uint32_t *n_contrib, uint32_t *last_contrib,
                                uint32_t *n_eval, void *stream);

/* The work gs_rasterize_fwd performs, for measurement: the same blend with
 * the same outputs, plus n_tested [H,W] uint32 = kernel evaluations done for
 * the pixel (list entries its wave did not skip, while the pixel was alive,
 * the entry that stopped it included). The forward skips an entry for a wave
 * when a conservative box around the entry's threshold ellipse (Q <= x_e,
 * the region where alpha >= eps) misses the wave's pixels, so n_tested <=
 * n_eval and n_tested >= n_contrib. Slower than gs_rasterize_fwd (an extra
 * counter in the inner loop); n_eval may be NULL, n_tested may not. */
gs_status gs_rasterize_fwd_count(const gs_camera *cam, const gs_kernel *kernel, const gs_params *params, int64_t n,
                                 const float *means2d, const float *conic_opacity, const float *rgb,
                                 const uint32_t *vals, const uint32_t *ranges, const uint32_t *tile_order,
                                 float *image, float *final_T, uint32_t *n_contrib, uint32_t *last_contrib,
                                 uint32_t *n_eval, uint32_t *n_tested, void *stream);

/* ---------------------------------------------------------------------- */
/* backward path (the derivative of the ReLU-polynomial kernel the paper   */
/* adds to optimise scenes with it, Sec. 4.3)                              */
/* ---------------------------------------------------------------------- */

/* Adjoint of gs_rasterize_fwd. Per pixel, back to front from final_T and
 * last_contrib, recovering T before each splat by division by (1 - alpha)
 * (no per-pair state is stored). Included pairs have alpha >= eps > 0, so a
 * polynomial kernel is on its smooth branch there and the ReLU kink never
 * enters; a clamped alpha (alpha_max) has zero derivative.
 * in : the forward's inputs and outputs, dL_dimage [3,H,W].
 * out: dL_dmeans2d [n,2], dL_dconic_opacity [n,4] (gradient w.r.t. a, b, c
 *      and o' of conic_opacity; b is the off-diagonal entry, counted once),
 *      dL_drgb [n,3]. The outputs are zeroed, then accumulated. */
gs_status gs_rasterize_bwd(const gs_camera *cam, const gs_kernel *kernel, const gs_params *params, int64_t n,
                           const float *means2d, const float *conic_opacity, const float *rgb,
                           const uint32_t *vals, const uint32_t *ranges, const uint32_t *tile_order,
                           const float *final_T, const uint32_t *last_contrib, const float *dL_dimage,
                           float *dL_dmeans2d, float *dL_dconic_opacity, float *dL_drgb, void *stream);

/* Adjoint of gs_preprocess: chains the 2D gradients through the anti-aliasing
 * factor, the conic inverse, EWA, the rotation and scale and the spherical
 * harmonics to the scene parameters. Splats with tiles_touched = 0 get zero
 * gradients. The rectangle is piecewise constant and carries none.
 * in : gs_preprocess's inputs, its tiles_touched output, and the outputs of
 *      gs_rasterize_bwd.
 * out: dL_dmeans3d [n,3], dL_dscales [n,3], dL_dquats [n,4] (w.r.t. the
 *      unnormalised input), dL_dopacities [n], dL_dsh [n,(d+1)^2,3];
 *      every entry is written. */
gs_status gs_preprocess_bwd(const gs_camera *cam, const gs_kernel *kernel, const gs_params *params, int64_t n,
                            const float *means3d, const float *scales, const float *quats,
                            const float *opacities, const float *sh, int32_t sh_degree,
                            const uint32_t *tiles_touched, const float *dL_dmeans2d,
                            const float *dL_dconic_opacity, const float *dL_drgb, float *dL_dmeans3d,
                            float *dL_dscales, float *dL_dquats, float *dL_dopacities, float *dL_dsh,
                            void *stream);

/* ---------------------------------------------------------------------- */
/* batched rendering: many (scene, view) pairs in one graph-capturable     */
/* frame                                                                   */
/* ---------------------------------------------------------------------- */

/* A scene: n splats in the layouts gs_preprocess takes (device pointers). */
typedef struct {
  int64_t n;
  const float *means3d, *scales, *quats, *opacities, *sh;
  int32_t sh_degree;  /* must be the same for every scene of a batch */
  int32_t reserved;   /* must be 0 */
} gs_scene;

/* A view: which scene it renders, with which camera, and where its outputs
 * go: image [3,H,W] at images + image_offset, and the [H,W] planes at
 * final_T / n_contrib / last_contrib + pixel_offset (element offsets). */
typedef struct {
  gs_camera cam;
  int32_t scene;
  int32_t reserved;   /* must be 0 */
  int64_t image_offset;
  int64_t pixel_offset;
} gs_view;

/* Sizes of a batch: num_pairs (scene splats per view, each view padded to a
 * multiple of 64), the virtual tile grid (width = widest view's tile columns,
 * height = all views' tile rows stacked) and the workspace bytes
 * gs_render_batched needs for the given key capacity. Host only. */
gs_status gs_batch_layout(const gs_scene *scenes, int32_t num_scenes, const gs_view *views, int32_t num_views,
                          int64_t key_capacity, int64_t *num_pairs, int32_t *grid_w, int32_t *grid_h,
                          size_t *workspace_bytes);

/* Renders every view of `views` (host copy, validated here) with one batched
 * projection, one binning and sort of all views' keys in a shared virtual tile
 * grid (the keys of Sec. 2.1's tile partitioning with view tile rows stacked),
 * and one persistent blend launch whose workgroups take tiles from a device
 * queue. `views_device` must hold the same table in device memory: kernels
 * read it there, so the call enqueues kernels only (no host copies, no
 * allocation, no memset) and can be captured in a graph and replayed; a device
 * entry that fails the host's bounds checks, or whose pairs would not fit the
 * num_pairs slots sized from the host table, renders nothing. Outputs equal
 * gs_rasterize_fwd's for each view bit for bit. workgroups: persistent blend
 * workgroups (0 = library default). images_len / planes_len: lengths (in
 * elements) of the output buffers, checked against every view's range.
 * num_keys / overflow as in gs_bin_sort (on overflow nothing is blended).
 * view_keys (device int64 [num_views], may be NULL): the keys of each view,
 * i.e. the copies its splats made in its own tile grid (0 for every view on
 * overflow); they sum to *num_keys. */
gs_status gs_render_batched(const gs_kernel *kernel, const gs_params *params, const gs_scene *scenes,
                            int32_t num_scenes, const gs_view *views, const gs_view *views_device,
                            int32_t num_views, int64_t key_capacity, int32_t workgroups, void *workspace,
                            size_t workspace_bytes, float *images, int64_t images_len, float *final_T,
                            uint32_t *n_contrib, uint32_t *last_contrib, int64_t planes_len, int64_t *num_keys,
                            int32_t *overflow, int64_t *view_keys, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
