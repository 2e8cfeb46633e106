/*
 * tilegs.h -- C ABI of the MI355X (gfx950) tile-local depth-binned 3D Gaussian
 * splatting rasterizer.
 *
 * The library implements the forward path of "TileGS: Tile-Local Depth
 * Binning for Gaussian Splatting Rasterization" and the globally sorted
 * comparator it is measured against:
 *
 *   tgs_project    3DGS projection + spherical-harmonic colour (the paper keeps
 *                  the baseline projection unchanged; method section,
 *                  "Baseline 3DGS rasterization").
 *   tgs_bin        GLOBAL: one (tile, depth) key per Gaussian-tile entry and a
 *                  device radix sort (the baseline's globally sorted stream);
 *                  BINNED: robust depth range (supplement, Algorithm
 *                  "Robust depth-range estimation"), tile-local log-depth bins
 *                  by count / exclusive scan / scatter (Algorithm "Tile-local
 *                  bin construction") and exact repair of the (tile, bin)
 *                  segments (section "Repair for correctness", Algorithm
 *                  "Selective repair selection and local exact sorting").
 *   tgs_rasterize  front-to-back alpha compositing of each tile's one
 *                  contiguous range (Algorithm "Binned raster traversal after
 *                  repair").
 *   tgs_rasterize_backward, tgs_project_backward
 *                  the gradient of a loss of the image with respect to the
 *                  splats and then to the Gaussian parameters. The paper
 *                  names training as future work (Conclusion); these are the
 *                  derivatives of the forward model above over the same
 *                  entry streams.
 *
 * Conventions
 *  - Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *    tensors); everything else is host memory. The caller owns every buffer,
 *    including the workspace; the library never allocates or frees device
 *    memory. Workspaces must be 256-byte aligned (hipMalloc and torch
 *    allocations are); another start address fails with TGS_ERR_WORKSPACE.
 *  - Every call enqueues on `stream` (a hipStream_t, NULL = default stream)
 *    and returns without waiting, except tgs_bin with a non-NULL
 *    num_entries_host, which waits for the entry count (both orders).
 *  - Arguments are validated on the host before anything is launched; on an
 *    error nothing is enqueued and outputs are untouched. tgs_last_error()
 *    returns a message for the last failing call on the calling thread.
 *  - Per-Gaussian invalid data (non-finite values, a zero quaternion, depth
 *    outside (znear, zfar), a singular screen covariance, opacity < 1/255) is
 *    not an error: that Gaussian is invisible (empty rect).
 *  - Limits: 0 <= n < 2^31, sh_degree 0..3, width and height 1..16384,
 *    tile_size 8, 16 or 32 (8 and 32 with the WAVE raster and packed = 0),
 *    1 <= num_bins <= 1024, 0 < znear < zfar, entries < 2^32.
 */
#ifndef TILEGS_H
#define TILEGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TGS_API __attribute__((visibility("default")))

/* Most cameras (views) of one batched call. */
#define TGS_MAX_VIEWS 16

typedef enum {
    TGS_OK = 0,
    TGS_ERR_INVALID_ARG = 1,
    TGS_ERR_CAPACITY = 2,    /* more entries than the binned buffers hold */
    TGS_ERR_HIP = 3,         /* a HIP runtime call or launch failed */
    TGS_ERR_UNSUPPORTED = 4, /* a valid but unimplemented option */
    TGS_ERR_WORKSPACE = 5    /* workspace missing, smaller than required or misaligned */
} tgs_status;

/* Orders of the entry stream. */
enum { TGS_ORDER_GLOBAL = 0, TGS_ORDER_BINNED = 1 };
/* Raster kernels. PLAIN: one 256-lane workgroup per tile walks shared
   batches gathered by Gaussian id (the baseline's kernel structure). WAVE:
   each 64-lane wavefront owns an 8x8 pixel block, streams the tile's range,
   drops entries that provably cannot reach alpha 1/255 anywhere in its block
   and exits on its own. Both produce bit-identical images. */
enum { TGS_RASTER_PLAIN = 0, TGS_RASTER_WAVE = 1 };

/* Repair of the (tile, bin) segments of the BINNED order (section "Repair
   for correctness"). ALL: every segment of two or more entries is sorted by
   its (depth bits, id) pairs, which with near_shift = 0 makes the stream
   equal to the globally sorted one, tile by tile. RULES: the paper's
   selective repair (Table "Exact-repair selection rules" and the
   supplement's Algorithm "Selective repair selection and local exact
   sorting"): a segment of length l >= 2 is kept when l >= 320, l > 512,
   100 l >= 45 l_tile, 129 <= l <= 256 and 100 l >= 10 l_tile, or bin < 2
   and l >= 16 (l_tile: the entries of its tile); kept segments are taken in
   (tile, bin) order while the taken entries stay within floor(repair_budget
   M) (first fit) and only those are sorted. NONE: no segment is sorted.
   With RULES and NONE, the entries of an unsorted segment keep the order of
   the parallel scatter, which varies from call to call. */
enum { TGS_REPAIR_ALL = 0, TGS_REPAIR_RULES = 1, TGS_REPAIR_NONE = 2 };

/* Footprint: the tile rect tgs_project writes for a Gaussian.
   OPACITY_AWARE: the tiles meeting the bounding box of the ellipse where
   o exp(-q/2) >= 1/255 (q <= 2 ln(255 o)), widened by a relative 1e-4 and
   1e-3 px; Gaussians with opacity < 1/255 are invisible. A superset of the
   alpha support, so images do not depend on the tile size or the bins.
   THREE_SIGMA: the rule of the baseline rasterizer the paper compares
   against (section "Baseline 3DGS rasterization"): the tiles meeting the
   square of half side ceil(3 sqrt(lambda_max)) px around the mean,
   lambda_max = mid + sqrt(max(0.1, mid^2 - det)) of the screen covariance
   (mid = its mean diagonal), no opacity cut. The alpha support is cut at
   those tiles, so images depend on the tile size. */
enum { TGS_FOOTPRINT_OPACITY_AWARE = 0, TGS_FOOTPRINT_THREE_SIGMA = 1 };

/* Pinhole camera, host struct. p_cam = R p_world + t, R row-major, image x
   right, y down, z forward; pixel (i, j) is sampled at (i + 0.5, j + 0.5). */
typedef struct {
    double R[9];
    double t[3];
    double fx, fy, cx, cy;
    int32_t width, height;
    double znear, zfar;
} tgs_camera;

/* Gaussians, device pointers, fp32:
   means [n][3]; log_scales [n][3]; quats [n][4] as (w, x, y, z), need not be
   normalised; logits [n] (opacity = sigmoid(logit)); sh [n][(D+1)^2][3] real
   SH coefficients in the order l*l + l + m, m = -l..l. */
typedef struct {
    const float* means_dev;
    const float* log_scales_dev;
    const float* quats_dev;
    const float* logits_dev;
    const float* sh_dev;
    int64_t n;
    int32_t sh_degree;
} tgs_gaussians;

/* Projected Gaussians, device pointers (written by tgs_project, read by
   tgs_bin and tgs_rasterize; callers may also fill them directly):
   splats [n][16] fp32 (one 64-byte line per Gaussian): mean_x, mean_y
       (binary32 rounding of the pixel-space mean), mean_x_lo, mean_y_lo (the
       remainders, so hi + lo is the mean to about 1e-11 px), conic_a,
       conic_b, conic_c (inverse screen covariance, q = a dx^2 + 2 b dx dy +
       c dy^2), opacity, r, g, b, s_max (the largest axis scale
       exp(log_scale), world units; read by tgs_bin with near_shift = 1),
       then four zero words.
   info [n][4] uint32: depth (binary32 bits of the camera-space z, the
       ordering key), x0 | y0 << 16, x1 | y1 << 16 (half-open tile rect),
       number of tiles (x1 - x0) * (y1 - y0); an empty rect = invisible. */
typedef struct {
    float* splats_dev;
    uint32_t* info_dev;
    int64_t n;
} tgs_projected;

/* Ordering and raster options (tgs_default_params fills the paper's values). */
typedef struct {
    int32_t tile_size;    /* tile edge in pixels: 16; 8 and 32 with the WAVE
                             raster and packed = 0 */
    int32_t num_bins;     /* K, 64 (with per_tile_bins_dev: the upper bound of
                             the per-tile counts, a power of two) */
    int32_t sample_count; /* depth-range samples, 8192 */
    float p_lo, p_hi;     /* depth-range percentiles, 1 and 99 */
    float pad;            /* depth-range padding fraction, 0.05 */
    int32_t raster;       /* TGS_RASTER_* */
    int32_t packed;       /* BINNED order only. 0: the WAVE raster gathers each
                             entry's splat by id and tests it against its
                             block; 1: tgs_bin also writes per-entry staged
                             records and block masks, the raster reads the
                             records of the entries its block's mask keeps;
                             2: block masks only, the raster gathers the kept
                             entries by id */
    const int32_t* per_tile_bins_dev; /* NULL: num_bins bins in every tile.
                             Otherwise (BINNED, packed = 0) device int32 [T]:
                             the bin count of each tile, clamped to
                             1..num_bins and rounded down to a power of two;
                             tile t's segments are numbered from seg_base[t],
                             the prefix sum of the counts. The bin map of a
                             tile with K_t bins is the paper's log-depth map
                             with K_t in place of K; images are unchanged. */
    int32_t repair;       /* BINNED: TGS_REPAIR_*, ALL by default; RULES and
                             NONE need packed = 0, RULES also a uniform K */
    float repair_budget;  /* RULES: the entry budget as a fraction of M,
                             0.25; 0..1 */
    int32_t near_shift;   /* BINNED: 0 (default) bins the depth z; 1 bins the
                             near-depth key z - min(alpha s_max, gamma z),
                             clamped to [max(znear, 1e-4), zfar], for both the
                             depth range and the bin map (supplement,
                             Algorithm "Robust depth-range estimation", and
                             the paragraph after the log-depth bin map); the
                             pairs keep the depth bits */
    float shift_alpha;    /* alpha >= 0, 1.0 */
    float shift_gamma;    /* gamma in [0, 1), 0.25 */
    int32_t split_entries; /* 0, or a power of two in 256..2^24 (2048): with
                             the WAVE raster, 16-pixel tiles, packed = 0 and
                             a tile order, the tiles with at least this many
                             entries and split_mean_factor x the mean of the
                             non-empty tiles (the threshold raised by powers
                             of two to at most 1024 tiles) get 4 wavefronts
                             per 8x8 block, one per 4x4 quarter, with four
                             lanes per pixel taking four entries per step
                             through the same per-pixel arithmetic: images,
                             last ids and counts other than n_visit (the
                             finer quarter cull visits fewer entries) are
                             bitwise those of the unsplit raster */
    int32_t split_mean_factor; /* 0..64 (2); 0: the threshold is split_entries
                             alone. Otherwise no tile is split unless the
                             longest tiles reach twice factor x the mean (a
                             long tail): where every tile is long, no tile
                             is on the critical path alone, and the quad
                             walk's extra instructions per entry cost more
                             than its shorter walks gain */
    int32_t footprint;    /* TGS_FOOTPRINT_*: the tiles tgs_project gives a
                             Gaussian (OPACITY_AWARE by default) */
    int32_t sub_bins;     /* BINNED with exact repair (repair = ALL, packed =
                             0, near_shift = 0): the binning first orders each
                             (tile, bin) segment by this many sub-bins of the
                             same log-depth map, and the repair sorts the
                             sub-segments. 1, 2, 4 or 8; 0 = the default 8
                             (1 where a group's segments times the sub-bins
                             exceed the group sort's 4096 counters, e.g. 8-
                             pixel tiles at K = 256, or without groups).
                             The stream is the same for every value: only the
                             split of the work between the binning and the
                             repair changes (fewer sub-bins: fewer, longer
                             sub-segments) */
} tgs_params;

/* Entry buffers written by tgs_bin and read by tgs_rasterize. All device
   pointers; sized for `capacity` entries, T = tiles_x * tiles_y tiles.
   GLOBAL order: keys [capacity] (tile << 32 | depth bits, sorted),
       vals [capacity] (Gaussian ids in that order), offsets [T + 1].
   BINNED order: pairs [capacity] (depth bits << 32 | id in tile-bin-major
       order, every (tile, bin) segment sorted), offsets [T * K + 1] (bin
       offsets, tile-major), records [capacity][12] when params.packed (the
       splat of each entry with its mean relative to the entry's tile
       origin: mx - 16 tx, my - 16 ty, a, b, c, opacity, r, g, b, id bits,
       0, 0), zrange [2] (the depth range).
   counters [4] int64: entries M, visible Gaussians V, overflow flag (1 when
       M > capacity: the stream was truncated and tgs_rasterize writes NaN),
       repaired entries (BINNED: the entries of the sorted segments).
   tile_order [T + 2] (optional, NULL = none): tgs_bin writes the tiles in
       descending order of their entry count (grouped by the bit length of
       the count) and the WAVE raster dispatches tiles in that order, so the
       longest tiles start first; tile_order[T] = the number of tiles the
       raster splits (the first ones of the order): those with at least
       tile_order[T + 1] entries, the smallest power of two >=
       params.split_entries and >= params.split_mean_factor x the mean
       entries of the non-empty tiles (this bound only when the non-empty
       tiles have at least 8192 blocks, enough wavefronts to fill the GPU)
       that leaves at most 1024 of them; 0 and 0 when split_entries is 0,
       or when the bound from the mean applies and the longest tiles' bit
       length puts them below twice it.
   seg_base [T + 1] (required with params.per_tile_bins_dev, else unused):
       tgs_bin writes the first segment of each tile, seg_base[T] = the
       number of segments S; offsets then holds S + 1 meaningful words (size
       it for T * num_bins + 1).
   repaired [T * K] (optional, NULL = none; BINNED): 1 for every segment
       tgs_bin sorted, else 0 (with per-tile bin counts the first S words,
       in the segment numbering of seg_base). */
typedef struct {
    int64_t capacity;
    uint64_t* keys_dev;
    uint32_t* vals_dev;
    uint64_t* pairs_dev;
    uint32_t* offsets_dev;
    float* records_dev;
    uint8_t* masks_dev;
    float* zrange_dev;
    int64_t* counters_dev;
    uint32_t* tile_order_dev;
    uint32_t* seg_base_dev;
    uint8_t* repaired_dev;
} tgs_binned;

/* Fills the paper's defaults (16 px tiles, K = 64, S = 8192, 1st / 99th
   percentiles, 5 % pad, repair budget 0.25, shift alpha 1 and gamma 0.25),
   the WAVE raster gathering by id (packed = 0), exact repair (repair =
   ALL, near_shift = 0) and the opacity-aware footprint. The paper's own selective mode is repair = RULES
   with near_shift = 1. */
TGS_API void tgs_default_params(tgs_params* params);

/* Projection + SH colour + opacity-aware tile rect for every Gaussian. The
   geometry is evaluated in binary64 and rounded once to the fp32 outputs;
   the depth key is the binary32 rounding of ((R20 x + R21 y) + R22 z) + t2
   evaluated in binary64 without contraction. */
TGS_API tgs_status tgs_project(const tgs_gaussians* gaussians, const tgs_camera* camera,
                       const tgs_params* params, tgs_projected* out, void* stream);

/* tgs_project for num_views (1..TGS_MAX_VIEWS) cameras of the same
   Gaussians: cameras, params and out are host arrays of num_views
   elements, out[v] receives exactly what tgs_project(gaussians, &cameras[v],
   &params[v], &out[v]) writes (bitwise). Each launch reads every
   Gaussian's parameters once and writes up to 8 views. */
TGS_API tgs_status tgs_project_views(const tgs_gaussians* gaussians, int32_t num_views, const tgs_camera* cameras,
                             const tgs_params* params, tgs_projected* out, void* stream);

/* Workspace bytes tgs_bin needs for n Gaussians, `capacity` entries, this
   camera, params and order. */
TGS_API size_t tgs_bin_workspace_size(int64_t n, int64_t capacity, const tgs_camera* camera,
                              const tgs_params* params, int32_t order);

/* Builds the entry stream of `order`. num_entries_host: NULL = no host
   synchronisation (an overflow is only reported through counters[2]);
   non-NULL = wait for the entry count, store it there, and return
   TGS_ERR_CAPACITY without building the stream when it exceeds capacity.
   GLOBAL order without the host count: the radix sort runs over all
   `capacity` slots, those past the entry count padded with keys past the
   last tile (they stay out of the tile ranges), so its cost follows the
   capacity; size it close to the expected entry count. */
TGS_API tgs_status tgs_bin(const tgs_projected* projected, const tgs_camera* camera,
                   const tgs_params* params, int32_t order, void* workspace_dev,
                   size_t workspace_bytes, tgs_binned* out, int64_t* num_entries_host,
                   void* stream);

/* Composites every pixel front to back over its tile's range. bg: host
   float[3]. Outputs (device): rgb [H][W][3], alpha [H][W] (= 1 - final
   transmittance), last [H][W] int32 stream position of the last composited
   entry or -1. Optional counters (NULL to skip; any non-NULL selects the
   instrumented kernel instance): n_contrib [H][W] composited entries,
   n_visit [H][W] entries the pixel evaluated before it stopped, n_support
   [H][W] evaluated entries with alpha >= 1/255 (including the one that
   stopped the pixel). trans_dev [H][W] (optional, WAVE raster only): the
   final transmittance T itself (alpha = 1 - T loses its low bits), which
   tgs_rasterize_backward can take instead of repeating the forward walk. */
TGS_API tgs_status tgs_rasterize(const tgs_projected* projected, const tgs_binned* binned,
                         const tgs_camera* camera, const tgs_params* params, int32_t order,
                         const float* bg, float* rgb_dev, float* alpha_dev, int32_t* last_dev,
                         int32_t* n_contrib_dev, int32_t* n_visit_dev, int32_t* n_support_dev,
                         float* trans_dev, void* stream);

/* Gradient lines of tgs_rasterize_backward: [n][12] fp32 per Gaussian,
   dL/d of the splat's mean_x, mean_y (the mean hi + lo), conic_a, conic_b,
   conic_c, opacity, r, g, b, then three zero words. */
#define TGS_GRAD_WORDS 12

/* Backward of tgs_rasterize for the same projected splats, entry stream
   (tgs_bin output of `order`, unchanged since), camera, params and bg:
   given d_rgb [H][W][3] = dL/d rgb and d_alpha [H][W] = dL/d alpha (NULL =
   zero), writes d_splats [n][TGS_GRAD_WORDS] (overwritten; entries of
   Gaussians that no pixel composited are zero). trans_dev and last_dev
   [H][W]: the forward's final transmittance and last position (both from a
   tgs_rasterize of the same stream, WAVE raster), or both NULL, when the
   per-pixel forward walk is recomputed from the stream instead. Gradients
   are summed with float atomics: the summation order, and so the last bits,
   may differ between runs. With the overflow flag set in counters[2] the
   result is all zero. */
TGS_API tgs_status tgs_rasterize_backward(const tgs_projected* projected, const tgs_binned* binned,
                                  const tgs_camera* camera, const tgs_params* params, int32_t order,
                                  const float* bg, const float* d_rgb_dev, const float* d_alpha_dev,
                                  const float* trans_dev, const int32_t* last_dev, float* d_splats_dev,
                                  void* stream);

/* Parameter gradients, device pointers, fp32, in the layouts of
   tgs_gaussians (sh: [n][(D+1)^2][3]); every element is overwritten. */
typedef struct {
    float* means_dev;
    float* log_scales_dev;
    float* quats_dev;
    float* logits_dev;
    float* sh_dev;
} tgs_gaussian_grads;

/* Backward of tgs_project: from the gradient lines d_splats [n][12] to
   dL/d(means, log_scales, quats, logits, sh), recomputing the projection in
   binary64. Gaussians that tgs_project makes invisible get zero gradients;
   colour channels clamped at zero and the frustum guard of the Jacobian
   pass no gradient, as in the forward definition. */
TGS_API tgs_status tgs_project_backward(const tgs_gaussians* gaussians, const tgs_camera* camera,
                                const float* d_splats_dev, tgs_gaussian_grads* grads, void* stream);

/* Batched rendering: up to TGS_MAX_VIEWS cameras (views), each with its own
   projected splats, tgs_bin stream (any order, tile size and bin counts of
   its params), composited in ONE persistent launch. Work items are (view,
   tile, 8x8 block), ordered heaviest tile first over all views and pulled
   by wavefronts from device-scope cursors until none is left; each item is
   the WAVE raster's block walk, so every view's rgb / alpha / last are
   bit-identical to tgs_rasterize with that view's arguments. All host
   arrays have num_views elements; rgb / alpha / last are host arrays of
   device pointers. The call enqueues a fill, two small ordering launches
   and the persistent launch on `stream` and never synchronises, so it can
   be captured in a HIP graph (the view descriptors travel in the kernel
   arguments). Workspace: tgs_batch_workspace_size bytes, caller-owned. */
TGS_API size_t tgs_batch_workspace_size(int32_t num_views, const tgs_camera* cameras, const tgs_params* params);
TGS_API tgs_status tgs_rasterize_batch(int32_t num_views, const tgs_projected* projected, const tgs_binned* binned,
                               const tgs_camera* cameras, const tgs_params* params, const int32_t* orders,
                               const float* bg, float* const* rgb_dev, float* const* alpha_dev,
                               int32_t* const* last_dev, void* workspace_dev, size_t workspace_bytes,
                               void* stream);

/* tgs_rasterize_batch for callers that cannot allocate device memory: code
   under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc. Same arguments, outputs and errors as tgs_rasterize_batch
   without the workspace: the batch's control words and work list live in a
   fixed scratch array inside the library, 4 MiB on every device the library
   runs on (held until the process ends), enough for about one million 8x8
   pixel blocks over all views (e.g. 16 views of 3840x2160). Views needing
   more (tgs_batch_workspace_size above 4 MiB) are rejected with
   TGS_ERR_WORKSPACE before anything is enqueued. The call allocates
   nothing; its first call on a device looks up that device's scratch
   address (make that first call outside a graph capture). Every call on a
   device shares that device's scratch: calls that overlap in time on one
   device (two streams, two threads) race and must be serialised by the
   caller; the control words are cleared by a fill kernel at the start of
   every call. */
TGS_API tgs_status tgs_rasterize_batch_noalloc(int32_t num_views, const tgs_projected* projected,
                                       const tgs_binned* binned, const tgs_camera* cameras,
                                       const tgs_params* params, const int32_t* orders, const float* bg,
                                       float* const* rgb_dev, float* const* alpha_dev, int32_t* const* last_dev,
                                       void* stream);

/* Learned bin-count proposal. The paper fixes K = 64 bins per tile (section
   "Implementation details") and varies K per frame in its bin-count table;
   this addition picks K_t per tile with a small network from the previous
   frame's per-tile depth histogram and counts. Exact repair keeps every
   image unchanged whatever it picks (only bin construction and repair time
   move), and the fixed K remains the fallback.
   Network: 16 features -> 64 -> 64 -> 8 (ReLU), fp32 parameters in one
   array of TGS_MLP_PARAMS floats, row-major: W1 [16][64], b1 [64],
   W2 [64][64], b2 [64], W3 [64][8], b3 [8]; choice k -> K_t = 2^(k+1).
   Features [T][16] of tile t (K_t bins, lengths l_b, n_t = sum l_b, M
   entries): log2(1+n_t); an 8-cell depth histogram / max(n_t,1) (bins
   merged, or spread evenly when K_t < 8); log2(1+max l_b); non-empty bins
   / K_t; log2(K_t)/8; entries in bins of 2 or more / max(n_t,1);
   log2(1 + sum l_b^2 / max(n_t,1)); log2(1+M/T); log2(1+n_t) - log2(1+M/T). */
#define TGS_MLP_PARAMS 5768

/* Features [T][16] of the stream in `binned` (written by tgs_bin with the
   same camera and params). */
TGS_API tgs_status tgs_tile_features(const tgs_binned* binned, const tgs_camera* camera, const tgs_params* params,
                             float* features_dev, void* stream);

/* per_tile_bins [T] = 2^(argmax logit + 1) for each tile (first maximum on
   ties); fallback_bins everywhere when a weight is not finite, and where a
   logit is not finite. logits [T][8] are written when not NULL (not for a
   non-finite weight vector). */
TGS_API tgs_status tgs_propose_bins(const float* weights_dev, const float* features_dev, int64_t num_tiles,
                            int32_t fallback_bins, int32_t* per_tile_bins_dev, float* logits_dev, void* stream);

/* One training step on T tiles: loss L = (1/T) sum_t sum_k softmax(z_t)_k
   regret[t][k] (regret: the cost of choice k above the tile's best, [T][8]),
   its gradient g by backpropagation, then velocity = momentum * velocity +
   g and weights -= lr * velocity. loss_dev (nullable) receives L. With lr
   = momentum = 0 and a zero velocity, velocity returns g. Workspace:
   tgs_mlp_train_workspace_size(T) bytes. */
TGS_API size_t tgs_mlp_train_workspace_size(int64_t num_tiles);
TGS_API tgs_status tgs_mlp_train_step(float* weights_dev, float* velocity_dev, const float* features_dev,
                              const float* regret_dev, int64_t num_tiles, float lr, float momentum,
                              void* workspace_dev, size_t workspace_bytes, float* loss_dev, void* stream);

/* Message for the last failing call on this thread ("" if none). */
TGS_API const char* tgs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TILEGS_H */
