// Shared device helpers and the internal host interface of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tilegs.h"

namespace tgs {

constexpr int kWave = 64;
constexpr int kTile = 16;          // tile edge in pixels
constexpr int kSplatVec = 4;       // float4s per splat (64 bytes)
constexpr int kRecordVec = 3;      // float4s per packed record (48 bytes)
constexpr int kInfoWords = 4;

// Fixed thresholds of the 3DGS image model.
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ int lane() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

// Number of set bits of `mask` below the calling lane.
__device__ __forceinline__ uint32_t rank_in(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

__device__ __forceinline__ uint32_t shfl_up_u32(uint32_t v, int d) { return (uint32_t)__shfl_up((int)v, d, kWave); }
__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, int src) { return (uint32_t)__shfl((int)v, src, kWave); }
__device__ __forceinline__ uint32_t shfl_xor_u32(uint32_t v, int m) { return (uint32_t)__shfl_xor((int)v, m, kWave); }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    uint32_t lo = shfl_xor_u32((uint32_t)v, m);
    uint32_t hi = shfl_xor_u32((uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive prefix sum across the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t o = shfl_up_u32(v, d);
        if (lane() >= d) v += o;
    }
    return v;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Give each XCD a contiguous run of work items so that neighbouring
// tiles, which share Gaussians, meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    constexpr int X = 8;
    int per = nblocks / X, rem = nblocks % X;
    int x = b % X, k = b / X;
    return x * per + (x < rem ? x : rem) + k;
}

__host__ __device__ __forceinline__ int div_up(int a, int b) { return (a + b - 1) / b; }

// Tile rect of an info record, clipped to the tile grid; returns the number
// of tiles (0 = invisible). Every stage derives the entries of a Gaussian
// from this, so a caller-filled rect can never address outside the grid.
__device__ __forceinline__ int rect_of(const uint4& in, int tiles_x, int tiles_y, int& x0, int& y0, int& x1,
                                       int& y1) {
    x0 = min((int)(in.y & 0xFFFFu), tiles_x);
    y0 = min((int)(in.y >> 16), tiles_y);
    x1 = min((int)(in.z & 0xFFFFu), tiles_x);
    y1 = min((int)(in.z >> 16), tiles_y);
    if (x1 <= x0 || y1 <= y0) return 0;
    return (x1 - x0) * (y1 - y0);
}

// XCD (accelerator complex die) executing the calling wave, 0..7.
__device__ __forceinline__ int xcc_id() {
    return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u);
}
constexpr int kXcc = 8;
#ifndef TGS_COUNT_COPIES
#define TGS_COUNT_COPIES 8
#endif
// Copies of the (tile, bin) counts; waves count into copy xcc_id() mod kCopies.
constexpr int kCopies = TGS_COUNT_COPIES;

// -0.5 / ln 2: with the conic scaled by it, exp(-q / 2) = exp2(q').
constexpr float kHalfLog2e = -0.72134752044448170f;

// Staged form of a splat for one tile, as the raster consumes it: mean
// relative to the tile origin computed as (hi - origin) + lo, conic scaled
// by kHalfLog2e (off-diagonal doubled), opacity, colour. Both rasters and
// the packed records use this one function, so every route gives the same
// bits.
__device__ __forceinline__ void stage_splat(const float4& a, const float4& b, const float4& c, float ox, float oy,
                                            float4& s0, float4& s1, float& s2) {
#pragma clang fp contract(off)
    s0 = make_float4((a.x - ox) + a.z, (a.y - oy) + a.w, kHalfLog2e * b.x, (2.0f * kHalfLog2e) * b.y);
    s1 = make_float4(kHalfLog2e * b.z, b.w, c.x, c.y);
    s2 = c.z;
}

// Conservative block test: can q = a dx^2 + 2 b dx dy + c dy^2 (unscaled
// conic, mean mx, my) reach 2 ln(255 o) at some pixel centre of the box
// [xa, xb] x [ya, yb]? The minimum of the convex q over the box is 0 when
// the mean is inside. Otherwise it lies on an edge facing the mean: from a
// point of any other edge, q decreases toward the mean (where q = 0) and
// that direction enters the box. So the bound is the smaller of two edge
// minima: the vertical edge on the mean's side and the horizontal edge on
// the mean's side (either one of a pair when the mean lies between them,
// whose minimum is then at least the true one). The margin exceeds the
// binary32 error of both this bound and the per-pixel evaluation, so a
// block that fails the test fails the alpha >= 1/255 test at every one of
// its pixels. The edge minimisers use the hardware reciprocal: an edge
// point that misses the exact minimiser by a relative 1e-7 raises q only by
// c (1e-7 e)^2, far inside the margin.
__device__ __forceinline__ bool block_may_touch(float mx, float my, float a, float b, float c, float o, float xa,
                                                float xb, float ya, float yb) {
    const float dxl = mx - xb, dxh = mx - xa, dyl = my - yb, dyh = my - ya;
    const float ic = __builtin_amdgcn_rcpf(c), ia = __builtin_amdgcn_rcpf(a);
    float qx, qy;
    {
        const float d = dxh < 0.0f ? dxh : dxl, e = fminf(fmaxf(-b * d * ic, dyl), dyh);
        qx = a * d * d + 2.0f * b * d * e + c * e * e;
    }
    {
        const float e = dyh < 0.0f ? dyh : dyl, d = fminf(fmaxf(-b * e * ia, dxl), dxh);
        qy = a * d * d + 2.0f * b * d * e + c * e * e;
    }
    const bool inside = dxl <= 0.0f && dxh >= 0.0f && dyl <= 0.0f && dyh >= 0.0f;
    const float qmin = inside ? 0.0f : fminf(qx, qy);
    const float mxd = fmaxf(fabsf(dxl), fabsf(dxh)), myd = fmaxf(fabsf(dyl), fabsf(dyh));
    const float mag = a * mxd * mxd + c * myd * myd + 2.0f * fabsf(b) * mxd * myd;
    // 2 ln(255 o) from the hardware base-2 logarithm (relative error near
    // 1e-7, far inside the 1e-3 margin)
    const float tau = (2.0f * 0.69314718f) * __builtin_amdgcn_logf(255.0f * o);
    return qmin <= tau + 1e-3f + 4e-6f * mag;
}

// Pixel-centre box (tile-local) of the in-image pixels of the 8x8 block at
// tile-local offset (bx, by) of the tile whose first pixel is (x0, y0);
// false when the block lies outside the image.
__device__ __forceinline__ bool block_box_at(int bx, int by, int x0, int y0, int width, int height, float& xa,
                                             float& xb, float& ya, float& yb) {
    const int nx = min(8, width - (x0 + bx)), ny = min(8, height - (y0 + by));
    if (nx <= 0 || ny <= 0) return false;
    xa = bx + 0.5f;
    xb = bx + nx - 0.5f;
    ya = by + 0.5f;
    yb = by + ny - 0.5f;
    return true;
}

// The same for 8x8 block w (0..3, row-major) of 16x16 tile (tx, ty).
__device__ __forceinline__ bool block_box(int w, int tx, int ty, int width, int height, float& xa, float& xb,
                                          float& ya, float& yb) {
    return block_box_at((w & 1) * 8, (w >> 1) * 8, tx * kTile, ty * kTile, width, height, xa, xb, ya, yb);
}

// Where the entry-placing kernels put the per-entry raster data. masks ==
// null: nothing. Otherwise mask p gets bit w set when 8x8 block w of the
// entry's tile may see the splat, and, when records != null, record p the
// staged splat of the entry's Gaussian for its tile ({mx, my, a', 2b'},
// {c', opacity, r, g}, {b, id, 0, 0}).
struct RecordSink {
    const float4* splats;
    float4* records;
    uint8_t* masks;
    int K, tiles_x, width, height;
    __device__ __forceinline__ void put(uint32_t seg, uint32_t pos, uint64_t pair) const {
        if (!masks) return;
        const uint32_t t = seg / (uint32_t)K;
        const int tx = (int)(t % (uint32_t)tiles_x), ty = (int)(t / (uint32_t)tiles_x);
        const float ox = (float)(tx * kTile), oy = (float)(ty * kTile);
        const uint32_t gid = (uint32_t)pair;
        const float4* sp = splats + kSplatVec * (int64_t)gid;
        const float4 a = sp[0], b = sp[1], c = sp[2];
        float4 s0, s1;
        float s2;
        stage_splat(a, b, c, ox, oy, s0, s1, s2);
        if (records) {
            float4* rec = records + kRecordVec * (int64_t)pos;
            rec[0] = s0;
            rec[1] = s1;
            rec[2] = make_float4(s2, __uint_as_float(gid), 0.f, 0.f);
        }
        uint32_t m = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            float xa, xb, ya, yb;
            if (block_box(w, tx, ty, width, height, xa, xb, ya, yb) &&
                block_may_touch(s0.x, s0.y, b.x, b.y, b.z, b.w, xa, xb, ya, yb))
                m |= 1u << w;
        }
        masks[pos] = (uint8_t)m;
    }
};

// Segment numbering of the BINNED stream: segment first(t) + b is bin b of
// tile t. Uniform (seg_base == null): K bins per tile, first(t) = t K.
// Grouped binning (uniform K): groups of GT consecutive tiles, G groups,
// GS = GT K segments per group (group g holds segments g GS .. g GS + GS - 1).
// SB > 1 (exact repair with depth bins): every bin is split further into SB
// sub-bins of the log-depth map at SB K bins (bin = sub-bin / SB exactly),
// so the group sort leaves each segment ordered by sub-bin, which is the
// depth order between sub-bins, and the repair sorts only the sub-segments;
// entry code in the group = (tile in group K + bin) SB + sub.
// Per-tile bin counts (seg_base != null): K is their bound, group g holds
// segments seg_base[g GT] .. seg_base[min(T, g GT + GT)] - 1, and its
// sub-bin count is chosen per group (ginfo[g] = {first segment, segments,
// log2 sub-bins}, written by the group scan) so that its codes fit LDS; SB
// is then the largest sub-bin count and sub-segment ids are first segment
// SB + code.
struct GroupMap {
    int K, GT, G, GS, SB;
    int64_t T;
    const uint32_t* seg_base;
    const uint2* tile_seg;
    uint4* ginfo;
};
#ifndef TGS_GROUP_SEGS
#define TGS_GROUP_SEGS 512
#endif
#ifndef TGS_SUB_BINS
#define TGS_SUB_BINS 8
#endif
constexpr int kSubBins = TGS_SUB_BINS;  // sub-bins per bin in exact-repair mode
constexpr int kGroupSegTarget = TGS_GROUP_SEGS;  // segments per group aimed at
constexpr int kMaxGroups = 8192;      // LDS counters of one workgroup
constexpr int kMaxGroupSegs = 4096;   // LDS counters of one group sort
constexpr int kGroupChunk = 2048;     // Gaussians per workgroup of the group count / scatter
// The grouped path's group shape for T tiles and K bins: GT = max(1,
// kGroupSegTarget / K) tiles, doubled until G <= kMaxGroups; .G = 0 when GS
// would exceed kMaxGroupSegs (then the per-entry atomic path is used). SB =
// sub (a power of two) when GS sub <= kMaxGroupSegs, else 1.
GroupMap group_map(int64_t T, int K, int sub);
// The same for per-tile bin counts bounded by K (a power of two): GT =
// min(8, kMaxGroupSegs / K) tiles; sub-bins are chosen per group.
GroupMap group_map_var(int64_t T, int K, int sub);

// Per-tile bin counts: seg_base [T + 1] is the exclusive prefix sum of the
// counts (powers of two), first(t) = seg_base[t], and the number of
// segments S = seg_base[T] is known on the device only.
struct SegMap {
    const uint32_t* seg_base;
    int K;
    const uint2* tile_seg;  // per-tile bin counts: {seg_base[t], 32 - log2 K_t} [T]
    __device__ __forceinline__ uint32_t first(int64_t t) const {
        return seg_base ? seg_base[t] : (uint32_t)(t * K);
    }
};

// Binning key of a Gaussian. splats == null: its depth. Otherwise the
// near-depth key z - min(alpha s_max, gamma z) (s_max: splat word 11),
// clamped to [lo, hi] = [max(znear, 1e-4), zfar], in binary32 without
// contraction (supplement, Algorithm "Robust depth-range estimation",
// near-depth mode; the bin map takes the same key).
struct NearKey {
    const float4* splats;
    float alpha, gamma, lo, hi;
    __device__ __forceinline__ uint32_t operator()(uint32_t depth_bits, int64_t g) const {
#pragma clang fp contract(off)
        if (!splats) return depth_bits;
        const float z = __uint_as_float(depth_bits);
        const float smax = splats[kSplatVec * g + 2].w;
        const float a = alpha * smax, b = gamma * z;
        const float d = a < b ? a : b;
        float k = z - d;
        if (k < lo) k = lo;
        if (k > hi) k = hi;
        return __float_as_uint(k);
    }
};

struct Cam {
    double R[9], t[3];
    double fx, fy, cx, cy;
    double znear, zfar;
    double campos[3];
    double lim_xp, lim_xn, lim_yp, lim_yn;
    int width, height, tile, tiles_x, tiles_y;
    int footprint;  // TGS_FOOTPRINT_*
};

// tile: tile edge in pixels (8, 16 or 32); footprint: TGS_FOOTPRINT_*.
Cam make_cam(const tgs_camera& c, int tile, int footprint);

// Cameras of one projection launch: each lane reads its Gaussian once and
// writes its splat and info lines for every camera.
constexpr int kProjViews = 8;
struct ProjViews {
    Cam cam[kProjViews];
    float4* splats[kProjViews];
    uint4* info[kProjViews];
    int nv;
};
hipError_t launch_project_views(const tgs_gaussians& g, const ProjViews& views, hipStream_t s);

// Launch helpers (host), implemented next to their kernels.
hipError_t launch_project(const tgs_gaussians& g, const Cam& cam, float* splats, uint32_t* info,
                          hipStream_t s);

// Workgroups of the single-pass scans for n items (at least one).
int64_t scan_blocks(int64_t n);

// Entry emission scan over the info array: emit_off[g] = number of entries
// of the Gaussians before g, vis_ids[rank] = g for every visible Gaussian;
// counters[0] = M, counters[1] = V (visible), counters[2] = 1 when M
// exceeds `capacity` (every later stage then skips its writes beyond the
// buffers). ticket and status_x / status_y [scan_blocks(n)] must be zero.
hipError_t launch_emit_scan(const uint32_t* info, int64_t n, int tiles_x, int tiles_y, uint32_t* emit_off,
                            uint32_t* vis_ids, uint32_t* ticket, uint64_t* status_x, uint64_t* status_y,
                            int64_t* counters, int64_t capacity, hipStream_t s);

// Depth samples: the visible Gaussians at ranks floor(i V / S), i < S (all
// of them when V <= S), read through vis_ids; samples [S] is scratch for
// their keys.
hipError_t launch_depth_range(const uint32_t* info, const uint32_t* vis_ids, const int64_t* counters, NearKey nk,
                              int S, float p_lo, float p_hi, float pad, float znear, float zfar, float* zrange,
                              uint32_t* samples, hipStream_t s);
// The arguments of the depth range, for the launch that runs it beside the
// group count.
struct RangeArgs {
    const uint32_t* vis_ids;
    const int64_t* counters;
    NearKey nk;
    int S;
    float p_lo, p_hi, pad, znear, zfar;
    float* zrange;
    uint32_t* samples;  // [S] scratch for the gathered sample keys
};

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);

// (tile, bin) counting with one count copy per XCD: count [kXcc][S] (S =
// nseg, or seg_base[T] with per-tile bin counts). The rank of each entry in
// its copy, with the copy index in the top three bits, goes to entry_rank.
hipError_t launch_bin_count(const uint32_t* info, int64_t n, const uint32_t* emit_off, const float* zrange,
                            NearKey nk, SegMap sm, int tiles_x, int tiles_y, uint32_t* count, int64_t nseg,
                            uint32_t* entry_rank, int64_t capacity, hipStream_t s);
// Repair length buckets: 2..8, 9..16, 17..32, 33..64 (lane groups of one
// wavefront, registers), 65..512 (one wavefront, LDS), 513..4096 and
// 4097..8192 (one workgroup, LDS), above 8192 (one workgroup, global memory).
constexpr int kBuckets = 8;
__host__ __device__ __forceinline__ int bucket_of(uint32_t len) {
    if (len <= 1) return -1;
    if (len <= 8) return 0;
    if (len <= 16) return 1;
    if (len <= 32) return 2;
    if (len <= 64) return 3;
    if (len <= 512) return 4;
    if (len <= 4096) return 5;
    if (len <= 8192) return 6;
    return 7;
}

// bin_off[s] = exclusive scan of the summed copies (bin_off[S] = M);
// count[x][s] becomes the base position of copy x inside segment s. With
// queue_all, every segment of two or more entries is appended to
// lists[bucket][...] (bucket stride: nseg) with bucket_count[bucket]
// entries, its entries are added to counters[3] and repaired[s] (when not
// null) is set; nothing is queued when counters[2] flags an overflow.
// Without queue_all, repaired[s] = 0. S = nseg, or *nseg_dev when nseg_dev
// is not null (then nseg is its upper bound). ticket, status
// [scan_blocks(nseg)] and bucket_count must be zero.
hipError_t launch_bin_offsets(uint32_t* count, int64_t nseg, const uint32_t* nseg_dev, uint32_t* bin_off,
                              uint32_t* ticket, uint64_t* status, uint32_t* lists, uint32_t* bucket_count,
                              int64_t* counters, bool queue_all, uint8_t* repaired, hipStream_t s);
// Rule-based repair selection over the T * K segments (uniform K): the
// keep rules per segment, the prefix of the kept lengths by a single-pass
// scan (segments whose inclusive prefix is within the budget are queued as
// in launch_bin_offsets), then one workgroup continues the first-fit scan
// after the first kept segment that does not fit. ticket, status
// [scan_blocks(T K)] and ctl [2] must be zero; counters[3] gets the
// selected entries.
hipError_t launch_repair_select(const uint32_t* bin_off, int64_t T, int K, float budget, uint32_t* ticket,
                                uint64_t* status, uint32_t* ctl, uint32_t* lists, uint32_t* bucket_count,
                                int64_t* counters, uint8_t* repaired, hipStream_t s);
hipError_t launch_bin_scatter(const uint32_t* info, int64_t n, const uint32_t* emit_off, const float* zrange,
                              NearKey nk, SegMap sm, int tiles_x, int tiles_y, const uint32_t* bin_off,
                              const uint32_t* base, int64_t nseg, const uint32_t* entry_rank, uint64_t* pairs,
                              int64_t capacity, RecordSink rs, hipStream_t s);

// Grouped binning, see GroupMap. group_count: gcount [G] must be zero;
// wgbase [ceil(n / kGroupChunk) x G] receives each workgroup's slice base
// in the groups it touches. group_scan: group_off [G + 1] = exclusive
// prefix of gcount. group_scatter: tmp_pair / tmp_code [capacity] get every
// entry (pair, segment within its group) grouped by group; positions past
// the capacity are dropped; order [G] = the groups, longest first.
// group_sort: pairs in (tile, bin) order, bin_off
// [S + 1] (S = T K), repair queues and repaired[] as launch_bin_offsets,
// single-entry segments' records; bucket_count must be zero. With SB > 1
// the repair queues hold sub-segments as uint2 {begin, length} (list stride
// list_stride entries); repaired[] and counters[3] stay per segment.
// tile_hist != null: also adds each tile's bit-length bucket to the tile
// order histogram tile_hist [33] (zero before), so that only the placement
// half of the tile order is left (TileOrder). With SB > 1, a group of at
// most 4096 entries is staged through LDS and its sub-segments of up to 128
// entries come out in pair order (they are not queued).
// The group count needs no bins; its first workgroup computes the depth
// range (ra) meanwhile, which the group scatter then uses.
hipError_t launch_group_count(const uint32_t* info, int64_t n, const uint32_t* emit_off, GroupMap gm, int tiles_x,
                              int tiles_y, uint32_t* gcount, uint32_t* wgbase, const RangeArgs& ra, hipStream_t s);
hipError_t launch_group_scan(const uint32_t* gcount, GroupMap gm, uint32_t* group_off, uint32_t* order,
                             hipStream_t s);
hipError_t launch_group_scatter(const uint32_t* info, int64_t n, const uint32_t* emit_off, const float* zrange,
                                NearKey nk, GroupMap gm, int tiles_x, int tiles_y, const uint32_t* group_off,
                                const uint32_t* wgbase, uint64_t* tmp_pair, uint16_t* tmp_code, int64_t capacity,
                                hipStream_t s);
hipError_t launch_group_sort(const uint64_t* tmp_pair, const uint16_t* tmp_code, const uint32_t* group_off,
                             const uint32_t* order, GroupMap gm, int64_t nseg, int64_t capacity, uint64_t* pairs, uint32_t* bin_off,
                             uint32_t* lists, int64_t list_stride, uint32_t* bucket_count,
                             int64_t* counters, bool queue_all, uint8_t* repaired, RecordSink rs,
                             uint32_t* tile_hist, hipStream_t s);

// Per-tile bin counts: seg_base[t] = exclusive prefix sum of the bin counts
// (each clamped to 1..kmax and rounded down to a power of two), seg_base[T]
// = S, and tile_seg[t] = {seg_base[t], 32 - log2 K_t} for the entry
// kernels (one 8-byte load per entry). ticket and status [scan_blocks(T)]
// must be zero.
hipError_t launch_seg_base(const int32_t* per_tile_bins, int64_t T, int kmax, uint32_t* seg_base, uint2* tile_seg,
                           uint32_t* ticket, uint64_t* status, hipStream_t s);
// p[0 .. mult * *n_dev) = v.
hipError_t launch_fill_u32_dyn(uint32_t* p, uint32_t v, const uint32_t* n_dev, int mult, int64_t max_n,
                               hipStream_t s);

// Placement half of the tile order (launch_tile_order below) over a
// histogram that is already complete: hist [33] per bit-length bucket, then
// the 33 placement cursors, zero. order == null: none.
struct TileOrder {
    const uint32_t* offsets;
    SegMap sm;
    int64_t T;
    uint32_t* hist;
    uint32_t* order;
    int split, factor;
};

// Sorts every queued segment by its 64-bit pairs and writes its records.
// The lists hold segment ids located by bin_off (list stride nseg), or with
// desc uint2 {begin, length} entries (sub-segments; no records). to.order !=
// null: the last workgroups of the long-segment launch also place the tiles
// (the sorts do not change the offsets).
hipError_t launch_repair(const uint32_t* bin_off, int64_t nseg, uint64_t* pairs, const uint32_t* seg_lists,
                         const uint32_t* bucket_count, RecordSink rs, bool desc, const TileOrder& to, hipStream_t s);
// The placement half alone (tile order after a grouped sort without repair).
hipError_t launch_tile_place(const TileOrder& to, hipStream_t s);

// Tiles in descending order of their entry count (coarse: by bit length of
// the count), so the heaviest tiles are dispatched first. order[T] = the
// number of tiles the WAVE raster splits: those with at least order[T + 1]
// entries, the smallest power of two >= `split` (0: none) and >= factor x
// the mean count of the non-empty tiles (when their 4 block wavefronts each
// would fill the CUs) that leaves at most kSplitTiles of them; they come
// first. hist [66] must be zero.
constexpr int kSplitTiles = 1024;
constexpr int kFillWaves = 256 * 32;  // wavefronts the 256 CUs hold at 8 per SIMD
hipError_t launch_tile_order(const uint32_t* offsets, SegMap sm, int64_t T, uint32_t* hist, uint32_t* order, int split,
                             int factor, hipStream_t s);

hipError_t launch_emit_keys(const uint32_t* info, int64_t n, const uint32_t* emit_off, int tiles_x, int tiles_y,
                            uint64_t* keys, uint32_t* vals, int64_t capacity, hipStream_t s);
size_t global_sort_tmp_bytes(int64_t capacity, int end_bit);
hipError_t launch_global_sort(void* tmp, size_t tmp_bytes, uint64_t* keys_in, uint64_t* keys_out,
                              uint32_t* vals_in, uint32_t* vals_out, int64_t m, int end_bit, hipStream_t s);
hipError_t launch_tile_ranges(const uint64_t* keys, int64_t m, int64_t T, uint32_t* tile_off, hipStream_t s);
hipError_t launch_pad_keys(uint64_t* keys, uint32_t* vals, const int64_t* counters, int64_t capacity, int64_t T,
                           hipStream_t s);

struct RasterArgs {
    const float* splats;    // [n][16]
    const uint32_t* offsets;
    int stride;             // offsets index step per tile (1 for GLOBAL, K for BINNED)
    const uint32_t* seg_base;  // BINNED with per-tile bin counts: first segment of each tile [T + 1]
    const uint32_t* vals;   // GLOBAL ids
    const uint64_t* pairs;  // BINNED pairs
    const float* records;   // BINNED packed records or null
    const uint8_t* masks;   // block masks of the packed records
    const int64_t* counters;
    const uint32_t* order;  // tile dispatch order [T + 2] or null
    int split;              // WAVE, 16-pixel tiles, with order: split the first order[T] tiles
    int width, height, tile, tiles_x, tiles_y;  // tile: edge in pixels (the PLAIN raster: 16 only)
    float bg[3];
    float* rgb;
    float* alpha;
    int32_t* last;
    int32_t* n_contrib;
    int32_t* n_visit;
    int32_t* n_support;
    float* trans;           // final transmittance [H][W] (optional)
};
hipError_t launch_raster_plain(const RasterArgs& a, hipStream_t s);
hipError_t launch_raster_wave(const RasterArgs& a, hipStream_t s);

// Batched persistent raster: up to kMaxViews views in one launch (passed by
// value as the kernel argument, so a captured graph keeps them).
constexpr int kMaxViews = 16;
struct BatchView {
    const float* splats;
    const uint32_t* offsets;
    const uint32_t* seg_base;
    const uint32_t* vals;
    const uint64_t* pairs;
    const int64_t* counters;
    float* rgb;
    float* alpha;
    int32_t* last;
    int stride, width, height, tile, tiles_x, tiles_y;
};
struct BatchArgs {
    BatchView v[kMaxViews];
    uint32_t tile_base[kMaxViews + 1];  // first flattened tile of each view; [nv] = all tiles
    int nv;
    float bg[3];
};
// Bin-count proposal network (see mlp.hip).
int mlp_num_params();
hipError_t launch_tile_features(const uint32_t* offsets, SegMap sm, int64_t T, const int64_t* counters, float* feat,
                                hipStream_t s);
hipError_t launch_propose(const float* w, const float* feat, int64_t T, int32_t* bins, float* logits, int fallback,
                          hipStream_t s);
size_t mlp_train_workspace_floats(int64_t T);
hipError_t launch_mlp_train_step(float* w, float* v, const float* feat, const float* regret, int64_t T, float lr,
                                 float mu, float* ws, float* loss, hipStream_t s);

// ctl: 256 zeroed words; work: 8 * ceil(total_blocks / 8) words.
hipError_t launch_raster_batch(const BatchArgs& b, uint32_t* ctl, uint32_t* work, int64_t total_blocks, int grid,
                               hipStream_t s);

// Gradient lines: 12 floats per Gaussian (dL/d mean_x, mean_y, conic a, b,
// c, opacity, r, g, b, then 3 zero words).
constexpr int kGradWords = 12;

// dL/d(splat) into d_splats [n][kGradWords], which must be zero (float
// atomics accumulate into it).
hipError_t launch_raster_backward(const RasterArgs& a, const float* d_rgb, const float* d_alpha,
                                  const float* trans_in, const int32_t* last_in, float* d_splats, hipStream_t s);
// Parameter gradients from the gradient lines; every output is overwritten.
hipError_t launch_project_backward(const tgs_gaussians& g, const Cam& cam, const float* d_splats,
                                   const tgs_gaussian_grads& out, hipStream_t s);

}  // namespace tgs
