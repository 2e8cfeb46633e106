// C ABI: argument validation, workspace layout and the launch sequences of
// tgs_project / tgs_bin / tgs_rasterize.
#include <math.h>
#include <algorithm>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "common.hpp"

using namespace tgs;

namespace {

thread_local std::string g_err;

tgs_status fail(tgs_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
tgs_status fail(tgs_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

tgs_status hip_fail(hipError_t e, const char* where) {
    return fail(TGS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define TGS_HIP(call, where)                      \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

tgs_status check_camera(const tgs_camera* c) {
    if (!c) return fail(TGS_ERR_INVALID_ARG, "camera is NULL");
    if (c->width < 1 || c->width > 16384 || c->height < 1 || c->height > 16384)
        return fail(TGS_ERR_INVALID_ARG, "image size %dx%d outside 1..16384", c->width, c->height);
    if (!(c->znear > 0.0) || !(c->zfar > c->znear) || !isfinite(c->znear))
        return fail(TGS_ERR_INVALID_ARG, "need 0 < znear < zfar (got %g, %g)", c->znear, c->zfar);
    if (!(c->fx > 0.0) || !(c->fy > 0.0) || !isfinite(c->fx) || !isfinite(c->fy))
        return fail(TGS_ERR_INVALID_ARG, "focal lengths must be positive and finite");
    for (int i = 0; i < 9; ++i)
        if (!isfinite(c->R[i])) return fail(TGS_ERR_INVALID_ARG, "camera rotation is not finite");
    for (int i = 0; i < 3; ++i)
        if (!isfinite(c->t[i])) return fail(TGS_ERR_INVALID_ARG, "camera translation is not finite");
    if (!isfinite(c->cx) || !isfinite(c->cy)) return fail(TGS_ERR_INVALID_ARG, "principal point is not finite");
    return TGS_OK;
}

tgs_status check_params(const tgs_params* p) {
    if (!p) return fail(TGS_ERR_INVALID_ARG, "params is NULL");
    if (p->tile_size != 8 && p->tile_size != 16 && p->tile_size != 32)
        return fail(TGS_ERR_UNSUPPORTED, "tile_size %d (8, 16 or 32)", p->tile_size);
    if (p->num_bins < 1 || p->num_bins > 1024) return fail(TGS_ERR_INVALID_ARG, "num_bins %d outside 1..1024", p->num_bins);
    if (p->sample_count < 1 || p->sample_count > 8192)
        return fail(TGS_ERR_INVALID_ARG, "sample_count %d outside 1..8192", p->sample_count);
    if (!(p->p_lo >= 0.f && p->p_lo <= p->p_hi && p->p_hi <= 100.f))
        return fail(TGS_ERR_INVALID_ARG, "need 0 <= p_lo <= p_hi <= 100");
    if (!(p->pad >= 0.f) || !isfinite(p->pad)) return fail(TGS_ERR_INVALID_ARG, "pad must be >= 0");
    if (p->packed < 0 || p->packed > 2) return fail(TGS_ERR_INVALID_ARG, "packed must be 0, 1 or 2");
    if (p->raster != TGS_RASTER_PLAIN && p->raster != TGS_RASTER_WAVE)
        return fail(TGS_ERR_INVALID_ARG, "unknown raster %d", p->raster);
    if (p->tile_size != kTile && (p->raster == TGS_RASTER_PLAIN || p->packed != 0))
        return fail(TGS_ERR_UNSUPPORTED, "tile_size %d needs the WAVE raster with packed = 0", p->tile_size);
    if (p->per_tile_bins_dev) {
        if (p->num_bins & (p->num_bins - 1))
            return fail(TGS_ERR_INVALID_ARG, "num_bins %d must be a power of two with per_tile_bins", p->num_bins);
        if (p->packed != 0) return fail(TGS_ERR_UNSUPPORTED, "per_tile_bins needs packed = 0");
    }
    if (p->repair != TGS_REPAIR_ALL && p->repair != TGS_REPAIR_RULES && p->repair != TGS_REPAIR_NONE)
        return fail(TGS_ERR_INVALID_ARG, "unknown repair %d", p->repair);
    if (!(p->repair_budget >= 0.f && p->repair_budget <= 1.f))
        return fail(TGS_ERR_INVALID_ARG, "repair_budget must be in [0, 1]");
    if (p->repair != TGS_REPAIR_ALL && p->packed != 0)
        return fail(TGS_ERR_UNSUPPORTED, "repair RULES / NONE needs packed = 0");
    if (p->repair == TGS_REPAIR_RULES && p->per_tile_bins_dev)
        return fail(TGS_ERR_UNSUPPORTED, "repair RULES needs a uniform num_bins");
    if (p->near_shift != 0 && p->near_shift != 1) return fail(TGS_ERR_INVALID_ARG, "near_shift must be 0 or 1");
    if (p->split_entries != 0 &&
        (p->split_entries < 256 || p->split_entries > (1 << 24) || (p->split_entries & (p->split_entries - 1))))
        return fail(TGS_ERR_INVALID_ARG, "split_entries %d: 0 or a power of two in 256..2^24", p->split_entries);
    if (p->split_mean_factor < 0 || p->split_mean_factor > 64)
        return fail(TGS_ERR_INVALID_ARG, "split_mean_factor %d outside 0..64", p->split_mean_factor);
    if (!(p->shift_alpha >= 0.f) || !isfinite(p->shift_alpha))
        return fail(TGS_ERR_INVALID_ARG, "shift_alpha must be finite and >= 0");
    if (!(p->shift_gamma >= 0.f && p->shift_gamma < 1.f))
        return fail(TGS_ERR_INVALID_ARG, "shift_gamma must be in [0, 1)");
    if (p->footprint != TGS_FOOTPRINT_OPACITY_AWARE && p->footprint != TGS_FOOTPRINT_THREE_SIGMA)
        return fail(TGS_ERR_INVALID_ARG, "unknown footprint %d", p->footprint);
    if (p->sub_bins != 0 && p->sub_bins != 1 && p->sub_bins != 2 && p->sub_bins != 4 && p->sub_bins != 8)
        return fail(TGS_ERR_INVALID_ARG, "sub_bins %d (0, 1, 2, 4 or 8)", p->sub_bins);
    return TGS_OK;
}

tgs_status check_projected(const tgs_projected* pr) {
    if (!pr) return fail(TGS_ERR_INVALID_ARG, "projected is NULL");
    if (pr->n < 0 || pr->n >= (int64_t)1 << 31) return fail(TGS_ERR_INVALID_ARG, "n = %lld outside 0..2^31-1", (long long)pr->n);
    if (pr->n > 0 && (!pr->splats_dev || !pr->info_dev)) return fail(TGS_ERR_INVALID_ARG, "projected buffers are NULL");
    return TGS_OK;
}

inline size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
    size_t emit_off, vis_ids, zero, zero_words, status_emit_x, status_emit_y, status_bins, status_segs, status_sel,
        count,
        count_var, tile_seg, entry_rank, seg_lists, keys_in, vals_in, sort_tmp, sort_tmp_bytes, gcount, group_off,
        wgbase, tmp_pair, tmp_code, group_order, samples, ginfo, total;
    int64_t list_stride;  // entries per repair bucket list
    GroupMap gm;  // gm.G > 0: grouped binning
};

// Control words at the start of the zeroed region (uint32 offsets).
constexpr int kTicketEmit = 0;
constexpr int kTicketBins = 1;
constexpr int kTicketSegs = 2;
constexpr int kTicketSel = 3;
constexpr int kSelCtl = 4;  // 2 words: first rejected segment + 1, remaining budget
constexpr int kBucketCount = 16;
constexpr int kTileHist = 32;  // 66 words: histogram and cursors of the tile order
constexpr int kControlWords = 128;

int end_bit_for(int64_t T) {
    int b = 0;
    while (((int64_t)1 << b) < T) ++b;
    return 32 + (b > 0 ? b : 1);
}

// Workspace: [emit offsets][visible ids][zeroed region: control words,
// scan status words (with rule-based repair also those of the selection
// scan), then the group totals (grouped binning) or the per-XCD counts
// (uniform K, group shape out of range)] followed by, for BINNED, [depth
// samples] and then, grouped: [repair lists (uint2 {begin, length} entries
// with sub-bins)][group offsets][group order][workgroup slice bases]
// [grouped pairs][grouped codes] and, with per-tile bin counts, [tile
// segments][group info]; otherwise [entry ranks][repair lists] and, with
// per-tile bin counts, [per-XCD counts][tile segments]. GLOBAL: [unsorted
// keys][unsorted ids][sort scratch]. The zeroed region is cleared by one
// fill at the start of each tgs_bin; with per-tile bin counts only the
// first kCopies * S words of the counts are cleared, by a fill sized on the
// device. K is the uniform bin count or the bound of the per-tile counts.
// Sub-bins per bin of the grouped path: exact repair without records, and
// bins of the depth itself (the sub-bin order is the depth order only when
// the binning key is the sort key; the near-depth key is not).
int sub_bins_for(const tgs_params* p, int order) {
    const bool ok = order == TGS_ORDER_BINNED && p->repair == TGS_REPAIR_ALL && !p->packed && !p->near_shift;
    return ok ? (p->sub_bins > 0 ? p->sub_bins : kSubBins) : 1;
}

Layout layout(int64_t n, int64_t capacity, int64_t T, int K, int order, bool var, bool rules, int sub) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    const int64_t nseg = T * K;
    L.emit_off = take(sizeof(uint32_t) * (size_t)(n + 1));
    L.vis_ids = take(sizeof(uint32_t) * (size_t)(n + 1));
    // zeroed region, in uint32 words from L.zero
    size_t z = kControlWords;
    const size_t nbe = (size_t)scan_blocks(n), nbb = (size_t)scan_blocks(nseg);
    L.status_emit_x = z;
    z += 2 * nbe;
    L.status_emit_y = z;
    z += 2 * nbe;
    L.status_bins = z;
    z += 2 * nbb;
    L.status_segs = z;
    z += var ? 2 * (size_t)scan_blocks(T) : 0;
    L.status_sel = z;
    z += rules ? 2 * nbb : 0;
    L.gm = order != TGS_ORDER_BINNED ? GroupMap{K, 1, 0, 0, 1, T, nullptr, nullptr, nullptr}
           : var                     ? group_map_var(T, K, sub)
                                     : group_map(T, K, sub);
    const bool grouped = L.gm.G > 0;
    if (grouped) {
        z = (z + 63) & ~(size_t)63;
        L.gcount = z;
        z += (size_t)L.gm.G;
    } else if (order == TGS_ORDER_BINNED && !var) {
        z = (z + 63) & ~(size_t)63;
        L.count = z;
        z += (size_t)kCopies * (size_t)nseg;
    }
    L.zero_words = z;
    L.zero = take(sizeof(uint32_t) * z);
    if (order == TGS_ORDER_BINNED) L.samples = take(sizeof(uint32_t) * 8192);
    L.list_stride = nseg;
    if (grouped) {
        const size_t chunks = (size_t)((n + kGroupChunk - 1) / kGroupChunk);
        size_t entry = sizeof(uint32_t);
        if (L.gm.SB > 1) {
            // a queued sub-segment holds two or more of the at most capacity
            // entries; it is queued as {begin, length}
            L.list_stride = std::min<int64_t>(nseg * L.gm.SB, capacity / 2 + 1);
            entry = sizeof(uint2);
        }
        L.seg_lists = take(entry * (size_t)kBuckets * (size_t)L.list_stride);
        L.group_off = take(sizeof(uint32_t) * ((size_t)L.gm.G + 1));
        L.group_order = take(sizeof(uint32_t) * (size_t)L.gm.G);
        L.wgbase = take(sizeof(uint32_t) * (chunks > 0 ? chunks : 1) * (size_t)L.gm.G);
        L.tmp_pair = take(sizeof(uint64_t) * (size_t)capacity);
        L.tmp_code = take(sizeof(uint16_t) * (size_t)capacity);
        if (var) {
            L.tile_seg = take(sizeof(uint2) * (size_t)T);
            L.ginfo = take(sizeof(uint4) * (size_t)L.gm.G);
        }
    } else if (order == TGS_ORDER_BINNED) {
        L.entry_rank = take(sizeof(uint32_t) * (size_t)capacity);
        L.seg_lists = take(sizeof(uint32_t) * (size_t)kBuckets * (size_t)nseg);
        if (var) {
            L.count_var = take(sizeof(uint32_t) * (size_t)kCopies * (size_t)nseg);
            L.tile_seg = take(sizeof(uint2) * (size_t)T);
        }
    } else {
        L.keys_in = take(sizeof(uint64_t) * (size_t)capacity);
        L.vals_in = take(sizeof(uint32_t) * (size_t)capacity);
        L.sort_tmp_bytes = global_sort_tmp_bytes(capacity, end_bit_for(T + 1)) + 1024;
        L.sort_tmp = take(L.sort_tmp_bytes);
    }
    L.total = off;
    return L;
}

int64_t tiles_of(const tgs_camera* c, int tile) {
    return (int64_t)div_up(c->width, tile) * div_up(c->height, tile);
}

}  // namespace

extern "C" {

void tgs_default_params(tgs_params* p) {
    if (!p) return;
    p->tile_size = 16;
    p->num_bins = 64;
    p->sample_count = 8192;
    p->p_lo = 1.0f;
    p->p_hi = 99.0f;
    p->pad = 0.05f;
    p->raster = TGS_RASTER_WAVE;
    p->packed = 0;
    p->per_tile_bins_dev = nullptr;
    p->repair = TGS_REPAIR_ALL;
    p->repair_budget = 0.25f;
    p->near_shift = 0;
    p->shift_alpha = 1.0f;
    p->shift_gamma = 0.25f;
    p->split_entries = 2048;
    p->split_mean_factor = 2;
    p->footprint = TGS_FOOTPRINT_OPACITY_AWARE;
    p->sub_bins = 0;
}

const char* tgs_last_error(void) { return g_err.c_str(); }

tgs_status tgs_project(const tgs_gaussians* g, const tgs_camera* cam, const tgs_params* params, tgs_projected* out,
                       void* stream) {
    g_err.clear();
    if (!g) return fail(TGS_ERR_INVALID_ARG, "gaussians is NULL");
    if (g->n < 0 || g->n >= (int64_t)1 << 31) return fail(TGS_ERR_INVALID_ARG, "n = %lld outside 0..2^31-1", (long long)g->n);
    if (g->sh_degree < 0 || g->sh_degree > 3) return fail(TGS_ERR_INVALID_ARG, "sh_degree %d outside 0..3", g->sh_degree);
    if (g->n > 0 && (!g->means_dev || !g->log_scales_dev || !g->quats_dev || !g->logits_dev || !g->sh_dev))
        return fail(TGS_ERR_INVALID_ARG, "a Gaussian attribute pointer is NULL");
    tgs_status st = check_camera(cam);
    if (st) return st;
    if ((st = check_params(params))) return st;
    if (!out || out->n != g->n) return fail(TGS_ERR_INVALID_ARG, "projected output missing or n mismatch");
    if (g->n > 0 && (!out->splats_dev || !out->info_dev)) return fail(TGS_ERR_INVALID_ARG, "projected buffers are NULL");
    TGS_HIP(launch_project(*g, make_cam(*cam, params->tile_size, params->footprint), out->splats_dev, out->info_dev, (hipStream_t)stream),
            "project");
    return TGS_OK;
}

tgs_status tgs_project_views(const tgs_gaussians* g, int32_t num_views, const tgs_camera* cams,
                             const tgs_params* params, tgs_projected* out, void* stream) {
    g_err.clear();
    if (!g) return fail(TGS_ERR_INVALID_ARG, "gaussians is NULL");
    if (g->n < 0 || g->n >= (int64_t)1 << 31) return fail(TGS_ERR_INVALID_ARG, "n = %lld outside 0..2^31-1", (long long)g->n);
    if (g->sh_degree < 0 || g->sh_degree > 3) return fail(TGS_ERR_INVALID_ARG, "sh_degree %d outside 0..3", g->sh_degree);
    if (g->n > 0 && (!g->means_dev || !g->log_scales_dev || !g->quats_dev || !g->logits_dev || !g->sh_dev))
        return fail(TGS_ERR_INVALID_ARG, "a Gaussian attribute pointer is NULL");
    if (num_views < 1 || num_views > TGS_MAX_VIEWS)
        return fail(TGS_ERR_INVALID_ARG, "num_views %d outside 1..%d", num_views, TGS_MAX_VIEWS);
    if (!cams || !params || !out) return fail(TGS_ERR_INVALID_ARG, "an argument array is NULL");
    for (int v = 0; v < num_views; ++v) {
        tgs_status st = check_camera(&cams[v]);
        if (st) return st;
        if ((st = check_params(&params[v]))) return st;
        if (out[v].n != g->n) return fail(TGS_ERR_INVALID_ARG, "view %d: projected n mismatch", v);
        if (g->n > 0 && (!out[v].splats_dev || !out[v].info_dev))
            return fail(TGS_ERR_INVALID_ARG, "view %d: projected buffers are NULL", v);
    }
    for (int v0 = 0; v0 < num_views; v0 += kProjViews) {
        ProjViews pv{};
        pv.nv = std::min(kProjViews, num_views - v0);
        for (int k = 0; k < pv.nv; ++k) {
            pv.cam[k] = make_cam(cams[v0 + k], params[v0 + k].tile_size, params[v0 + k].footprint);
            pv.splats[k] = reinterpret_cast<float4*>(out[v0 + k].splats_dev);
            pv.info[k] = reinterpret_cast<uint4*>(out[v0 + k].info_dev);
        }
        TGS_HIP(launch_project_views(*g, pv, (hipStream_t)stream), "project views");
    }
    return TGS_OK;
}

size_t tgs_bin_workspace_size(int64_t n, int64_t capacity, const tgs_camera* cam, const tgs_params* params,
                              int32_t order) {
    if (!cam || !params || n < 0 || capacity < 0) return 0;
    if (cam->width < 1 || cam->height < 1 || params->num_bins < 1) return 0;
    if (params->tile_size != 8 && params->tile_size != 16 && params->tile_size != 32) return 0;
    return layout(n, capacity, tiles_of(cam, params->tile_size), params->num_bins, order,
                  params->per_tile_bins_dev != nullptr && order == TGS_ORDER_BINNED,
                  params->repair == TGS_REPAIR_RULES && order == TGS_ORDER_BINNED, sub_bins_for(params, order))
        .total;
}

tgs_status tgs_bin(const tgs_projected* pr, const tgs_camera* cam, const tgs_params* params, int32_t order, void* ws,
                   size_t ws_bytes, tgs_binned* out, int64_t* num_entries_host, void* stream) {
    g_err.clear();
    tgs_status st = check_projected(pr);
    if (st) return st;
    if ((st = check_camera(cam))) return st;
    if ((st = check_params(params))) return st;
    if (order != TGS_ORDER_GLOBAL && order != TGS_ORDER_BINNED) return fail(TGS_ERR_INVALID_ARG, "unknown order %d", order);
    if (!out) return fail(TGS_ERR_INVALID_ARG, "binned output is NULL");
    if (out->capacity < 0 || out->capacity >= ((int64_t)1 << 32)) return fail(TGS_ERR_INVALID_ARG, "capacity outside 0..2^32-1");
    if (!out->counters_dev || !out->offsets_dev) return fail(TGS_ERR_INVALID_ARG, "counters or offsets is NULL");
    const int64_t n = pr->n, cap = out->capacity, T = tiles_of(cam, params->tile_size);
    const int K = params->num_bins;
    const bool var = params->per_tile_bins_dev != nullptr;
    if (var && order != TGS_ORDER_BINNED) return fail(TGS_ERR_INVALID_ARG, "per_tile_bins needs the BINNED order");
    if (var && !out->seg_base_dev) return fail(TGS_ERR_INVALID_ARG, "seg_base is NULL with per_tile_bins");
    if (order == TGS_ORDER_BINNED) {
        if (!out->zrange_dev || (cap > 0 && !out->pairs_dev)) return fail(TGS_ERR_INVALID_ARG, "pairs or zrange is NULL");
        if (params->packed == 1 && cap > 0 && (!out->records_dev || !out->masks_dev))
            return fail(TGS_ERR_INVALID_ARG, "records or masks is NULL with packed=1");
        if (params->packed == 2 && cap > 0 && !out->masks_dev)
            return fail(TGS_ERR_INVALID_ARG, "masks is NULL with packed=2");
        if (T * K >= ((int64_t)1 << 31)) return fail(TGS_ERR_INVALID_ARG, "tiles * bins too large");
    } else if (cap > 0 && (!out->keys_dev || !out->vals_dev)) {
        return fail(TGS_ERR_INVALID_ARG, "keys or vals is NULL");
    }
    const bool rules = order == TGS_ORDER_BINNED && params->repair == TGS_REPAIR_RULES;
    const Layout L = layout(n, cap, T, K, order, var, rules, sub_bins_for(params, order));
    if (!ws || ws_bytes < L.total)
        return fail(TGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(TGS_ERR_WORKSPACE, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)ws;
    uint32_t* emit_off = (uint32_t*)(w + L.emit_off);
    uint32_t* vis_ids = (uint32_t*)(w + L.vis_ids);
    uint32_t* zero = (uint32_t*)(w + L.zero);
    const int S = params->sample_count;
    const int tiles_x = div_up(cam->width, params->tile_size), tiles_y = div_up(cam->height, params->tile_size);

    TGS_HIP(launch_fill_u32(zero, 0u, (int64_t)L.zero_words, s), "clear control words");
    TGS_HIP(launch_emit_scan(pr->info_dev, n, tiles_x, tiles_y, emit_off, vis_ids, zero + kTicketEmit,
                             (uint64_t*)(zero + L.status_emit_x), (uint64_t*)(zero + L.status_emit_y),
                             out->counters_dev, cap, s),
            "emit scan");
    int64_t M = -1;
    if (num_entries_host) {
        TGS_HIP(hipMemcpyAsync(&M, out->counters_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s), "read entry count");
        TGS_HIP(hipStreamSynchronize(s), "read entry count");
        if (num_entries_host) *num_entries_host = M;
        if (M > cap) return fail(TGS_ERR_CAPACITY, "%lld entries exceed the capacity %lld", (long long)M, (long long)cap);
    }
    if (order == TGS_ORDER_GLOBAL) {
        uint64_t* keys_in = (uint64_t*)(w + L.keys_in);
        uint32_t* vals_in = (uint32_t*)(w + L.vals_in);
        TGS_HIP(launch_emit_keys(pr->info_dev, n, emit_off, tiles_x, tiles_y, keys_in, vals_in, cap, s), "emit keys");
        // without the host count: sort every slot, the unused ones padded
        // with keys past the last tile
        int64_t sort_n = M;
        int end_bit = end_bit_for(T);
        if (M < 0) {
            TGS_HIP(launch_pad_keys(keys_in, vals_in, out->counters_dev, cap, T, s), "pad keys");
            sort_n = cap;
            end_bit = end_bit_for(T + 1);
        }
        TGS_HIP(launch_global_sort(w + L.sort_tmp, L.sort_tmp_bytes, keys_in, out->keys_dev, vals_in, out->vals_dev,
                                   sort_n, end_bit, s),
                "radix sort");
        TGS_HIP(launch_tile_ranges(out->keys_dev, sort_n, T, out->offsets_dev, s), "tile ranges");
        if (out->tile_order_dev)
            TGS_HIP(launch_tile_order(out->offsets_dev, SegMap{nullptr, 1, nullptr}, T, zero + kTileHist,
                                      out->tile_order_dev, params->split_entries, params->split_mean_factor, s),
                    "tile order");
        return TGS_OK;
    }
    uint32_t* count = var ? (uint32_t*)(w + L.count_var) : zero + L.count;
    uint2* tile_seg = var ? (uint2*)(w + L.tile_seg) : nullptr;
    const SegMap sm{var ? out->seg_base_dev : nullptr, K, tile_seg};
    const uint32_t* nseg_dev = var ? out->seg_base_dev + T : nullptr;
    uint32_t* entry_rank = (uint32_t*)(w + L.entry_rank);
    uint32_t* seg_lists = (uint32_t*)(w + L.seg_lists);
    uint32_t* bucket_count = zero + kBucketCount;
    const int64_t nseg = T * K;
    RecordSink rs{reinterpret_cast<const float4*>(pr->splats_dev),
                  params->packed == 1 ? reinterpret_cast<float4*>(out->records_dev) : nullptr,
                  params->packed ? out->masks_dev : nullptr, K, tiles_x, cam->width, cam->height};
    if (var) {
        TGS_HIP(launch_seg_base(params->per_tile_bins_dev, T, K, out->seg_base_dev, tile_seg, zero + kTicketSegs,
                                (uint64_t*)(zero + L.status_segs), s),
                "segment bases");
        if (L.gm.G == 0)
            TGS_HIP(launch_fill_u32_dyn(count, 0u, nseg_dev, kCopies, (int64_t)kCopies * nseg, s), "clear counts");
    }
    const float zn = (float)cam->znear, zf = (float)cam->zfar;
    const NearKey nk{params->near_shift ? reinterpret_cast<const float4*>(pr->splats_dev) : nullptr,
                     params->shift_alpha, params->shift_gamma, zn > 1e-4f ? zn : 1e-4f, zf};
    if (L.gm.G > 0) {
        GroupMap gm = L.gm;
        if (var) {
            gm.seg_base = out->seg_base_dev;
            gm.tile_seg = tile_seg;
            gm.ginfo = (uint4*)(w + L.ginfo);
        }
        uint32_t* gcount = zero + L.gcount;
        uint32_t* group_off = (uint32_t*)(w + L.group_off);
        uint32_t* wgbase = (uint32_t*)(w + L.wgbase);
        uint64_t* tmp_pair = (uint64_t*)(w + L.tmp_pair);
        uint16_t* tmp_code = (uint16_t*)(w + L.tmp_code);
        uint32_t* group_order = (uint32_t*)(w + L.group_order);
        const RangeArgs ra{vis_ids, out->counters_dev, nk, S, params->p_lo, params->p_hi, params->pad, zn, zf,
                           out->zrange_dev, (uint32_t*)(w + L.samples)};
        TGS_HIP(launch_group_count(pr->info_dev, n, emit_off, gm, tiles_x, tiles_y, gcount, wgbase, ra, s),
                "depth range and group count");
        TGS_HIP(launch_group_scan(gcount, gm, group_off, group_order, s), "group scan");
        TGS_HIP(launch_group_scatter(pr->info_dev, n, emit_off, out->zrange_dev, nk, gm, tiles_x, tiles_y, group_off,
                                     wgbase, tmp_pair, tmp_code, cap, s),
                "group scatter");
        // the group sort adds the tile-order histogram; the placement rides on
        // the repair's long-segment launch
        const TileOrder to{out->offsets_dev, sm, T, zero + kTileHist, out->tile_order_dev, params->split_entries,
                           params->split_mean_factor};
        TGS_HIP(launch_group_sort(tmp_pair, tmp_code, group_off, group_order, gm, nseg, cap, out->pairs_dev,
                                  out->offsets_dev, seg_lists, L.list_stride, bucket_count, out->counters_dev,
                                  params->repair == TGS_REPAIR_ALL, out->repaired_dev, rs,
                                  to.order ? to.hist : nullptr, s),
                "group sort");
        if (rules)
            TGS_HIP(launch_repair_select(out->offsets_dev, T, K, params->repair_budget, zero + kTicketSel,
                                         (uint64_t*)(zero + L.status_sel), zero + kSelCtl, seg_lists, bucket_count,
                                         out->counters_dev, out->repaired_dev, s),
                    "repair selection");
        // with sub-bins the queues hold sub-segment descriptors
        if (params->repair != TGS_REPAIR_NONE)
            TGS_HIP(launch_repair(out->offsets_dev, L.list_stride, out->pairs_dev, seg_lists, bucket_count, rs,
                                  gm.SB > 1, to, s),
                    "repair and tile order");
        else
            TGS_HIP(launch_tile_place(to, s), "tile order");
        return TGS_OK;
    }
    TGS_HIP(launch_depth_range(pr->info_dev, vis_ids, out->counters_dev, nk, S, params->p_lo, params->p_hi,
                               params->pad, zn, zf, out->zrange_dev, (uint32_t*)(w + L.samples), s),
            "depth range");
    TGS_HIP(launch_bin_count(pr->info_dev, n, emit_off, out->zrange_dev, nk, sm, tiles_x, tiles_y, count, nseg,
                             entry_rank, cap, s),
            "bin count");
    TGS_HIP(launch_bin_offsets(count, nseg, nseg_dev, out->offsets_dev, zero + kTicketBins,
                               (uint64_t*)(zero + L.status_bins), seg_lists, bucket_count, out->counters_dev,
                               params->repair == TGS_REPAIR_ALL, out->repaired_dev, s),
            "bin offsets");
    if (rules)
        TGS_HIP(launch_repair_select(out->offsets_dev, T, K, params->repair_budget, zero + kTicketSel,
                                     (uint64_t*)(zero + L.status_sel), zero + kSelCtl, seg_lists, bucket_count,
                                     out->counters_dev, out->repaired_dev, s),
                "repair selection");
    TGS_HIP(launch_bin_scatter(pr->info_dev, n, emit_off, out->zrange_dev, nk, sm, tiles_x, tiles_y, out->offsets_dev,
                               count, nseg, entry_rank, out->pairs_dev, cap, rs, s),
            "bin scatter");
    if (params->repair != TGS_REPAIR_NONE)
        TGS_HIP(launch_repair(out->offsets_dev, nseg, out->pairs_dev, seg_lists, bucket_count, rs, false, TileOrder{},
                              s),
                "repair");
    if (out->tile_order_dev)
        TGS_HIP(launch_tile_order(out->offsets_dev, sm, T, zero + kTileHist, out->tile_order_dev,
                                  params->split_entries, params->split_mean_factor, s),
                "tile order");
    return TGS_OK;
}

tgs_status tgs_rasterize(const tgs_projected* pr, const tgs_binned* b, const tgs_camera* cam, const tgs_params* params,
                         int32_t order, const float* bg, float* rgb, float* alpha, int32_t* last, int32_t* n_contrib,
                         int32_t* n_visit, int32_t* n_support, float* trans, void* stream) {
    g_err.clear();
    tgs_status st = check_projected(pr);
    if (st) return st;
    if ((st = check_camera(cam))) return st;
    if ((st = check_params(params))) return st;
    if (order != TGS_ORDER_GLOBAL && order != TGS_ORDER_BINNED) return fail(TGS_ERR_INVALID_ARG, "unknown order %d", order);
    if (!b || !b->offsets_dev || !b->counters_dev) return fail(TGS_ERR_INVALID_ARG, "binned buffers are NULL");
    if (!bg || !rgb || !alpha || !last) return fail(TGS_ERR_INVALID_ARG, "an output pointer is NULL");
    RasterArgs a{};
    a.splats = pr->splats_dev;
    a.offsets = b->offsets_dev;
    a.counters = b->counters_dev;
    a.order = b->tile_order_dev;
    if (order == TGS_ORDER_GLOBAL) {
        a.stride = 1;
        a.vals = b->vals_dev;
        if (!a.vals && b->capacity > 0) return fail(TGS_ERR_INVALID_ARG, "vals is NULL");
    } else {
        a.stride = params->num_bins;
        a.seg_base = params->per_tile_bins_dev ? b->seg_base_dev : nullptr;
        if (params->per_tile_bins_dev && !a.seg_base) return fail(TGS_ERR_INVALID_ARG, "seg_base is NULL with per_tile_bins");
        a.pairs = b->pairs_dev;
        a.records = params->packed == 1 ? b->records_dev : nullptr;
        a.masks = params->packed ? b->masks_dev : nullptr;
        if (b->capacity > 0 && !a.pairs) return fail(TGS_ERR_INVALID_ARG, "pairs is NULL");
        if (params->packed == 1 && b->capacity > 0 && !a.records)
            return fail(TGS_ERR_INVALID_ARG, "records or masks is NULL");
        if (params->packed && b->capacity > 0 && !a.masks) return fail(TGS_ERR_INVALID_ARG, "records or masks is NULL");
    }
    if (pr->n > 0 && !a.splats && !a.records) return fail(TGS_ERR_INVALID_ARG, "splats is NULL");
    a.width = cam->width;
    a.height = cam->height;
    a.tile = params->tile_size;
    a.tiles_x = div_up(cam->width, params->tile_size);
    a.tiles_y = div_up(cam->height, params->tile_size);
    for (int i = 0; i < 3; ++i) a.bg[i] = bg[i];
    a.rgb = rgb;
    a.alpha = alpha;
    a.last = last;
    a.n_contrib = n_contrib;
    a.n_visit = n_visit;
    a.n_support = n_support;
    a.trans = trans;
    a.split = params->split_entries;
    if (trans && params->raster != TGS_RASTER_WAVE) return fail(TGS_ERR_UNSUPPORTED, "trans needs the WAVE raster");
    hipStream_t s = (hipStream_t)stream;
    if (params->raster == TGS_RASTER_PLAIN)
        TGS_HIP(launch_raster_plain(a, s), "raster");
    else
        TGS_HIP(launch_raster_wave(a, s), "raster");
    return TGS_OK;
}

tgs_status tgs_rasterize_backward(const tgs_projected* pr, const tgs_binned* b, const tgs_camera* cam,
                                  const tgs_params* params, int32_t order, const float* bg, const float* d_rgb,
                                  const float* d_alpha, const float* trans_in, const int32_t* last_in,
                                  float* d_splats, void* stream) {
    g_err.clear();
    tgs_status st = check_projected(pr);
    if (st) return st;
    if ((st = check_camera(cam))) return st;
    if ((st = check_params(params))) return st;
    if (order != TGS_ORDER_GLOBAL && order != TGS_ORDER_BINNED) return fail(TGS_ERR_INVALID_ARG, "unknown order %d", order);
    if (!b || !b->offsets_dev || !b->counters_dev) return fail(TGS_ERR_INVALID_ARG, "binned buffers are NULL");
    if (!bg || !d_rgb) return fail(TGS_ERR_INVALID_ARG, "bg or d_rgb is NULL");
    if (pr->n > 0 && !d_splats) return fail(TGS_ERR_INVALID_ARG, "d_splats is NULL");
    if ((trans_in == nullptr) != (last_in == nullptr))
        return fail(TGS_ERR_INVALID_ARG, "give both trans and last, or neither");
    RasterArgs a{};
    a.splats = pr->splats_dev;
    a.offsets = b->offsets_dev;
    a.counters = b->counters_dev;
    a.order = b->tile_order_dev;
    if (order == TGS_ORDER_GLOBAL) {
        a.stride = 1;
        a.vals = b->vals_dev;
        if (!a.vals && b->capacity > 0) return fail(TGS_ERR_INVALID_ARG, "vals is NULL");
    } else {
        a.stride = params->num_bins;
        a.seg_base = params->per_tile_bins_dev ? b->seg_base_dev : nullptr;
        if (params->per_tile_bins_dev && !a.seg_base) return fail(TGS_ERR_INVALID_ARG, "seg_base is NULL with per_tile_bins");
        a.pairs = b->pairs_dev;
        if (!a.pairs && b->capacity > 0) return fail(TGS_ERR_INVALID_ARG, "pairs is NULL");
    }
    a.width = cam->width;
    a.height = cam->height;
    a.tile = params->tile_size;
    a.tiles_x = div_up(cam->width, params->tile_size);
    a.tiles_y = div_up(cam->height, params->tile_size);
    for (int i = 0; i < 3; ++i) a.bg[i] = bg[i];
    hipStream_t s = (hipStream_t)stream;
    if (pr->n == 0) return TGS_OK;
    TGS_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(d_splats), 0u, pr->n * kGradWords, s), "fill");
    TGS_HIP(launch_raster_backward(a, d_rgb, d_alpha, trans_in, last_in, d_splats, s), "raster backward");
    return TGS_OK;
}

tgs_status tgs_project_backward(const tgs_gaussians* g, const tgs_camera* cam, const float* d_splats,
                                tgs_gaussian_grads* out, void* stream) {
    g_err.clear();
    if (!g) return fail(TGS_ERR_INVALID_ARG, "gaussians is NULL");
    if (g->n < 0 || g->n >= (int64_t)1 << 31) return fail(TGS_ERR_INVALID_ARG, "n = %lld outside 0..2^31-1", (long long)g->n);
    if (g->sh_degree < 0 || g->sh_degree > 3) return fail(TGS_ERR_INVALID_ARG, "sh_degree %d outside 0..3", g->sh_degree);
    if (g->n > 0 && (!g->means_dev || !g->log_scales_dev || !g->quats_dev || !g->logits_dev || !g->sh_dev))
        return fail(TGS_ERR_INVALID_ARG, "a Gaussian attribute pointer is NULL");
    tgs_status st = check_camera(cam);
    if (st) return st;
    if (!out) return fail(TGS_ERR_INVALID_ARG, "grads is NULL");
    if (g->n > 0 && (!d_splats || !out->means_dev || !out->log_scales_dev || !out->quats_dev || !out->logits_dev ||
                     !out->sh_dev))
        return fail(TGS_ERR_INVALID_ARG, "a gradient pointer is NULL");
    TGS_HIP(launch_project_backward(*g, make_cam(*cam, kTile, TGS_FOOTPRINT_OPACITY_AWARE), d_splats, *out, (hipStream_t)stream), "project backward");
    return TGS_OK;
}

size_t tgs_batch_workspace_size(int32_t num_views, const tgs_camera* cams, const tgs_params* params) {
    if (num_views < 1 || num_views > kMaxViews || !cams || !params) return 0;
    int64_t blocks = 0;
    for (int v = 0; v < num_views; ++v) {
        const int ts = params[v].tile_size;
        if (ts != 8 && ts != 16 && ts != 32) return 0;
        if (cams[v].width < 1 || cams[v].height < 1) return 0;
        blocks += tiles_of(&cams[v], ts) * (int64_t)((ts / 8) * (ts / 8));
    }
    return sizeof(uint32_t) * (size_t)(256 + 8 * ((blocks + 7) / 8));
}

}  // extern "C"

// Fixed scratch of tgs_rasterize_batch_noalloc: the batch control words and
// work list (tgs_batch_workspace_size bytes) of up to about one million 8x8
// blocks, e.g. 16 views of 3840x2160 (2.1M pixels each). Every device the
// library runs on holds its own copy until the process ends. In host code
// `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, once per device (scratch_on_current_device).
static constexpr size_t kScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) uint32_t scratch[kScratchBytes / sizeof(uint32_t)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_dev_mu;
void* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device
int g_batch_grid[kMaxDevices] = {};     // persistent-raster workgroups, per device

tgs_status current_device(int* dev) {
    TGS_HIP(hipGetDevice(dev), "current device");
    if (*dev < 0 || *dev >= kMaxDevices) return fail(TGS_ERR_UNSUPPORTED, "device index %d >= %d", *dev, kMaxDevices);
    return TGS_OK;
}

// Workgroups of the persistent raster on the current device: 8 per CU.
tgs_status batch_grid(int* grid) {
    int dev = 0;
    tgs_status st = current_device(&dev);
    if (st) return st;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (g_batch_grid[dev] == 0) {
        int cus = 0;
        TGS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device attributes");
        g_batch_grid[dev] = (cus > 0 ? cus : 1) * 8;
    }
    *grid = g_batch_grid[dev];
    return TGS_OK;
}

// Device address of the current device's copy of `scratch` (looked up on
// the first call on each device, with that device current).
tgs_status scratch_on_current_device(void** out) {
    int dev = 0;
    tgs_status st = current_device(&dev);
    if (st) return st;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        TGS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
        if (!p) return fail(TGS_ERR_HIP, "scratch address: null");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return TGS_OK;
}

// Checks the views and fills the kernel arguments of a batched raster;
// blocks = the 8x8 blocks of all views.
tgs_status batch_args(int32_t num_views, const tgs_projected* pr, const tgs_binned* b, const tgs_camera* cams,
                      const tgs_params* params, const int32_t* orders, const float* bg, float* const* rgb,
                      float* const* alpha, int32_t* const* last, BatchArgs& a, int64_t& blocks) {
    if (num_views < 1 || num_views > kMaxViews) return fail(TGS_ERR_INVALID_ARG, "num_views %d outside 1..%d", num_views, kMaxViews);
    if (!pr || !b || !cams || !params || !orders || !bg || !rgb || !alpha || !last)
        return fail(TGS_ERR_INVALID_ARG, "an argument array is NULL");
    a = BatchArgs{};
    a.nv = num_views;
    for (int i = 0; i < 3; ++i) a.bg[i] = bg[i];
    int64_t tiles = 0;
    blocks = 0;
    for (int v = 0; v < num_views; ++v) {
        tgs_status st = check_projected(&pr[v]);
        if (st) return st;
        if ((st = check_camera(&cams[v]))) return st;
        if ((st = check_params(&params[v]))) return st;
        if (orders[v] != TGS_ORDER_GLOBAL && orders[v] != TGS_ORDER_BINNED)
            return fail(TGS_ERR_INVALID_ARG, "view %d: unknown order %d", v, orders[v]);
        if (!b[v].offsets_dev || !b[v].counters_dev) return fail(TGS_ERR_INVALID_ARG, "view %d: binned buffers are NULL", v);
        if (!rgb[v] || !alpha[v] || !last[v]) return fail(TGS_ERR_INVALID_ARG, "view %d: an output pointer is NULL", v);
        if (pr[v].n > 0 && !pr[v].splats_dev) return fail(TGS_ERR_INVALID_ARG, "view %d: splats is NULL", v);
        BatchView& d = a.v[v];
        const int ts = params[v].tile_size;
        d.splats = pr[v].splats_dev;
        d.offsets = b[v].offsets_dev;
        d.counters = b[v].counters_dev;
        if (orders[v] == TGS_ORDER_GLOBAL) {
            d.stride = 1;
            d.vals = b[v].vals_dev;
            if (!d.vals && b[v].capacity > 0) return fail(TGS_ERR_INVALID_ARG, "view %d: vals is NULL", v);
        } else {
            d.stride = params[v].num_bins;
            d.seg_base = params[v].per_tile_bins_dev ? b[v].seg_base_dev : nullptr;
            if (params[v].per_tile_bins_dev && !d.seg_base)
                return fail(TGS_ERR_INVALID_ARG, "view %d: seg_base is NULL with per_tile_bins", v);
            d.pairs = b[v].pairs_dev;
            if (!d.pairs && b[v].capacity > 0) return fail(TGS_ERR_INVALID_ARG, "view %d: pairs is NULL", v);
        }
        d.width = cams[v].width;
        d.height = cams[v].height;
        d.tile = ts;
        d.tiles_x = div_up(cams[v].width, ts);
        d.tiles_y = div_up(cams[v].height, ts);
        d.rgb = rgb[v];
        d.alpha = alpha[v];
        d.last = last[v];
        a.tile_base[v] = (uint32_t)tiles;
        tiles += (int64_t)d.tiles_x * d.tiles_y;
        blocks += (int64_t)d.tiles_x * d.tiles_y * ((ts / 8) * (ts / 8));
    }
    if (tiles >= ((int64_t)1 << 31) || blocks >= ((int64_t)1 << 32)) return fail(TGS_ERR_INVALID_ARG, "too many tiles");
    a.tile_base[num_views] = (uint32_t)tiles;
    return TGS_OK;
}

// Enqueues the batched raster with its control words and work list in ws
// (at least tgs_batch_workspace_size bytes, 256-byte aligned): a fill kernel
// clears the control words, then the two ordering launches and the
// persistent launch.
tgs_status batch_launch(const BatchArgs& a, int64_t blocks, void* ws, void* stream) {
    int grid = 0;
    tgs_status st = batch_grid(&grid);
    if (st) return st;
    const int64_t want = (blocks + 3) / 4;
    const int g = (int)(want < grid ? want : grid);
    hipStream_t s = (hipStream_t)stream;
    uint32_t* ctl = (uint32_t*)ws;
    TGS_HIP(launch_fill_u32(ctl, 0u, 256, s), "clear batch control words");
    TGS_HIP(launch_raster_batch(a, ctl, ctl + 256, blocks, g > 0 ? g : 1, s), "batched raster");
    return TGS_OK;
}

}  // namespace

extern "C" {

tgs_status tgs_rasterize_batch(int32_t num_views, const tgs_projected* pr, const tgs_binned* b,
                               const tgs_camera* cams, const tgs_params* params, const int32_t* orders,
                               const float* bg, float* const* rgb, float* const* alpha, int32_t* const* last,
                               void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    BatchArgs a{};
    int64_t blocks = 0;
    tgs_status st = batch_args(num_views, pr, b, cams, params, orders, bg, rgb, alpha, last, a, blocks);
    if (st) return st;
    const size_t need = tgs_batch_workspace_size(num_views, cams, params);
    if (!ws || ws_bytes < need) return fail(TGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(TGS_ERR_WORKSPACE, "workspace not 256-byte aligned");
    return batch_launch(a, blocks, ws, stream);
}

tgs_status tgs_rasterize_batch_noalloc(int32_t num_views, const tgs_projected* pr, const tgs_binned* b,
                                       const tgs_camera* cams, const tgs_params* params, const int32_t* orders,
                                       const float* bg, float* const* rgb, float* const* alpha,
                                       int32_t* const* last, void* stream) {
    g_err.clear();
    BatchArgs a{};
    int64_t blocks = 0;
    tgs_status st = batch_args(num_views, pr, b, cams, params, orders, bg, rgb, alpha, last, a, blocks);
    if (st) return st;
    const size_t need = tgs_batch_workspace_size(num_views, cams, params);
    if (need > kScratchBytes)
        return fail(TGS_ERR_WORKSPACE,
                    "tgs_rasterize_batch_noalloc: these views need %zu bytes of scratch (%lld 8x8 blocks), the "
                    "fixed scratch holds %zu; use tgs_rasterize_batch with a workspace",
                    need, (long long)blocks, kScratchBytes);
    void* ws = nullptr;
    if ((st = scratch_on_current_device(&ws))) return st;
    return batch_launch(a, blocks, ws, stream);
}

tgs_status tgs_tile_features(const tgs_binned* b, const tgs_camera* cam, const tgs_params* params, float* features,
                             void* stream) {
    g_err.clear();
    tgs_status st = check_camera(cam);
    if (st) return st;
    if ((st = check_params(params))) return st;
    if (!b || !b->offsets_dev || !b->counters_dev) return fail(TGS_ERR_INVALID_ARG, "binned buffers are NULL");
    if (!features) return fail(TGS_ERR_INVALID_ARG, "features is NULL");
    if (params->per_tile_bins_dev && !b->seg_base_dev)
        return fail(TGS_ERR_INVALID_ARG, "seg_base is NULL with per_tile_bins");
    const SegMap sm{params->per_tile_bins_dev ? b->seg_base_dev : nullptr, params->num_bins, nullptr};
    TGS_HIP(launch_tile_features(b->offsets_dev, sm, tiles_of(cam, params->tile_size), b->counters_dev, features,
                                 (hipStream_t)stream),
            "tile features");
    return TGS_OK;
}

tgs_status tgs_propose_bins(const float* weights, const float* features, int64_t num_tiles, int32_t fallback_bins,
                            int32_t* per_tile_bins, float* logits, void* stream) {
    g_err.clear();
    if (num_tiles < 0 || num_tiles >= ((int64_t)1 << 31)) return fail(TGS_ERR_INVALID_ARG, "num_tiles outside 0..2^31-1");
    if (num_tiles > 0 && (!weights || !features || !per_tile_bins))
        return fail(TGS_ERR_INVALID_ARG, "weights, features or per_tile_bins is NULL");
    if (fallback_bins < 1 || fallback_bins > 1024) return fail(TGS_ERR_INVALID_ARG, "fallback_bins outside 1..1024");
    TGS_HIP(launch_propose(weights, features, num_tiles, per_tile_bins, logits, fallback_bins, (hipStream_t)stream),
            "bin proposal");
    return TGS_OK;
}

size_t tgs_mlp_train_workspace_size(int64_t num_tiles) {
    if (num_tiles < 0) return 0;
    return sizeof(float) * mlp_train_workspace_floats(num_tiles);
}

tgs_status tgs_mlp_train_step(float* weights, float* velocity, const float* features, const float* regret,
                              int64_t num_tiles, float lr, float momentum, void* ws, size_t ws_bytes, float* loss,
                              void* stream) {
    g_err.clear();
    if (num_tiles < 0 || num_tiles >= ((int64_t)1 << 31)) return fail(TGS_ERR_INVALID_ARG, "num_tiles outside 0..2^31-1");
    if (!weights || !velocity) return fail(TGS_ERR_INVALID_ARG, "weights or velocity is NULL");
    if (num_tiles > 0 && (!features || !regret)) return fail(TGS_ERR_INVALID_ARG, "features or regret is NULL");
    if (!isfinite(lr) || !isfinite(momentum)) return fail(TGS_ERR_INVALID_ARG, "lr and momentum must be finite");
    const size_t need = tgs_mlp_train_workspace_size(num_tiles);
    if (!ws || ws_bytes < need) return fail(TGS_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(TGS_ERR_WORKSPACE, "workspace not 256-byte aligned");
    TGS_HIP(launch_mlp_train_step(weights, velocity, features, regret, num_tiles, lr, momentum, (float*)ws, loss,
                                  (hipStream_t)stream),
            "network training step");
    return TGS_OK;
}

}  // extern "C"
