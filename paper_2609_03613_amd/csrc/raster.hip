// Front-to-back alpha compositing of each 16x16 tile's one contiguous entry
// range (supplement, Algorithm "Binned raster traversal after repair"; the
// per-pixel test and update are the baseline's, unchanged).
//
// Two kernels with bit-identical per-pixel arithmetic:
//
// raster_plain  The baseline's structure: one 256-lane workgroup per tile,
//               lane = pixel; batches of 256 entries are gathered by Gaussian
//               id into LDS, every lane walks every batch entry, and the
//               workgroup leaves when all 256 pixels have terminated.
//
// raster_wave   The binned path's kernel. Each 64-lane wavefront owns one
//               8x8 pixel block of the tile and walks the tile range on its
//               own, 64 entries at a time. An entry survives for the block
//               when a conservative bound says its splat can reach alpha
//               1/255 at some pixel centre of the block (the tile alpha cull
//               of the paper's binned kernel, at block granularity): with
//               packed records the bound was evaluated once per entry when
//               the record was written (a 4-bit block mask), otherwise each
//               wavefront evaluates it on the gathered splat. Survivors are
//               compacted into wavefront-private LDS by ballot + prefix count
//               (colour staging) and composited by all lanes; a wavefront
//               exits when all its pixels have terminated, without workgroup
//               barriers. Culled entries are exactly those whose alpha test
//               fails at every pixel of the block, so images, last ids and
//               contribution counts are unchanged.
#include <math.h>

#include "common.hpp"

namespace tgs {

namespace {

// One staged entry (see stage_splat) and its stream position.
struct Staged {
    float4 a;  // mx, my, a', 2b'
    float4 b;  // c', opacity, r, g
    float2 c;  // b, position bits
};

struct Pix {
    float T, r, g, b;
    int32_t last, ncon, nvis, nsup;
    bool done;
};

// The per-pixel step shared by both kernels, without branches (explicit
// operation order, no implicit contraction, so both produce identical bits):
// skip when q < 0 (rounding only) or alpha < 1/255; stop, without
// compositing, when T (1 - alpha) < 1e-4; otherwise C += alpha T c and
// T *= 1 - alpha.
template <bool COUNT>
__device__ __forceinline__ void blend(Pix& p, float px, float py, const Staged& s) {
#pragma clang fp contract(off)
    const float dx = s.a.x - px;
    const float dy = s.a.y - py;
    const float w = fmaf(s.a.z, dx, s.a.w * dy);
    const float q2 = fmaf(dx, w, (s.b.x * dy) * dy);  // = -q / (2 ln 2)
    const float araw = s.b.y * __builtin_amdgcn_exp2f(q2);
    const bool live = !p.done;
    const bool sup = live && (q2 <= 0.0f) && (araw >= kAlphaMin);
    const float alpha = fminf(kAlphaMax, araw);
    const float test = p.T * (1.0f - alpha);
    const bool comp = sup && (test >= kTMin);
    if (COUNT) {
        p.nvis += live ? 1 : 0;
        p.nsup += sup ? 1 : 0;
        p.ncon += comp ? 1 : 0;
    }
    p.done = p.done || (sup && !comp);
    const float wt = comp ? alpha * p.T : 0.0f;
    p.r = fmaf(wt, s.b.z, p.r);
    p.g = fmaf(wt, s.b.w, p.g);
    p.b = fmaf(wt, s.c.x, p.b);
    p.T = comp ? test : p.T;
    p.last = comp ? __float_as_int(s.c.y) : p.last;
}

__device__ __forceinline__ void write_pixel(const RasterArgs& A, int x, int y, const Pix& p, bool bad) {
    const int64_t i = (int64_t)y * A.width + x;
    if (bad) {
        const float nan = __builtin_nanf("");
        A.rgb[3 * i] = nan; A.rgb[3 * i + 1] = nan; A.rgb[3 * i + 2] = nan;
        A.alpha[i] = nan;
        A.last[i] = -1;
        if (A.n_contrib) A.n_contrib[i] = 0;
        if (A.n_visit) A.n_visit[i] = 0;
        if (A.n_support) A.n_support[i] = 0;
        return;
    }
    A.rgb[3 * i] = p.r + p.T * A.bg[0];
    A.rgb[3 * i + 1] = p.g + p.T * A.bg[1];
    A.rgb[3 * i + 2] = p.b + p.T * A.bg[2];
    A.alpha[i] = 1.0f - p.T;
    A.last[i] = p.last;
    if (A.n_contrib) A.n_contrib[i] = p.ncon;
    if (A.n_visit) A.n_visit[i] = p.nvis;
    if (A.n_support) A.n_support[i] = p.nsup;
}

enum Src { SRC_VALS = 0, SRC_PAIRS = 1, SRC_PACKED = 2 };

template <int SRC>
__device__ __forceinline__ uint32_t id_at(const RasterArgs& A, uint32_t p) {
    if (SRC == SRC_VALS) return A.vals[p];
    return (uint32_t)A.pairs[p];
}

// The staged entry at stream position p (packed records are already staged).
template <int SRC>
__device__ __forceinline__ Staged load_entry(const RasterArgs& A, uint32_t p, float ox, float oy) {
    Staged s;
    if (SRC == SRC_PACKED) {
        const float4* r = reinterpret_cast<const float4*>(A.records) + kRecordVec * (int64_t)p;
        s.a = r[0];
        s.b = r[1];
        s.c = make_float2(r[2].x, __int_as_float((int32_t)p));
        return s;
    }
    const uint32_t g = id_at<SRC>(A, p);
    const float4* q = reinterpret_cast<const float4*>(A.splats) + kSplatVec * (int64_t)g;
    float s2;
    stage_splat(q[0], q[1], q[2], ox, oy, s.a, s.b, s2);
    s.c = make_float2(s2, __int_as_float((int32_t)p));
    return s;
}

__device__ __forceinline__ int tile_of_block(const RasterArgs& A) {
    const int T = A.tiles_x * A.tiles_y;
    return A.order ? (int)A.order[blockIdx.x] : xcd_remap(blockIdx.x, T);
}

// ---------------------------------------------------------------------------

template <int SRC, bool COUNT>
__global__ void __launch_bounds__(256) raster_plain_kernel(RasterArgs A) {
    __shared__ float4 sa[256];
    __shared__ float4 sb[256];
    __shared__ float2 sc[256];
    const int t = tile_of_block(A);
    const int tx = t % A.tiles_x, ty = t / A.tiles_x;
    const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
    const int x = tx * kTile + lx, y = ty * kTile + ly;
    const bool inside = x < A.width && y < A.height;
    const bool bad = A.counters[2] != 0;
    const float ox = (float)(tx * kTile), oy = (float)(ty * kTile);
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    Pix p{1.0f, 0.f, 0.f, 0.f, -1, 0, 0, 0, !inside || bad};
    const uint32_t begin = A.offsets[(int64_t)t * A.stride];
    const uint32_t end = bad ? begin : A.offsets[(int64_t)(t + 1) * A.stride];
    for (uint32_t base = begin; base < end; base += 256) {
        if (__syncthreads_count(p.done) == 256) break;
        const uint32_t e = base + threadIdx.x;
        if (e < end) {
            const Staged s = load_entry<SRC>(A, e, ox, oy);
            sa[threadIdx.x] = s.a;
            sb[threadIdx.x] = s.b;
            sc[threadIdx.x] = s.c;
        }
        __syncthreads();
        const int cnt = (int)min(256u, end - base);
        for (int j = 0; j < cnt; ++j) {
            if (p.done) break;
            Staged s;
            s.a = sa[j];
            s.b = sb[j];
            s.c = sc[j];
            blend<COUNT>(p, px, py, s);
        }
    }
    if (inside) write_pixel(A, x, y, p, bad);
}

// ---------------------------------------------------------------------------

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Composites the cnt staged survivors of st[], reading the next one from LDS
// while the current one is evaluated.
template <bool COUNT>
__device__ __forceinline__ void composite_staged(Pix& p, float px, float py, const Staged* st, int cnt) {
    if (cnt == 0) return;
    Staged cur = st[0];
    for (int j = 1; j < cnt; ++j) {
        const Staged nxt = st[j];
        blend<COUNT>(p, px, py, cur);
        cur = nxt;
    }
    blend<COUNT>(p, px, py, cur);
}

template <int SRC, bool COUNT>
__global__ void __launch_bounds__(256) raster_wave_kernel(RasterArgs A) {
    __shared__ Staged stage[4][kWave];
    const int t = tile_of_block(A);
    const int tx = t % A.tiles_x, ty = t / A.tiles_x;
    const int w = threadIdx.x / kWave, l = lane();
    float xa, xb, ya, yb;
    if (!block_box(w, tx, ty, A.width, A.height, xa, xb, ya, yb)) return;  // block outside the image
    const int lx = (w & 1) * 8 + (l & 7), ly = (w >> 1) * 8 + (l >> 3);
    const int x = tx * kTile + lx, y = ty * kTile + ly;
    const bool inside = x < A.width && y < A.height;
    const bool bad = A.counters[2] != 0;
    const float ox = (float)(tx * kTile), oy = (float)(ty * kTile);
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    Pix p{1.0f, 0.f, 0.f, 0.f, -1, 0, 0, 0, !inside || bad};
    const uint32_t begin = A.offsets[(int64_t)t * A.stride];
    const uint32_t end = bad ? begin : A.offsets[(int64_t)(t + 1) * A.stride];
    Staged* st = stage[w];
    const uint32_t bit = 1u << w;
    for (uint32_t base = begin; base < end; base += kWave) {
        if (ballot(!p.done) == 0) break;
        const uint32_t e = base + l;
        bool keep = e < end;
        Staged s;
        if (A.masks) {
            // the block mask decides; only survivors fetch their entry
            if (keep) keep = (A.masks[e] & bit) != 0;
            if (keep) s = load_entry<SRC>(A, e, ox, oy);
        } else if (keep) {
            const uint32_t g = id_at<SRC>(A, e);
            const float4* q = reinterpret_cast<const float4*>(A.splats) + kSplatVec * (int64_t)g;
            const float4 q0 = q[0], q1 = q[1], q2 = q[2];
            float s2;
            stage_splat(q0, q1, q2, ox, oy, s.a, s.b, s2);
            s.c = make_float2(s2, __int_as_float((int32_t)e));
            keep = block_may_touch(s.a.x, s.a.y, q1.x, q1.y, q1.z, q1.w, xa, xb, ya, yb);
        }
        const uint64_t m = ballot(keep);
        if (m == 0) continue;
        if (keep) st[rank_in(m)] = s;
        wave_sync();
        composite_staged<COUNT>(p, px, py, st, __builtin_popcountll(m));
        wave_sync();
    }
    if (inside) write_pixel(A, x, y, p, bad);
}

template <int SRC>
hipError_t plain_dispatch(const RasterArgs& a, hipStream_t s) {
    const int T = a.tiles_x * a.tiles_y;
    if (a.n_visit || a.n_support || a.n_contrib)
        hipLaunchKernelGGL((raster_plain_kernel<SRC, true>), dim3(T), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((raster_plain_kernel<SRC, false>), dim3(T), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int SRC>
hipError_t wave_dispatch(const RasterArgs& a, hipStream_t s) {
    const int T = a.tiles_x * a.tiles_y;
    if (a.n_visit || a.n_support || a.n_contrib)
        hipLaunchKernelGGL((raster_wave_kernel<SRC, true>), dim3(T), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((raster_wave_kernel<SRC, false>), dim3(T), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_raster_plain(const RasterArgs& a, hipStream_t s) {
    if (a.tiles_x * a.tiles_y == 0) return hipSuccess;
    if (a.records) return plain_dispatch<SRC_PACKED>(a, s);
    if (a.vals) return plain_dispatch<SRC_VALS>(a, s);
    return plain_dispatch<SRC_PAIRS>(a, s);
}

hipError_t launch_raster_wave(const RasterArgs& a, hipStream_t s) {
    if (a.tiles_x * a.tiles_y == 0) return hipSuccess;
    if (a.records) return wave_dispatch<SRC_PACKED>(a, s);
    if (a.vals) return wave_dispatch<SRC_VALS>(a, s);
    return wave_dispatch<SRC_PAIRS>(a, s);
}

}  // namespace tgs
