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
//               own, 64 entries at a time: every lane loads one entry (a
//               coalesced packed record, or a gather by id), tests with a
//               conservative bound whether the splat can reach alpha 1/255
//               at any pixel centre of the block (the tile alpha cull of the
//               paper's binned kernel, at block granularity), the survivors
//               are compacted into wavefront-private LDS by ballot + prefix
//               count (colour staging), and the lanes composite them. A
//               wavefront exits when all its pixels have terminated, without
//               workgroup barriers. Culled entries are exactly those whose
//               alpha test would fail at every pixel of the block, so images,
//               last ids and contribution counts are unchanged.
#include <math.h>

#include "common.hpp"

namespace tgs {

namespace {

// -0.5 / ln 2: q' = k q lets exp(-q/2) be evaluated as exp2(q').
constexpr float kHalfLog2e = -0.72134752044448170f;

// One staged entry: mean relative to the tile origin, conic scaled by
// kHalfLog2e (b doubled), opacity, colour, stream position.
struct Staged {
    float4 a;  // mx, my, ca', cb2'
    float4 b;  // cc', opacity, r, g
    float2 c;  // b, position bits
};

struct Pix {
    float T, r, g, b;
    int32_t last, ncon, nvis, nsup;
    bool done;
};

// The per-pixel step shared by both kernels (explicit operation order, no
// implicit contraction, so both produce identical bits).
template <bool COUNT>
__device__ __forceinline__ void blend(Pix& p, float px, float py, const Staged& s) {
#pragma clang fp contract(off)
    const float dx = s.a.x - px;
    const float dy = s.a.y - py;
    const float w = fmaf(s.a.z, dx, s.a.w * dy);
    const float q2 = fmaf(dx, w, (s.b.x * dy) * dy);  // = -q / (2 ln 2)
    if (q2 > 0.0f) return;                              // q < 0: rounding only
    const float araw = s.b.y * __builtin_amdgcn_exp2f(q2);
    if (araw < kAlphaMin) return;
    if (COUNT) p.nsup++;
    const float alpha = fminf(kAlphaMax, araw);
    const float test = p.T * (1.0f - alpha);
    if (test < kTMin) {
        p.done = true;
        return;
    }
    const float wt = alpha * p.T;
    p.r = fmaf(wt, s.b.z, p.r);
    p.g = fmaf(wt, s.b.w, p.g);
    p.b = fmaf(wt, s.c.x, p.b);
    p.T = test;
    p.last = __float_as_int(s.c.y);
    p.ncon++;
}

// Stage a splat (12-word layout) for tile origin (ox, oy).
__device__ __forceinline__ Staged stage_splat(const float4& a, const float4& b, const float4& c, float ox, float oy,
                                              int32_t pos) {
#pragma clang fp contract(off)
    Staged s;
    s.a = make_float4((a.x - ox) + a.z, (a.y - oy) + a.w, kHalfLog2e * b.x, (2.0f * kHalfLog2e) * b.y);
    s.b = make_float4(kHalfLog2e * b.z, b.w, c.x, c.y);
    s.c = make_float2(c.z, __int_as_float(pos));
    return s;
}

// Stage a packed record (mean already relative to the tile origin).
__device__ __forceinline__ Staged stage_record(const float4& a, const float4& b, const float4& c, int32_t pos) {
#pragma clang fp contract(off)
    Staged s;
    s.a = make_float4(a.x, a.y, kHalfLog2e * a.z, (2.0f * kHalfLog2e) * a.w);
    s.b = make_float4(kHalfLog2e * b.x, b.y, b.z, b.w);
    s.c = make_float2(c.x, __int_as_float(pos));
    return s;
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

template <int SRC>
__device__ __forceinline__ Staged load_entry(const RasterArgs& A, uint32_t p, float ox, float oy) {
    if (SRC == SRC_PACKED) {
        const float4* r = reinterpret_cast<const float4*>(A.records) + 3 * (int64_t)p;
        return stage_record(r[0], r[1], r[2], (int32_t)p);
    }
    const uint32_t g = id_at<SRC>(A, p);
    const float4* s = reinterpret_cast<const float4*>(A.splats) + 3 * (int64_t)g;
    return stage_splat(s[0], s[1], s[2], ox, oy, (int32_t)p);
}

// ---------------------------------------------------------------------------

template <int SRC, bool COUNT>
__global__ void __launch_bounds__(256) raster_plain_kernel(RasterArgs A) {
    __shared__ float4 sa[256];
    __shared__ float4 sb[256];
    __shared__ float2 sc[256];
    const int T = A.tiles_x * A.tiles_y;
    const int t = A.order ? (int)A.order[blockIdx.x] : xcd_remap(blockIdx.x, T);
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
            if (COUNT) p.nvis++;
            blend<COUNT>(p, px, py, s);
        }
    }
    if (inside) write_pixel(A, x, y, p, bad);
}

// ---------------------------------------------------------------------------

// Conservative block test: can q = a dx^2 + 2 b dx dy + c dy^2 reach
// 2 ln(255 o) at some pixel centre of the block? The minimum of the convex
// q over the box of centres [xa, xb] x [ya, yb] is 0 when the mean is inside,
// otherwise the smallest of the four edge minima. The margin exceeds the
// binary32 error of both this bound and the per-pixel evaluation.
__device__ __forceinline__ bool block_may_touch(float mx, float my, float a, float b, float c, float o, float xa,
                                                float xb, float ya, float yb) {
    const float dxl = mx - xb, dxh = mx - xa, dyl = my - yb, dyh = my - ya;
    float qmin = 0.0f;
    if (!(dxl <= 0.0f && dxh >= 0.0f && dyl <= 0.0f && dyh >= 0.0f)) {
        const float ic = 1.0f / c, ia = 1.0f / a;
        qmin = INFINITY;
        {
            const float d = dxl, e = fminf(fmaxf(-b * d * ic, dyl), dyh);
            qmin = fminf(qmin, a * d * d + 2.0f * b * d * e + c * e * e);
        }
        {
            const float d = dxh, e = fminf(fmaxf(-b * d * ic, dyl), dyh);
            qmin = fminf(qmin, a * d * d + 2.0f * b * d * e + c * e * e);
        }
        {
            const float e = dyl, d = fminf(fmaxf(-b * e * ia, dxl), dxh);
            qmin = fminf(qmin, a * d * d + 2.0f * b * d * e + c * e * e);
        }
        {
            const float e = dyh, d = fminf(fmaxf(-b * e * ia, dxl), dxh);
            qmin = fminf(qmin, a * d * d + 2.0f * b * d * e + c * e * e);
        }
    }
    const float mxd = fmaxf(fabsf(dxl), fabsf(dxh)), myd = fmaxf(fabsf(dyl), fabsf(dyh));
    const float mag = a * mxd * mxd + c * myd * myd + 2.0f * fabsf(b) * mxd * myd;
    const float tau = 2.0f * __logf(255.0f * o);
    return qmin <= tau + 1e-3f + 4e-6f * mag;
}

// Loads the raw 12-word record or splat of entry e for the cull test and
// staging.
template <int SRC>
__device__ __forceinline__ void fetch_entry(const RasterArgs& A, uint32_t e, float4& r0, float4& r1, float4& r2) {
    if (SRC == SRC_PACKED) {
        const float4* r = reinterpret_cast<const float4*>(A.records) + 3 * (int64_t)e;
        r0 = r[0];
        r1 = r[1];
        r2 = r[2];
    } else {
        const uint32_t g = id_at<SRC>(A, e);
        const float4* q = reinterpret_cast<const float4*>(A.splats) + 3 * (int64_t)g;
        r0 = q[0];
        r1 = q[1];
        r2 = q[2];
    }
}

template <int SRC, bool COUNT, bool CULL>
__global__ void __launch_bounds__(256) raster_wave_kernel(RasterArgs A) {
    __shared__ Staged stage[4][kWave];
    const int T = A.tiles_x * A.tiles_y;
    const int t = A.order ? (int)A.order[blockIdx.x] : xcd_remap(blockIdx.x, T);
    const int tx = t % A.tiles_x, ty = t / A.tiles_x;
    const int w = threadIdx.x / kWave, l = lane();
    const int bx = (w & 1) * 8, by = (w >> 1) * 8;
    const int lx = bx + (l & 7), ly = by + (l >> 3);
    const int x = tx * kTile + lx, y = ty * kTile + ly;
    const bool inside = x < A.width && y < A.height;
    const bool bad = A.counters[2] != 0;
    // pixel-centre box of the block's in-image pixels (tile-local)
    const int nx = min(8, A.width - (tx * kTile + bx)), ny = min(8, A.height - (ty * kTile + by));
    if (nx <= 0 || ny <= 0) return;  // whole wavefront outside the image
    const float xa = bx + 0.5f, xb = bx + nx - 0.5f, ya = by + 0.5f, yb = by + ny - 0.5f;
    const float ox = (float)(tx * kTile), oy = (float)(ty * kTile);
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    Pix p{1.0f, 0.f, 0.f, 0.f, -1, 0, 0, 0, !inside || bad};
    const uint32_t begin = A.offsets[(int64_t)t * A.stride];
    const uint32_t end = bad ? begin : A.offsets[(int64_t)(t + 1) * A.stride];
    Staged* st = stage[w];
    // software pipeline: the next 64 entries are in flight while the current
    // ones are culled and composited
    float4 n0 = make_float4(0.f, 0.f, 0.f, 0.f), n1 = n0, n2 = n0;
    if (begin + l < end) fetch_entry<SRC>(A, begin + l, n0, n1, n2);
    for (uint32_t base = begin; base < end; base += kWave) {
        if (ballot(!p.done) == 0) break;
        const uint32_t e = base + l;
        const float4 r0 = n0, r1 = n1, r2 = n2;
        if (e + kWave < end) fetch_entry<SRC>(A, e + kWave, n0, n1, n2);
        bool keep = e < end;
        Staged s;
        if (SRC == SRC_PACKED) {
            if (CULL && keep) keep = block_may_touch(r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, xa, xb, ya, yb);
            s = stage_record(r0, r1, r2, (int32_t)e);
        } else {
            s = stage_splat(r0, r1, r2, ox, oy, (int32_t)e);
            if (CULL && keep) keep = block_may_touch(s.a.x, s.a.y, r1.x, r1.y, r1.z, r1.w, xa, xb, ya, yb);
        }
        const uint64_t m = ballot(keep);
        if (keep) st[rank_in(m)] = s;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int cnt = __builtin_popcountll(m);
        for (int j = 0; j < cnt; ++j) {
            if (!p.done) {
                if (COUNT) p.nvis++;
                blend<COUNT>(p, px, py, st[j]);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
        hipLaunchKernelGGL((raster_wave_kernel<SRC, true, true>), dim3(T), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((raster_wave_kernel<SRC, false, true>), dim3(T), dim3(256), 0, s, a);
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
