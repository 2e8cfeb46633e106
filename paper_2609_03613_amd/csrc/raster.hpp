// Per-pixel compositing step, entry staging and the 8x8-block walk shared by
// the forward rasters, the batched persistent raster and the backward raster
// (device code, included by the raster sources only).
#pragma once

#include "common.hpp"

namespace tgs {
namespace raster {

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

// The per-pixel step shared by all rasters, without branches (explicit
// operation order, no implicit contraction, so every kernel produces
// identical bits): skip when q < 0 (rounding only) or alpha < 1/255; with
// w = alpha T, stop, without compositing, when the transmittance after the
// entry, T - w, is below 1e-4; otherwise C += w c and T = T - w.
// The entry's alpha at the pixel (px, py) and whether it passes the support
// test (q <= 0 and alpha >= 1/255), in the one operation order every
// raster uses.
__device__ __forceinline__ float entry_alpha(float px, float py, const Staged& s, bool& sup) {
#pragma clang fp contract(off)
    const float dx = s.a.x - px;
    const float dy = s.a.y - py;
    const float w = fmaf(s.a.z, dx, s.a.w * dy);
    const float q2 = fmaf(dx, w, (s.b.x * dy) * dy);  // = -q / (2 ln 2)
    const float araw = s.b.y * __builtin_amdgcn_exp2f(q2);
    sup = (q2 <= 0.0f) && (araw >= kAlphaMin);
    return fminf(kAlphaMax, araw);
}

template <bool COUNT>
__device__ __forceinline__ void blend(Pix& p, float px, float py, const Staged& s) {
#pragma clang fp contract(off)
    bool in_support;
    const float alpha = entry_alpha(px, py, s, in_support);
    const bool live = !p.done;
    const bool sup = live && in_support;
    const float wt0 = alpha * p.T;
    const float next = p.T - wt0;
    const bool pass = next >= kTMin;
    const bool comp = sup && pass;
    if (COUNT) {
        p.nvis += live ? 1 : 0;
        p.nsup += sup ? 1 : 0;
        p.ncon += comp ? 1 : 0;
    }
    p.done = p.done || (sup && !pass);
    const float wt = comp ? wt0 : 0.0f;
    p.r = fmaf(wt, s.b.z, p.r);
    p.g = fmaf(wt, s.b.w, p.g);
    p.b = fmaf(wt, s.c.x, p.b);
    p.T = comp ? next : p.T;
    p.last = comp ? __float_as_int(s.c.y) : p.last;
}

__device__ __forceinline__ void write_pixel(const RasterArgs& A, int x, int y, const Pix& p, bool bad) {
    const int64_t i = (int64_t)y * A.width + x;
    if (bad) {
        const float nan = __builtin_nanf("");
        A.rgb[3 * i] = nan; A.rgb[3 * i + 1] = nan; A.rgb[3 * i + 2] = nan;
        A.alpha[i] = nan;
        A.last[i] = -1;
        if (A.trans) A.trans[i] = nan;
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
    if (A.trans) A.trans[i] = p.T;
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

// First and one-past-last stream position of tile t.
__device__ __forceinline__ uint32_t tile_begin(const RasterArgs& A, int t) {
    return A.offsets[A.seg_base ? (int64_t)A.seg_base[t] : (int64_t)t * A.stride];
}
__device__ __forceinline__ uint32_t tile_end(const RasterArgs& A, int t) {
    return A.offsets[A.seg_base ? (int64_t)A.seg_base[t + 1] : (int64_t)(t + 1) * A.stride];
}

__device__ __forceinline__ int tile_of_block(const RasterArgs& A) {
    const int T = A.tiles_x * A.tiles_y;
    return A.order ? (int)A.order[blockIdx.x] : xcd_remap(blockIdx.x, T);
}

// 8x8 pixel blocks per tile and workgroups (of up to four 64-lane
// wavefronts, one block each) per tile for a tile edge of `tile` pixels.
__host__ __device__ __forceinline__ int blocks_per_tile(int tile) { return (tile >> 3) * (tile >> 3); }
__host__ __device__ __forceinline__ int groups_per_tile(int tile) { return (blocks_per_tile(tile) + 3) >> 2; }

// The block a wavefront of the WAVE rasters owns: tile t = (tx, ty) and the
// block's tile-local pixel offset (bx, by) and index bi. Workgroup i serves
// group i % G of tile slot i / G (slot = position in the dispatch order, or
// the XCD-aware remap of i); false for the idle wavefronts of a short last
// group.
struct WaveBlock {
    int t, tx, ty, bi, bx, by;
};
__device__ __forceinline__ bool block_of_wave(const RasterArgs& A, int w, WaveBlock& b) {
    const int nb = A.tile >> 3, B = nb * nb, G = (B + 3) >> 2;
    const int T = A.tiles_x * A.tiles_y;
    int slot, grp;
    if (A.order) {
        slot = (int)blockIdx.x / G;
        grp = (int)blockIdx.x % G;
        b.t = (int)A.order[slot];
    } else {
        const int i = xcd_remap((int)blockIdx.x, T * G);
        slot = i / G;
        grp = i % G;
        b.t = slot;
    }
    b.bi = grp * 4 + w;
    if (b.bi >= B) return false;
    b.tx = b.t % A.tiles_x;
    b.ty = b.t / A.tiles_x;
    b.bx = (b.bi % nb) * 8;
    b.by = (b.bi / nb) * 8;
    return true;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One entry of a group in which no pixel stops: blend's arithmetic without
// the stop test (comp = supported and the pixel live; a = its alpha, 0
// otherwise).
__device__ __forceinline__ void blend_pass(Pix& p, float alpha, bool comp, const Staged& s) {
#pragma clang fp contract(off)
    const float a = comp ? alpha : 0.0f;
    const float wt = a * p.T;
    p.T = p.T - wt;
    p.r = fmaf(wt, s.b.z, p.r);
    p.g = fmaf(wt, s.b.w, p.g);
    p.b = fmaf(wt, s.c.x, p.b);
    p.last = comp ? __float_as_int(s.c.y) : p.last;
}

// Four entries. The transmittance only decreases, and a stopped pixel keeps
// one of at least 1e-4, so when every lane's transmittance after the four
// is at least 1e-4 no pixel stopped inside them: each supported entry was
// composited, with exactly blend's operations, and the per-entry stop tests
// and selects are skipped. Otherwise the four are redone by blend.
template <bool COUNT>
__device__ __forceinline__ void blend4(Pix& p, float px, float py, const Staged& s0, const Staged& s1,
                                       const Staged& s2, const Staged& s3) {
    const Pix p0 = p;
    const bool live = !p.done;
    bool u0, u1, u2, u3;
    const float a0 = entry_alpha(px, py, s0, u0), a1 = entry_alpha(px, py, s1, u1);
    const float a2 = entry_alpha(px, py, s2, u2), a3 = entry_alpha(px, py, s3, u3);
    blend_pass(p, a0, live && u0, s0);
    blend_pass(p, a1, live && u1, s1);
    blend_pass(p, a2, live && u2, s2);
    blend_pass(p, a3, live && u3, s3);
    if (COUNT) {
        p.nvis += live ? 4 : 0;
        const int su = (u0 ? 1 : 0) + (u1 ? 1 : 0) + (u2 ? 1 : 0) + (u3 ? 1 : 0);
        p.nsup += live ? su : 0;
        p.ncon += live ? su : 0;
    }
    if (ballot(p.T < kTMin) != 0) {
        p = p0;
        blend<COUNT>(p, px, py, s0);
        blend<COUNT>(p, px, py, s1);
        blend<COUNT>(p, px, py, s2);
        blend<COUNT>(p, px, py, s3);
    }
}

// Composites the cnt staged survivors of st[], four at a time (all four read
// from LDS before the first is evaluated: more independent work per
// wavefront hides the LDS latency better than more wavefronts would; eight
// at a time costs too many registers).
template <bool COUNT>
__device__ __forceinline__ void composite_staged(Pix& p, float px, float py, const Staged* st, int cnt) {
    int j = 0;
    for (; j + 4 <= cnt; j += 4) {
        const Staged s0 = st[j], s1 = st[j + 1], s2 = st[j + 2], s3 = st[j + 3];
        blend4<COUNT>(p, px, py, s0, s1, s2, s3);
    }
    for (; j < cnt; ++j) blend<COUNT>(p, px, py, st[j]);
}


// The forward walk of one 8x8 block over the tile range [begin, end) (the
// WAVE raster's main loop): 64 entries at a time, kept when the block mask
// (A.masks) or the conservative block test on the gathered splat says they
// can reach alpha 1/255 in the block, compacted into the wavefront's LDS
// slots st[] and composited by every lane. Without masks the gathers are
// software-pipelined: while chunk i is culled and composited, the splats of
// chunk i + 1 and the ids of chunk i + 2 are in flight.
template <int SRC, bool COUNT>
__device__ __forceinline__ void wave_forward(const RasterArgs& A, Staged* st, int bi, uint32_t begin, uint32_t end,
                                             float ox, float oy, float px, float py, float xa, float xb, float ya,
                                             float yb, Pix& p) {
    const int l = lane();
    if (A.masks) {
        const uint32_t bit = 1u << bi;  // block masks exist for 16-pixel tiles only (bi < 4)
        for (uint32_t base = begin; base < end; base += kWave) {
            if (ballot(!p.done) == 0) break;
            const uint32_t e = base + l;
            bool keep = e < end;
            Staged s;
            // the block mask decides; only survivors fetch their entry
            if (keep) keep = (A.masks[e] & bit) != 0;
            if (keep) s = load_entry<SRC>(A, e, ox, oy);
            const uint64_t m = ballot(keep);
            if (m != 0) {
                if (keep) st[rank_in(m)] = s;
                wave_sync();
                composite_staged<COUNT>(p, px, py, st, __builtin_popcountll(m));
                wave_sync();
            }
        }
        return;
    }
    if (begin >= end) return;
    const float4* sp = reinterpret_cast<const float4*>(A.splats);
    // Two register sets alternate (the loop is unrolled by two, so no set is
    // copied while its loads are in flight): chunk i is processed from one
    // set while the other receives chunk i + 1, whose ids arrived during
    // chunk i - 1. Every lane issues every load (lanes past the range read
    // the range's last entry and are dropped by the range test), so the
    // loads stay in issue order and only the older set is waited for.
    auto id_clamped = [&](uint32_t e) { return id_at<SRC>(A, e < end ? e : end - 1); };
    auto gather = [&](uint32_t g, float4& r0, float4& r1, float4& r2) {
        const float4* q = sp + kSplatVec * (int64_t)g;
        r0 = q[0];
        r1 = q[1];
        r2 = q[2];
    };
    auto chunk = [&](uint32_t base, const float4& c0, const float4& c1, const float4& c2, uint32_t g_next,
                     float4& n0, float4& n1, float4& n2, uint32_t& g_after) {
        const uint32_t e = base + l;
        bool keep = e < end;
        gather(g_next, n0, n1, n2);
        g_after = id_clamped(e + 2 * kWave);
        Staged s;
        if (keep) {
            float s2;
            stage_splat(c0, c1, c2, ox, oy, s.a, s.b, s2);
            s.c = make_float2(s2, __int_as_float((int32_t)e));
            keep = block_may_touch(s.a.x, s.a.y, c1.x, c1.y, c1.z, c1.w, xa, xb, ya, yb);
        }
        const uint64_t m = ballot(keep);
        if (m != 0) {
            if (keep) st[rank_in(m)] = s;
            wave_sync();
            composite_staged<COUNT>(p, px, py, st, __builtin_popcountll(m));
            wave_sync();
        }
    };
    float4 a0, a1, a2, b0, b1, b2;
    uint32_t ga = id_clamped(begin + l), gb;
    gather(ga, a0, a1, a2);
    gb = id_clamped(begin + kWave + l);
    for (uint32_t base = begin;;) {
        if (base >= end || ballot(!p.done) == 0) break;
        chunk(base, a0, a1, a2, gb, b0, b1, b2, ga);
        base += kWave;
        if (base >= end || ballot(!p.done) == 0) break;
        chunk(base, b0, b1, b2, ga, a0, a1, a2, gb);
        base += kWave;
    }
}

// ---------------------------------------------------------------------------
// Quad walk (the heavy tiles of the split raster). A wavefront owns a 4x4
// quarter of an 8x8 block with four lanes per pixel: lane 4 i + k serves
// pixel i of the quarter in role k. Survivors are taken four at a time:
// lane k evaluates the alpha of survivor 4 s + k at its pixel, then each of
// the pixel's four lanes runs the pixel's transmittance chain over the four
// entries in stream order, on alphas broadcast within the lane quad, with
// blend's binary32 operations (w = alpha T, T' = T - w, stop when T' <
// 1e-4), and lane k < 3 adds w times colour channel k. The chain therefore
// gives, per pixel, exactly blend's values: images, last ids and counts are
// bitwise those of the one-lane-per-pixel walk, while a heavy tile's walk is
// spread over 16 wavefronts that each take four entries per step.
struct QuadPix {
    float T;       // transmittance before the next entry; 0 once the pixel has stopped (and
                   // for pixels outside the image), otherwise at least 1e-4
    float Tend;    // transmittance at the stop
    float acc;     // colour channel k (roles 0..2)
    int32_t last;  // position of this lane's last composited entry (the quad's largest is the pixel's)
    int32_t ncon, nvis, nsup;  // this lane's entries (summed over the quad at the end)
};

// Lane 4 (lane / 4) + J's value, for every lane of the quad.
template <int J>
__device__ __forceinline__ int quad_bcast(int v) {
    return __builtin_amdgcn_mov_dpp(v, J * 0x55, 0xF, 0xF, true);
}
template <int J>
__device__ __forceinline__ float quad_bcast(float v) {
    return __int_as_float(quad_bcast<J>(__float_as_int(v)));
}
// Sum / maximum over the lane quad, in every lane of it.
__device__ __forceinline__ int quad_sum(int v) {
    v += __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);  // lanes (1, 0, 3, 2)
    return v + __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);  // lanes (2, 3, 0, 1)
}
__device__ __forceinline__ int quad_max(int v) {
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true));
    return max(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true));
}

// Entry J of a step in which some pixel of the wavefront stops: blend's
// chain for one entry, with the stop (aj = entry J's alpha or 0, c its
// colour channel k; own = this lane holds entry J, real = it exists).
template <bool COUNT, int J>
__device__ __forceinline__ void quad_entry(QuadPix& p, int k, float aj, int32_t pos, float c, bool real) {
#pragma clang fp contract(off)
    const bool own = k == J;
    const bool live = p.T > 0.0f;
    float wt = aj * p.T;
    float next = p.T - wt;
    const bool stop = live && next < kTMin;
    if (COUNT && own && real) {
        p.nvis += live ? 1 : 0;
        p.nsup += (live && aj > 0.0f) ? 1 : 0;
    }
    p.Tend = stop ? p.T : p.Tend;
    wt = stop ? 0.0f : wt;
    next = stop ? 0.0f : next;
    const bool comp = own && wt > 0.0f;
    if (COUNT) p.ncon += comp ? 1 : 0;
    p.last = comp ? pos : p.last;
    p.acc = fmaf(wt, c, p.acc);
    p.T = next;
}

// Four entries (this lane's: alpha a, or 0 when unsupported or padding;
// own = a > 0; real = the entry exists; c = colour channel k of the four).
// The transmittance only decreases along the chain, so when the fourth
// value is at least 1e-4 for every live pixel no pixel stops inside the
// step: then every supported entry is composited, which is blend's result
// for all four, and the lane's own entry decides its last position.
// Otherwise the step is redone entry by entry from its saved state.
template <bool COUNT>
__device__ __forceinline__ void quad_step(QuadPix& p, int k, float a, bool own, bool real, int32_t pos,
                                          const float4& c) {
#pragma clang fp contract(off)
    const QuadPix p0 = p;
    const float a0 = quad_bcast<0>(a), a1 = quad_bcast<1>(a), a2 = quad_bcast<2>(a), a3 = quad_bcast<3>(a);
    const bool live = p.T > 0.0f;
    const float w0 = a0 * p.T;
    const float t1 = p.T - w0;
    const float w1 = a1 * t1;
    const float t2 = t1 - w1;
    const float w2 = a2 * t2;
    const float t3 = t2 - w2;
    const float w3 = a3 * t3;
    const float t4 = t3 - w3;
    p.acc = fmaf(w0, c.x, p.acc);
    p.acc = fmaf(w1, c.y, p.acc);
    p.acc = fmaf(w2, c.z, p.acc);
    p.acc = fmaf(w3, c.w, p.acc);
    p.T = t4;
    const bool comp = own && live;
    p.last = comp ? pos : p.last;
    if (COUNT) {
        p.nvis += (real && live) ? 1 : 0;
        p.nsup += comp ? 1 : 0;
        p.ncon += comp ? 1 : 0;
    }
    if ((ballot(t4 < kTMin) & ballot(live)) != 0) {
        p = p0;
        quad_entry<COUNT, 0>(p, k, a0, pos, c.x, real);
        quad_entry<COUNT, 1>(p, k, a1, pos, c.y, real);
        quad_entry<COUNT, 2>(p, k, a2, pos, c.z, real);
        quad_entry<COUNT, 3>(p, k, a3, pos, c.w, real);
    }
}

// The cnt staged survivors st[] (colour channel ch of survivor i at
// col[ch kWave + i]; slots cnt .. cnt rounded up to 4 hold 0).
template <bool COUNT>
__device__ __forceinline__ void composite_quad(QuadPix& p, int k, float px, float py, const Staged* st,
                                               const float* col, int cnt) {
    const Staged* sk = st + k;
    const float* ck = col + (k < 3 ? k : 2) * kWave;
    for (int s4 = 0; s4 < cnt; s4 += 4) {
        // slots past cnt (at most the last three of the step) hold stale
        // entries: their alpha is replaced by 0 and their colours are 0
        const Staged s = sk[s4];
        const float4 c4 = *reinterpret_cast<const float4*>(ck + s4);
        const bool real = s4 + k < cnt;
        bool sup;
        const float alpha = entry_alpha(px, py, s, sup);
        const bool own = sup && real;
        const float a = own ? alpha : 0.0f;
        quad_step<COUNT>(p, k, a, own, real, __float_as_int(s.c.y), c4);
    }
}

// The quad walk of one 4x4 quarter (box [xa, xb] x [ya, yb]) over the tile
// range [begin, end): wave_forward's pipelined gathers and cull, survivors
// staged with their colours split by channel, composited by composite_quad.
template <int SRC, bool COUNT>
__device__ __forceinline__ void quad_forward(const RasterArgs& A, Staged* st, float* col, uint32_t begin,
                                             uint32_t end, float ox, float oy, float px, float py, float xa,
                                             float xb, float ya, float yb, QuadPix& p) {
    if (begin >= end) return;
    const int l = lane(), k = l & 3;
    const float4* sp = reinterpret_cast<const float4*>(A.splats);
    auto id_clamped = [&](uint32_t e) { return id_at<SRC>(A, e < end ? e : end - 1); };
    auto gather = [&](uint32_t g, float4& r0, float4& r1, float4& r2) {
        const float4* q = sp + kSplatVec * (int64_t)g;
        r0 = q[0];
        r1 = q[1];
        r2 = q[2];
    };
    auto chunk = [&](uint32_t base, const float4& c0, const float4& c1, const float4& c2, uint32_t g_next,
                     float4& n0, float4& n1, float4& n2, uint32_t& g_after) {
        const uint32_t e = base + l;
        bool keep = e < end;
        gather(g_next, n0, n1, n2);
        g_after = id_clamped(e + 2 * kWave);
        Staged s;
        if (keep) {
            float s2;
            stage_splat(c0, c1, c2, ox, oy, s.a, s.b, s2);
            s.c = make_float2(s2, __int_as_float((int32_t)e));
            keep = block_may_touch(s.a.x, s.a.y, c1.x, c1.y, c1.z, c1.w, xa, xb, ya, yb);
        }
        const uint64_t m = ballot(keep);
        if (m != 0) {
            const int cnt = __builtin_popcountll(m);
            if (keep) {
                const uint32_t r = rank_in(m);
                st[r] = s;
                col[r] = s.b.z;
                col[kWave + r] = s.b.w;
                col[2 * kWave + r] = s.c.x;
            }
            if (l >= cnt && l < ((cnt + 3) & ~3)) {
                col[l] = 0.0f;
                col[kWave + l] = 0.0f;
                col[2 * kWave + l] = 0.0f;
            }
            wave_sync();
            composite_quad<COUNT>(p, k, px, py, st, col, cnt);
            wave_sync();
        }
    };
    float4 a0, a1, a2, b0, b1, b2;
    uint32_t ga = id_clamped(begin + l), gb;
    gather(ga, a0, a1, a2);
    gb = id_clamped(begin + kWave + l);
    for (uint32_t base = begin;;) {
        if (base >= end || ballot(p.T > 0.0f) == 0) break;
        chunk(base, a0, a1, a2, gb, b0, b1, b2, ga);
        base += kWave;
        if (base >= end || ballot(p.T > 0.0f) == 0) break;
        chunk(base, b0, b1, b2, ga, a0, a1, a2, gb);
        base += kWave;
    }
}

// write_pixel for the quad walk (called by all four lanes of the quad):
// role k < 3 writes colour channel k, role 3 the alpha, last id and the
// optional planes (the same expressions).
template <bool COUNT>
__device__ __forceinline__ void write_quad(const RasterArgs& A, int x, int y, int k, bool inside, QuadPix p,
                                           bool bad) {
    p.last = quad_max(p.last);
    if (COUNT) {
        p.ncon = quad_sum(p.ncon);
        p.nvis = quad_sum(p.nvis);
        p.nsup = quad_sum(p.nsup);
    }
    if (!inside) return;
    const int64_t i = (int64_t)y * A.width + x;
    const float T = p.T > 0.0f ? p.T : p.Tend;
    if (bad) {
        const float nan = __builtin_nanf("");
        if (k < 3) {
            A.rgb[3 * i + k] = nan;
            return;
        }
        A.alpha[i] = nan;
        A.last[i] = -1;
        if (A.trans) A.trans[i] = nan;
        if (A.n_contrib) A.n_contrib[i] = 0;
        if (A.n_visit) A.n_visit[i] = 0;
        if (A.n_support) A.n_support[i] = 0;
        return;
    }
    if (k == 0) A.rgb[3 * i] = p.acc + T * A.bg[0];
    if (k == 1) A.rgb[3 * i + 1] = p.acc + T * A.bg[1];
    if (k == 2) A.rgb[3 * i + 2] = p.acc + T * A.bg[2];
    if (k < 3) return;
    A.alpha[i] = 1.0f - T;
    A.last[i] = p.last;
    if (A.trans) A.trans[i] = T;
    if (A.n_contrib) A.n_contrib[i] = p.ncon;
    if (A.n_visit) A.n_visit[i] = p.nvis;
    if (A.n_support) A.n_support[i] = p.nsup;
}

}  // namespace raster
}  // namespace tgs
