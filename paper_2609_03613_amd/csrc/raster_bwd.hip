// Backward of the compositing: dL/d(splat) of every Gaussian from dL/d rgb
// and dL/d alpha of the image. The paper has no backward pass (it lists
// training as future work in its Conclusion); this is the derivative of the
// per-pixel step the forward rasters evaluate, over the same entry stream.
//
// Each 64-lane wavefront owns one 8x8 pixel block, as in the forward WAVE
// raster. Pass 1 repeats the forward walk (same staging, culling and blend,
// so the final transmittance and the last composited position come out
// bit-identical to the forward's), unless the forward's saved final
// transmittance and last position are given. Pass 2 walks the range backwards from
// the largest last position in the block, 64 entries at a time, with the
// same block cull and LDS compaction; each lane recovers the transmittance
// in front of an entry by dividing by the same binary32 (1 - alpha) the
// forward multiplied by (a hardware reciprocal, within an ulp), and keeps the
// colour behind it,
// S = T_final bg + sum over later entries of T alpha c. Per entry k:
//   dL/dc_k     = g T_k alpha_k
//   dL/dalpha_k = sum_ch g_ch (T_k c_ch - S_ch / (1 - alpha_k))
//                 + g_alpha T_final / (1 - alpha_k)
// and, when alpha is not capped at 0.99, through alpha = o exp2(q'):
// dL/do = dL/dalpha exp2(q'), dL/dq' = dL/dalpha alpha ln 2, with q' the
// scaled quadratic form of the staged conic. The 9 per-lane gradients of an
// entry are summed over the wavefront (recursive halving with DPP within the
// rows of 16 lanes, then two lane swaps) and nine lanes of row 0 add the 9
// sums to the Gaussian's gradient line with one float atomic each.
#include <math.h>

#include "raster.hpp"

namespace tgs {

namespace {

using namespace raster;

// v + the value of the DPP partner (control CTRL) of the lane.
template <int CTRL>
__device__ __forceinline__ float dpp_add(float v, float send) {
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), CTRL, 0xF, 0xF, false));
}

// One halving step of the row reduction: the lane keeps the slots of its
// side (hi: the upper set) and adds its partner's copy of them, which the
// partner, on the other side, sends.
template <int CTRL>
__device__ __forceinline__ float halve(bool hi, float lower, float upper) {
    return dpp_add<CTRL>(hi ? upper : lower, hi ? lower : upper);
}

// Word of the gradient line whose wavefront sum wave_sums9 leaves in lane
// i (0..15) of a row, 0xF for none: lanes 0, 1, 2, 4, 5 hold words 0..4,
// lanes 8, 9, 10, 12 words 5..8.
constexpr uint64_t kSumWord = 0xFFF8F765FF43F210ull;

// Wavefront sums of 9 values by recursive halving within the rows of 16
// lanes: each step pairs every lane with a partner on the other side of a
// split (row mirror: i and 15 - i; half-row mirror: i and 7 - i within each
// half; then lane ^ 2 and lane ^ 1), the lane keeps half of its value slots
// and adds the partner's copy of them (9 -> 5 -> 3 -> 2 -> 1 slots), so that
// after four steps every lane holds one value summed over its row; the four
// rows are then added by two lane swaps. The sum of word w ends in the row-0
// lane whose kSumWord nibble is w.
__device__ __forceinline__ float wave_sums9(const float* d) {
    const int i = lane() & 15;
    const bool ha = i >= 8, hb = (i & 4) != 0, hc = (i & 2) != 0, hd = (i & 1) != 0;
    float a[5];
#pragma unroll
    for (int s = 0; s < 4; ++s) a[s] = halve<0x140>(ha, d[s], d[5 + s]);
    a[4] = halve<0x140>(ha, d[4], 0.f);
    float b[3];
#pragma unroll
    for (int t = 0; t < 2; ++t) b[t] = halve<0x141>(hb, a[t], a[3 + t]);
    b[2] = halve<0x141>(hb, a[2], 0.f);
    const float c0 = halve<0x4E>(hc, b[0], b[2]);
    const float c1 = halve<0x4E>(hc, b[1], 0.f);
    float mine = halve<0xB1>(hd, c0, c1);
    mine += __shfl_xor(mine, 16, kWave);
    mine += __shfl_xor(mine, 32, kWave);
    return mine;
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v = max(v, __shfl_xor(v, d, kWave));
    return v;
}

constexpr float kLn2 = 0.69314718055994531f;

template <int SRC>
__global__ void __launch_bounds__(256) raster_bwd_kernel(RasterArgs A, const float* __restrict__ d_rgb,
                                                         const float* __restrict__ d_alpha,
                                                         const float* __restrict__ trans_in,
                                                         const int32_t* __restrict__ last_in,
                                                         float* __restrict__ d_splats) {
#pragma clang fp contract(off)
    __shared__ Staged stage[4][kWave];
    __shared__ uint32_t ids[4][kWave];
    const int w = threadIdx.x / kWave, l = lane();
    WaveBlock wb;
    if (!block_of_wave(A, w, wb)) return;
    const int x0 = wb.tx * A.tile, y0 = wb.ty * A.tile;
    float xa, xb, ya, yb;
    if (!block_box_at(wb.bx, wb.by, x0, y0, A.width, A.height, xa, xb, ya, yb)) return;  // block outside the image
    if (A.counters[2] != 0) return;  // truncated stream: the forward image is NaN, no gradient
    const int lx = wb.bx + (l & 7), ly = wb.by + (l >> 3);
    const int x = x0 + lx, y = y0 + ly;
    const bool inside = x < A.width && y < A.height;
    const float ox = (float)x0, oy = (float)y0;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    const uint32_t begin = tile_begin(A, wb.t);
    const uint32_t end = tile_end(A, wb.t);
    Staged* st = stage[w];
    uint32_t* idw = ids[w];

    // pass 1: the forward walk, or the forward's saved T and last
    Pix p{1.0f, 0.f, 0.f, 0.f, -1, 0, 0, 0, !inside};
    if (trans_in) {
        if (inside) {
            const int64_t i = (int64_t)y * A.width + x;
            p.T = trans_in[i];
            p.last = last_in[i];
        }
    } else {
        wave_forward<SRC, false>(A, st, wb.bi, begin, end, ox, oy, px, py, xa, xb, ya, yb, p);
    }

    // pass 2: backwards from the last composited entry
    const int hi = wave_max_i32(p.last);
    if (hi < 0) return;
    float gr = 0.f, gg = 0.f, gb = 0.f, ga = 0.f;
    if (inside) {
        const int64_t i = (int64_t)y * A.width + x;
        gr = d_rgb[3 * i];
        gg = d_rgb[3 * i + 1];
        gb = d_rgb[3 * i + 2];
        ga = d_alpha ? d_alpha[i] : 0.f;
    }
    const float Tf = p.T;
    const float gaT = ga * Tf;
    // the gradient word this lane adds (row 0 only)
    const int sum_word = l < 16 ? (int)((kSumWord >> (4 * l)) & 0xF) : 0xF;
    float T = Tf;
    float Sr = Tf * A.bg[0], Sg = Tf * A.bg[1], Sb = Tf * A.bg[2];
    // Chunks of 64 entries downwards from hi; lane l holds entry top - l. The
    // gathers are software-pipelined as in the forward walk: while chunk i
    // is processed, the splats of chunk i + 1 are in flight and the ids of
    // chunk i + 2 follow once chunk i's ids are staged. Every lane issues
    // every load (lanes below the range read its first entry and are
    // dropped by the range test).
    const float4* sp = reinterpret_cast<const float4*>(A.splats);
    auto id_clamped = [&](int64_t e) { return id_at<SRC>(A, (uint32_t)(e >= (int64_t)begin ? e : (int64_t)begin)); };
    auto gather = [&](uint32_t g, float4& r0, float4& r1, float4& r2) {
        const float4* q = sp + kSplatVec * (int64_t)g;
        r0 = q[0];
        r1 = q[1];
        r2 = q[2];
    };
    auto chunk = [&](int64_t top, const float4& q0, const float4& q1, const float4& q2, uint32_t& gcur,
                     uint32_t g_next, float4& n0, float4& n1, float4& n2) {
        const int64_t e = top - l;
        bool keep = e >= (int64_t)begin;
        gather(g_next, n0, n1, n2);
        Staged s;
        if (keep) {
            float s2;
            stage_splat(q0, q1, q2, ox, oy, s.a, s.b, s2);
            s.c = make_float2(s2, __int_as_float((int32_t)e));
            keep = block_may_touch(s.a.x, s.a.y, q1.x, q1.y, q1.z, q1.w, xa, xb, ya, yb);
        }
        const uint64_t m = ballot(keep);
        if (keep) {
            const uint32_t r = rank_in(m);
            st[r] = s;
            idw[r] = gcur;
        }
        gcur = id_clamped(e - 2 * kWave);  // this set's next chunk (i + 2)
        if (m == 0) return;
        wave_sync();
        const int cnt = __builtin_popcountll(m);
        for (int j = 0; j < cnt; ++j) {
            const Staged c = st[j];
            const int pos = __float_as_int(c.c.y);
            // the forward's per-pixel test, same operations
            const float dx = c.a.x - px;
            const float dy = c.a.y - py;
            const float wq = fmaf(c.a.z, dx, c.a.w * dy);
            const float q2 = fmaf(dx, wq, (c.b.x * dy) * dy);
            const float G = __builtin_amdgcn_exp2f(q2);
            const float araw = c.b.y * G;
            const bool comp = pos <= p.last && q2 <= 0.0f && araw >= kAlphaMin;
            if (ballot(comp) == 0) continue;
            float d[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (comp) {
                // the gradient arithmetic may fuse (the bars are not bitwise);
                // the compositing decision above repeats the forward exactly
#pragma clang fp contract(fast)
                const float alpha = fminf(kAlphaMax, araw);
                const float om = 1.0f - alpha;
                // 1 / (1 - alpha) to within an ulp (hardware reciprocal);
                // the gradients carry a 1e-3 tolerance, not the forward's
                // bit-exactness
                const float inv = __builtin_amdgcn_rcpf(om);
                T = T * inv;
                const float wt = alpha * T;
                d[6] = gr * wt;
                d[7] = gg * wt;
                d[8] = gb * wt;
                const float dLda = gaT * inv + gr * (T * c.b.z - Sr * inv) + gg * (T * c.b.w - Sg * inv) +
                                   gb * (T * c.c.x - Sb * inv);
                Sr = fmaf(wt, c.b.z, Sr);
                Sg = fmaf(wt, c.b.w, Sg);
                Sb = fmaf(wt, c.c.x, Sb);
                if (araw <= kAlphaMax) {
                    const float dq = dLda * araw * kLn2;  // dL/dq'
                    // q' = a' dx^2 + 2b' dx dy + c' dy^2 with (a', 2b', c') =
                    // kHalfLog2e (a, 2b, c); dx = mean_x - pixel_x
                    d[0] = dq * (2.0f * c.a.z * dx + c.a.w * dy);
                    d[1] = dq * (c.a.w * dx + 2.0f * c.b.x * dy);
                    const float k = dq * kHalfLog2e;
                    d[2] = k * dx * dx;
                    d[3] = 2.0f * k * dx * dy;
                    d[4] = k * dy * dy;
                    d[5] = dLda * G;
                }
            }
            const float mine = wave_sums9(d);
            if (sum_word != 0xF) unsafeAtomicAdd(d_splats + kGradWords * (int64_t)idw[j] + sum_word, mine);
        }
        wave_sync();
    };
    float4 a0, a1, a2, b0, b1, b2;
    uint32_t ida = id_clamped((int64_t)hi - l), idb;
    gather(ida, a0, a1, a2);
    idb = id_clamped((int64_t)hi - kWave - l);
    for (int64_t top = hi;;) {
        if (top < (int64_t)begin) break;
        chunk(top, a0, a1, a2, ida, idb, b0, b1, b2);
        top -= kWave;
        if (top < (int64_t)begin) break;
        chunk(top, b0, b1, b2, idb, ida, a0, a1, a2);
        top -= kWave;
    }
}

}  // namespace

hipError_t launch_raster_backward(const RasterArgs& a, const float* d_rgb, const float* d_alpha,
                                  const float* trans_in, const int32_t* last_in, float* d_splats, hipStream_t s) {
    const int T = a.tiles_x * a.tiles_y;
    if (T == 0) return hipSuccess;
    const int B = blocks_per_tile(a.tile), G = groups_per_tile(a.tile);
    const dim3 grid((unsigned)(T * G)), block((unsigned)(kWave * (B < 4 ? B : 4)));
    if (a.vals)
        hipLaunchKernelGGL((raster_bwd_kernel<SRC_VALS>), grid, block, 0, s, a, d_rgb, d_alpha, trans_in, last_in,
                           d_splats);
    else
        hipLaunchKernelGGL((raster_bwd_kernel<SRC_PAIRS>), grid, block, 0, s, a, d_rgb, d_alpha, trans_in, last_in,
                           d_splats);
    return hipGetLastError();
}

}  // namespace tgs
