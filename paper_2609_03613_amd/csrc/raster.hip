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

#include <algorithm>

#include "raster.hpp"

namespace tgs {

namespace {

using namespace raster;

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
    const uint32_t begin = tile_begin(A, t);
    const uint32_t end = bad ? begin : tile_end(A, t);
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

// Heavy-tile split. A pixel is composited sequentially over its tile's
// whole range, so the wavefronts of the few longest tiles decide when the
// kernel ends. With A.split, the first NS = min(order[T], kSplitTiles)
// tiles of the dispatch order (those with at least A.split entries) get one
// workgroup per 8x8 block instead of one per tile, whose 4 wavefronts take
// the 4 quarters of the range in two passes. Pass 1: each wavefront finds
// its quarter's local transmittance T_k (every supported entry applied, no
// stop test). From these each wavefront derives its entering transmittance
// T_in = T_0 ... T_{k-1}, or that the pixel stopped in an earlier quarter
// (a running product below 1e-4: the local transmittance only decreases, so
// a quarter's last value is its smallest test). Pass 2: each wavefront
// composites its quarter from T_in with the stop test, and the quarter-0
// wavefront adds the colours and takes T and the last id of the last live
// quarter. Images equal the unsplit ones up to the rounding of the
// regrouped products; the critical path is about half a tile walk.
constexpr int kSplitTiles = 1024;

struct PixLds {
    float r, g, b, T;
    int32_t last, ncon, nvis, nsup, live;
};

template <int SRC, bool COUNT>
__global__ void __launch_bounds__(256) raster_wave_kernel(RasterArgs A) {
    __shared__ Staged stage[4][kWave];
    __shared__ float tloc[4][kWave];
    const int w = threadIdx.x / kWave, l = lane();
    WaveBlock wb;
    bool heavy = false;
    if (A.split) {
        // 16-pixel tiles, dispatch order present
        const int T = A.tiles_x * A.tiles_y;
        const int ns = min(min((int)A.order[T], T), kSplitTiles);
        const int i = (int)blockIdx.x;
        int slot;
        if (i < 4 * ns) {
            heavy = true;
            slot = i >> 2;
            wb.bi = i & 3;
        } else {
            slot = ns + (i - 4 * ns);
            if (slot >= T) return;
            wb.bi = w;
        }
        wb.t = (int)A.order[slot];
        wb.tx = wb.t % A.tiles_x;
        wb.ty = wb.t / A.tiles_x;
        wb.bx = (wb.bi & 1) * 8;
        wb.by = (wb.bi >> 1) * 8;
    } else if (!block_of_wave(A, w, wb)) {
        return;
    }
    const int x0 = wb.tx * A.tile, y0 = wb.ty * A.tile;
    float xa, xb, ya, yb;
    // block outside the image (uniform over a heavy tile's workgroup)
    if (!block_box_at(wb.bx, wb.by, x0, y0, A.width, A.height, xa, xb, ya, yb)) return;
    const int lx = wb.bx + (l & 7), ly = wb.by + (l >> 3);
    const int x = x0 + lx, y = y0 + ly;
    const bool inside = x < A.width && y < A.height;
    const bool bad = A.counters[2] != 0;
    const float ox = (float)x0, oy = (float)y0;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    const uint32_t begin = tile_begin(A, wb.t);
    const uint32_t end = bad ? begin : tile_end(A, wb.t);
    Pix p{1.0f, 0.f, 0.f, 0.f, -1, 0, 0, 0, !inside || bad};
    if (!heavy) {
        wave_forward<SRC, COUNT>(A, stage[w], wb.bi, begin, end, ox, oy, px, py, xa, xb, ya, yb, p);
        if (inside) write_pixel(A, x, y, p, bad);
        return;
    }
    const uint64_t len = end - begin;
    const uint32_t qa = begin + (uint32_t)(len * (uint64_t)w / 4), qb = begin + (uint32_t)(len * (uint64_t)(w + 1) / 4);
    const bool out = !inside || bad;
    float t_in = 1.0f;
    bool dead = out;
    for (int pass = 0; pass < 2; ++pass) {
        p = Pix{t_in, 0.f, 0.f, 0.f, -1, 0, 0, 0, dead};
        wave_forward<SRC, COUNT>(A, stage[w], wb.bi, qa, qb, ox, oy, px, py, xa, xb, ya, yb, p, pass == 0);
        if (pass == 0) {
            tloc[w][l] = p.T;
            __syncthreads();
            for (int j = 0; j < w; ++j) {
                const float tt = t_in * tloc[j][l];
                dead = dead || tt < kTMin;
                t_in = dead ? t_in : tt;
            }
        }
    }
    if (w > 0) reinterpret_cast<PixLds*>(stage[w])[l] = PixLds{p.r, p.g, p.b, p.T, p.last, p.ncon, p.nvis, p.nsup,
                                                                dead ? 0 : 1};
    __syncthreads();
    if (w > 0) return;
    for (int j = 1; j < 4; ++j) {
        const PixLds r = reinterpret_cast<const PixLds*>(stage[j])[l];
        p.r += r.r;
        p.g += r.g;
        p.b += r.b;
        p.T = r.live ? r.T : p.T;
        p.last = r.live && r.last >= 0 ? r.last : p.last;
        if (COUNT) {
            p.ncon += r.ncon;
            p.nvis += r.nvis;
            p.nsup += r.nsup;
        }
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
    const int B = blocks_per_tile(a.tile), G = groups_per_tile(a.tile);
    const int extra = a.split ? 3 * std::min(T, kSplitTiles) : 0;
    const dim3 grid((unsigned)(T * G + extra)), block((unsigned)(kWave * (B < 4 ? B : 4)));
    if (a.n_visit || a.n_support || a.n_contrib)
        hipLaunchKernelGGL((raster_wave_kernel<SRC, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((raster_wave_kernel<SRC, false>), grid, block, 0, s, a);
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
    RasterArgs b = a;
    // the split needs the dispatch order, 16-pixel tiles and gathered entries
    if (!(b.order && b.tile == kTile && !b.records && !b.masks)) b.split = 0;
    if (b.records) return wave_dispatch<SRC_PACKED>(b, s);
    if (b.vals) return wave_dispatch<SRC_VALS>(b, s);
    return wave_dispatch<SRC_PAIRS>(b, s);
}

}  // namespace tgs
