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

template <int SRC, bool COUNT>
__global__ void __launch_bounds__(256) raster_wave_kernel(RasterArgs A) {
    __shared__ Staged stage[4][kWave];
    const int w = threadIdx.x / kWave, l = lane();
    WaveBlock wb;
    if (!block_of_wave(A, w, wb)) return;
    const int x0 = wb.tx * A.tile, y0 = wb.ty * A.tile;
    float xa, xb, ya, yb;
    if (!block_box_at(wb.bx, wb.by, x0, y0, A.width, A.height, xa, xb, ya, yb)) return;  // block outside the image
    const int lx = wb.bx + (l & 7), ly = wb.by + (l >> 3);
    const int x = x0 + lx, y = y0 + ly;
    const bool inside = x < A.width && y < A.height;
    const bool bad = A.counters[2] != 0;
    const float ox = (float)x0, oy = (float)y0;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    Pix p{1.0f, 0.f, 0.f, 0.f, -1, 0, 0, 0, !inside || bad};
    const uint32_t begin = tile_begin(A, wb.t);
    const uint32_t end = bad ? begin : tile_end(A, wb.t);
    wave_forward<SRC, COUNT>(A, stage[w], wb.bi, begin, end, ox, oy, px, py, xa, xb, ya, yb, p);
    if (inside) write_pixel(A, x, y, p, bad);
}

// ---------------------------------------------------------------------------
// Heavy-tile split (16-pixel tiles, heaviest-first dispatch order). A pixel
// is composited sequentially over its tile's whole range, so the
// wavefronts of the few longest tiles decide when the WAVE raster ends.
// Workgroups of kSplitWaves = 4 wavefronts take, in this order: the first
// NA = order[T] tiles of the order (those with at least order[T + 1] >=
// A.split entries, at most kSplitTiles) one 8x8 block each, with 4 parts of
// the range; all other tiles one per workgroup, one wavefront per block, as
// in the WAVE raster. (Workgroups of 8 wavefronts, 8 parts for the split
// blocks and two other tiles per workgroup, were measured 3 % slower at
// 1080p and 10 % on the dense 500k training scene: a workgroup holds its
// slots until its slowest wavefront ends.) Part 0 of a block composites as
// usual; parts 1..
// composite every supported entry from a local transmittance of 1, giving
// local colour C_k and transmittance T_k. Each part then derives its
// entering transmittance T_in = T_0 ... T_{k-1}, or that the pixel stopped
// in an earlier part (a running product below 1e-4: the local
// transmittance only decreases, so a part's last value is its smallest
// test). A live part contributes T_in C_k and leaves T_in T_k, except where
// T_in T_k < 1e-4: the pixel stops inside it, and the part is walked again
// from T_in with the stop test. The part-0 wavefront adds the colours and
// takes T and the last id of the last live part. Images equal the unsplit
// ones up to the rounding of the regrouped products.
constexpr int kSplitWaves = 4;

struct PixLds {
    float r, g, b, T;
    int32_t last, ncon, nvis, nsup, live;
};

template <int SRC, bool COUNT>
__global__ void __launch_bounds__(kSplitWaves * kWave) raster_split_kernel(RasterArgs A) {
    __shared__ Staged stage[kSplitWaves][kWave];
    __shared__ float tloc[kSplitWaves][kWave];
    const int w = threadIdx.x / kWave, l = lane();
    const int T = A.tiles_x * A.tiles_y;
    const int na = min(min((int)A.order[T], T), kSplitTiles);
    const int i = (int)blockIdx.x;
    int slot, bi, parts, part;
    if (i < 4 * na) {
        slot = i >> 2;
        bi = i & 3;
        parts = kSplitWaves;
        part = w;
    } else {
        slot = na + (kSplitWaves / 4) * (i - 4 * na) + (w >> 2);
        bi = w & 3;
        parts = 1;
        part = 0;
        if (slot >= T) return;
    }
    const int t = (int)A.order[slot];
    const int bx = (bi & 1) * 8, by = (bi >> 1) * 8;
    const int x0 = (t % A.tiles_x) * kTile, y0 = (t / A.tiles_x) * kTile;
    float xa, xb, ya, yb;
    // block outside the image (uniform over the wavefronts of a split block)
    const bool valid = block_box_at(bx, by, x0, y0, A.width, A.height, xa, xb, ya, yb);
    if (parts == 1 && !valid) return;
    const int lx = bx + (l & 7), ly = by + (l >> 3);
    const int x = x0 + lx, y = y0 + ly;
    const bool inside = valid && x < A.width && y < A.height;
    const bool bad = A.counters[2] != 0;
    const float ox = (float)x0, oy = (float)y0;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    const uint32_t begin = tile_begin(A, t);
    const uint32_t end = bad ? begin : tile_end(A, t);
    const bool out = !inside || bad;
    Pix p{1.0f, 0.f, 0.f, 0.f, -1, 0, 0, 0, out};
    if (parts == 1) {
        wave_forward<SRC, COUNT>(A, stage[w], bi, begin, end, ox, oy, px, py, xa, xb, ya, yb, p);
        if (inside) write_pixel(A, x, y, p, bad);
        return;
    }
    const int w0 = w - part;  // the block's part-0 wavefront
    const uint64_t len = end - begin;
    const uint32_t qa = begin + (uint32_t)(len * (uint64_t)part / parts);
    const uint32_t qb = begin + (uint32_t)(len * (uint64_t)(part + 1) / parts);
    // part 0 composites exactly; parts 1.. composite every supported entry
    // from a local transmittance of 1. After every chunk a part publishes
    // its running local transmittance (0 once part 0's pixel has stopped)
    // and drops the pixels whose earlier parts' running product is already
    // below 1e-4: the final product can only be smaller, so those pixels
    // stop before this part. Reading a stale value only delays the drop.
    tloc[w][l] = 1.0f;
    __syncthreads();
    auto progress = [&](Pix& q) {
        tloc[w][l] = (part == 0 && q.done) ? 0.0f : q.T;
        if (part > 0) {
            float prod = 1.0f;
            for (int j = 0; j < part; ++j) prod *= tloc[w0 + j][l];
            q.done = q.done || prod < kTMin;
        }
    };
    if (valid)
        wave_forward<SRC, COUNT>(A, stage[w], bi, qa, qb, ox, oy, px, py, xa, xb, ya, yb, p, part > 0, progress);
    // (a pixel that stopped inside part 0 publishes 0: every later part is dead)
    tloc[w][l] = (part == 0 && p.done) ? 0.0f : p.T;
    __syncthreads();
    float t_in = 1.0f;
    bool dead = out;
    for (int j = 0; j < part; ++j) {
        const float tt = t_in * tloc[w0 + j][l];
        dead = dead || tt < kTMin;
        t_in = dead ? t_in : tt;
    }
    // a pixel whose running product falls below 1e-4 inside this part stops
    // in it: the part is walked again for those pixels, from t_in with the
    // stop test (the other lanes are marked done, which leaves them as they are)
    const bool fix = part > 0 && !dead && t_in * p.T < kTMin;
    if (ballot(fix) != 0) {
        if (fix) p = Pix{t_in, 0.f, 0.f, 0.f, -1, 0, 0, 0, false};
        const bool keep_done = p.done;
        p.done = !fix;
        wave_forward<SRC, COUNT>(A, stage[w], bi, qa, qb, ox, oy, px, py, xa, xb, ya, yb, p);
        p.done = keep_done;
    }
    if (part > 0 && !fix) {
        p.r *= t_in;
        p.g *= t_in;
        p.b *= t_in;
        p.T *= t_in;
    }
    if (part > 0) reinterpret_cast<PixLds*>(stage[w])[l] = PixLds{p.r, p.g, p.b, p.T, p.last, p.ncon, p.nvis, p.nsup,
                                                                   dead ? 0 : 1};
    __syncthreads();
    if (part > 0) return;
    for (int j = 1; j < parts; ++j) {
        const PixLds r = reinterpret_cast<const PixLds*>(stage[w + j])[l];
        if (!r.live) continue;  // the pixel stopped in an earlier part
        p.r += r.r;
        p.g += r.g;
        p.b += r.b;
        p.T = r.T;
        p.last = r.last >= 0 ? r.last : p.last;
        if (COUNT) {
            p.ncon += r.ncon;
            p.nvis += r.nvis;
            p.nsup += r.nsup;
        }
    }
    if (inside) write_pixel(A, x, y, p, bad);
}

template <int SRC>
hipError_t split_dispatch(const RasterArgs& a, hipStream_t s) {
    const int T = a.tiles_x * a.tiles_y;
    // split blocks first (one workgroup per 8x8 block), then one light tile
    // per workgroup; workgroups past the last item leave at once
    const int grid = 4 * std::min(T, kSplitTiles) + (T + kSplitWaves / 4 - 1) / (kSplitWaves / 4);
    if (a.n_visit || a.n_support || a.n_contrib)
        hipLaunchKernelGGL((raster_split_kernel<SRC, true>), dim3(grid), dim3(kSplitWaves * kWave), 0, s, a);
    else
        hipLaunchKernelGGL((raster_split_kernel<SRC, false>), dim3(grid), dim3(kSplitWaves * kWave), 0, s, a);
    return hipGetLastError();
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
    if (a.split) return split_dispatch<SRC>(a, s);
    const int T = a.tiles_x * a.tiles_y;
    const int B = blocks_per_tile(a.tile), G = groups_per_tile(a.tile);
    const dim3 grid((unsigned)(T * G)), block((unsigned)(kWave * (B < 4 ? B : 4)));
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
