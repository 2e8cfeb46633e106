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
// Workgroups of 4 wavefronts take, in this order: the first NA = order[T]
// tiles of the order (those with at least order[T + 1] >= A.split entries,
// at most kSplitTiles) one 8x8 block each, a 4x4 quarter of it per
// wavefront, in the quad walk (four lanes per pixel, four entries per
// step, the per-pixel chain unchanged); all other tiles one per workgroup,
// one wavefront per block, as in the WAVE raster. Every wavefront walks
// independently, so images, last ids and counts are bitwise those of the
// WAVE raster.
template <int SRC, bool COUNT>
__global__ void __launch_bounds__(4 * kWave) raster_split_kernel(RasterArgs A) {
    __shared__ Staged stage[4][kWave];
    __shared__ float4 colq[4][3 * kWave / 4];
    const int w = threadIdx.x / kWave, l = lane();
    const int T = A.tiles_x * A.tiles_y;
    const int na = min(min((int)A.order[T], T), kSplitTiles);
    const int i = (int)blockIdx.x;
    const bool heavy = i < 4 * na;
    int slot, bi;
    if (heavy) {
        slot = i >> 2;
        bi = i & 3;
    } else {
        slot = na + (i - 4 * na);
        bi = w;
        if (slot >= T) return;
    }
    const int t = (int)A.order[slot];
    const int x0 = (t % A.tiles_x) * kTile, y0 = (t / A.tiles_x) * kTile;
    const bool bad = A.counters[2] != 0;
    const float ox = (float)x0, oy = (float)y0;
    const uint32_t begin = tile_begin(A, t);
    const uint32_t end = bad ? begin : tile_end(A, t);
    float xa, xb, ya, yb;
    if (!heavy) {
        const int bx = (bi & 1) * 8, by = (bi >> 1) * 8;
        if (!block_box_at(bx, by, x0, y0, A.width, A.height, xa, xb, ya, yb)) return;  // block outside the image
        const int lx = bx + (l & 7), ly = by + (l >> 3);
        const int x = x0 + lx, y = y0 + ly;
        const bool inside = x < A.width && y < A.height;
        const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
        Pix p{1.0f, 0.f, 0.f, 0.f, -1, 0, 0, 0, !inside || bad};
        wave_forward<SRC, COUNT>(A, stage[w], bi, begin, end, ox, oy, px, py, xa, xb, ya, yb, p);
        if (inside) write_pixel(A, x, y, p, bad);
        return;
    }
    // quarter w of block bi: pixel (l / 4) of the quarter, role l % 4
    const int qx = (bi & 1) * 8 + (w & 1) * 4, qy = (bi >> 1) * 8 + (w >> 1) * 4;
    const int nx = min(4, A.width - (x0 + qx)), ny = min(4, A.height - (y0 + qy));
    if (nx <= 0 || ny <= 0) return;  // quarter outside the image
    xa = qx + 0.5f;
    xb = qx + nx - 0.5f;
    ya = qy + 0.5f;
    yb = qy + ny - 0.5f;
    const int pi = l >> 2, k = l & 3;
    const int lx = qx + (pi & 3), ly = qy + (pi >> 2);
    const int x = x0 + lx, y = y0 + ly;
    const bool inside = x < A.width && y < A.height;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    const bool live = inside && !bad;
    QuadPix p{live ? 1.0f : 0.0f, 1.0f, 0.0f, -1, 0, 0, 0};
    quad_forward<SRC, COUNT>(A, stage[w], reinterpret_cast<float*>(colq[w]), begin, end, ox, oy, px, py, xa, xb,
                             ya, yb, p);
    write_quad<COUNT>(A, x, y, k, inside, p, bad);
}

template <int SRC>
hipError_t split_dispatch(const RasterArgs& a, hipStream_t s) {
    const int T = a.tiles_x * a.tiles_y;
    // split blocks first (one workgroup per 8x8 block), then one light tile
    // per workgroup; workgroups past the last item leave at once
    const int grid = 4 * std::min(T, kSplitTiles) + T;
    if (a.n_visit || a.n_support || a.n_contrib)
        hipLaunchKernelGGL((raster_split_kernel<SRC, true>), dim3(grid), dim3(4 * kWave), 0, s, a);
    else
        hipLaunchKernelGGL((raster_split_kernel<SRC, false>), dim3(grid), dim3(4 * kWave), 0, s, a);
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
