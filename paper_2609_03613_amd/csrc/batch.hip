// Batched rendering of several cameras (views) in one persistent raster
// launch. The paper renders one camera at a time; this is the multi-view
// extension of its raster traversal (Algorithm "Binned raster traversal
// after repair"), with each view's stream built by the ordinary tgs_bin.
//
// Work items are (view, tile, 8x8 block) triples. Two small launches order
// them heaviest tile first over all views (a counting sort on the bit
// length of the tile's entry count, blocks of one tile adjacent), and the
// items are dealt round-robin into 8 partitions. The persistent kernel's
// wavefronts then pull items one at a time, first from the partition of
// the XCD they run on, then from the others, with device-scope atomic
// cursors, so every item is taken exactly once and every wavefront ends
// when all partitions are drained. Each item runs the WAVE raster's block
// walk and writes the block's pixels, so images are bit-identical to
// per-view tgs_rasterize calls with the same tile size and stream.
#include "raster.hpp"

namespace tgs {

namespace {

using namespace raster;

constexpr int kHistBuckets = 33;  // bit length of the entry count (0 = empty tile last)
constexpr int kParts = 8;

__device__ __forceinline__ int view_of(const BatchArgs& B, int64_t i) {
    int v = 0;
    while (v + 1 < B.nv && (int64_t)B.tile_base[v + 1] <= i) ++v;
    return v;
}

__device__ __forceinline__ RasterArgs view_args(const BatchArgs& B, int v) {
    const BatchView& V = B.v[v];
    RasterArgs A{};
    A.splats = V.splats;
    A.offsets = V.offsets;
    A.stride = V.stride;
    A.seg_base = V.seg_base;
    A.vals = V.vals;
    A.pairs = V.pairs;
    A.counters = V.counters;
    A.width = V.width;
    A.height = V.height;
    A.tile = V.tile;
    A.tiles_x = V.tiles_x;
    A.tiles_y = V.tiles_y;
    A.bg[0] = B.bg[0];
    A.bg[1] = B.bg[1];
    A.bg[2] = B.bg[2];
    A.rgb = V.rgb;
    A.alpha = V.alpha;
    A.last = V.last;
    return A;
}

__device__ __forceinline__ int count_bucket(uint32_t c) { return c ? __builtin_clz(c) : 32; }

// Wave-aggregated add of `amount` to ctr[b] (one LDS atomic per distinct b
// in the wavefront); returns the lane's offset inside its bucket.
__device__ __forceinline__ uint32_t wave_bucket_add(uint32_t* ctr, int b, uint32_t amount, bool active) {
    uint32_t slot = 0;
    uint64_t pending = ballot(active);
    while (pending) {
        const int leader = __builtin_ctzll(pending);
        const int lb = (int)shfl_u32((uint32_t)b, leader);
        const bool mine = active && b == lb;
        const uint64_t m = ballot(mine);
        // exclusive prefix of `amount` over the lanes of this bucket
        uint32_t pre = 0, tot = 0;
        for (uint64_t q = m; q; q &= q - 1) {
            const int ln = __builtin_ctzll(q);
            const uint32_t a = shfl_u32(amount, ln);
            if (ln < lane()) pre += a;
            tot += a;
        }
        uint32_t base = 0;
        if (lane() == leader) base = atomicAdd(&ctr[lb], tot);
        base = shfl_u32(base, leader);
        if (mine) slot = base + pre;
        pending &= ~m;
    }
    return slot;
}

// (1) blocks per bucket over every (view, tile).
__global__ void __launch_bounds__(256) batch_hist_kernel(BatchArgs B, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[kHistBuckets];
    if (threadIdx.x < kHistBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i < (int64_t)B.tile_base[B.nv];
    int b = 0;
    uint32_t nb = 0;
    if (act) {
        const int v = view_of(B, i);
        const RasterArgs A = view_args(B, v);
        const int t = (int)(i - B.tile_base[v]);
        b = count_bucket(tile_end(A, t) - tile_begin(A, t));
        nb = (uint32_t)blocks_per_tile(A.tile);
    }
    (void)wave_bucket_add(h, b, nb, act);
    __syncthreads();
    if (threadIdx.x < kHistBuckets && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// (2) placement: item k of the ordered list goes to partition k % 8, slot
// k / 8; items are view << 28 | block << 24 | tile.
__global__ void __launch_bounds__(256) batch_place_kernel(BatchArgs B, const uint32_t* __restrict__ hist,
                                                          uint32_t* __restrict__ cursor, uint32_t* __restrict__ work,
                                                          int64_t part_stride) {
    __shared__ uint32_t h[kHistBuckets], base[kHistBuckets];
    if (threadIdx.x < kHistBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i < (int64_t)B.tile_base[B.nv];
    int b = 0, v = 0, t = 0;
    uint32_t nb = 0;
    if (act) {
        v = view_of(B, i);
        const RasterArgs A = view_args(B, v);
        t = (int)(i - B.tile_base[v]);
        b = count_bucket(tile_end(A, t) - tile_begin(A, t));
        nb = (uint32_t)blocks_per_tile(A.tile);
    }
    const uint32_t slot = wave_bucket_add(h, b, nb, act);
    __syncthreads();
    if (threadIdx.x < kHistBuckets) {
        uint32_t start = 0;
        for (int k = 0; k < (int)threadIdx.x; ++k) start += hist[k];
        base[threadIdx.x] = h[threadIdx.x] ? start + atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]) : 0u;
    }
    __syncthreads();
    if (!act) return;
    const uint32_t k0 = base[b] + slot;
    for (uint32_t j = 0; j < nb; ++j) {
        const uint32_t k = k0 + j;
        work[(int64_t)(k % kParts) * part_stride + k / kParts] = ((uint32_t)v << 28) | (j << 24) | (uint32_t)t;
    }
}

// Number of items in partition p of `total` dealt round-robin.
__device__ __forceinline__ uint32_t part_count(uint32_t total, int p) {
    return total / kParts + ((uint32_t)p < total % kParts ? 1u : 0u);
}

__device__ __forceinline__ void run_item(const BatchArgs& B, uint32_t item, Staged* st) {
    const int v = (int)(item >> 28), bi = (int)((item >> 24) & 15u), t = (int)(item & 0xFFFFFFu);
    const RasterArgs A = view_args(B, v);
    const int nb = A.tile >> 3;
    const int bx = (bi % nb) * 8, by = (bi / nb) * 8;
    const int tx = t % A.tiles_x, ty = t / A.tiles_x;
    const int x0 = tx * A.tile, y0 = ty * A.tile;
    float xa, xb, ya, yb;
    if (!block_box_at(bx, by, x0, y0, A.width, A.height, xa, xb, ya, yb)) return;
    const int l = lane();
    const int lx = bx + (l & 7), ly = by + (l >> 3);
    const int x = x0 + lx, y = y0 + ly;
    const bool inside = x < A.width && y < A.height;
    const bool bad = A.counters[2] != 0;
    const float ox = (float)x0, oy = (float)y0;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    Pix p{1.0f, 0.f, 0.f, 0.f, -1, 0, 0, 0, !inside || bad};
    const uint32_t begin = tile_begin(A, t);
    const uint32_t end = bad ? begin : tile_end(A, t);
    if (A.vals)
        wave_forward<SRC_VALS, false>(A, st, bi, begin, end, ox, oy, px, py, xa, xb, ya, yb, p);
    else
        wave_forward<SRC_PAIRS, false>(A, st, bi, begin, end, ox, oy, px, py, xa, xb, ya, yb, p);
    if (inside) write_pixel(A, x, y, p, bad);
}

__device__ __forceinline__ uint32_t take(uint32_t* cur) {
    uint32_t i = 0;
    if (lane() == 0) i = __hip_atomic_fetch_add(cur, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)i);
}

__global__ void __launch_bounds__(256) raster_persistent_kernel(BatchArgs B, const uint32_t* __restrict__ work,
                                                                int64_t part_stride, uint32_t* __restrict__ cursors,
                                                                uint32_t total) {
    __shared__ Staged stage[4][kWave];
    Staged* st = stage[threadIdx.x / kWave];
    const int x = xcc_id();
    for (int k = 0; k < kParts; ++k) {
        const int p = (x + k) % kParts;
        const uint32_t n = part_count(total, p);
        uint32_t* cur = cursors + p * 16;  // one 64-byte line per cursor
        for (uint32_t i = take(cur); i < n; i = take(cur)) run_item(B, work[(int64_t)p * part_stride + i], st);
    }
}

}  // namespace

hipError_t launch_raster_batch(const BatchArgs& b, uint32_t* ctl, uint32_t* work, int64_t total_blocks, int grid,
                               hipStream_t s) {
    const int64_t ntiles = b.tile_base[b.nv];
    if (ntiles == 0) return hipSuccess;
    // ctl: [0, 33) histogram, [64, 97) cursors, [128, 256) partition cursors
    const int64_t part_stride = (total_blocks + kParts - 1) / kParts;
    const unsigned g = (unsigned)((ntiles + 255) / 256);
    hipLaunchKernelGGL(batch_hist_kernel, dim3(g), dim3(256), 0, s, b, ctl);
    hipLaunchKernelGGL(batch_place_kernel, dim3(g), dim3(256), 0, s, b, ctl, ctl + 64, work, part_stride);
    hipLaunchKernelGGL(raster_persistent_kernel, dim3((unsigned)grid), dim3(256), 0, s, b, work, part_stride,
                       ctl + 128, (uint32_t)total_blocks);
    return hipGetLastError();
}

}  // namespace tgs
