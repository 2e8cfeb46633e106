// Single-pass exclusive prefix sums with decoupled look-back: each workgroup
// takes a ticket (so every workgroup it waits on is already running),
// publishes its aggregate, adds the aggregates / inclusive prefixes of its
// predecessors (a status word per workgroup: 2 flag bits + 62 value bits,
// exchanged with agent-scope relaxed atomics), publishes its inclusive
// prefix and writes its outputs. Items are read in coalesced rounds of 256.
// Used for the per-Gaussian entry offsets (fused with the visible-Gaussian
// list) and for the (tile, bin) counts -> bin offsets (fused with the
// per-XCD bases and the repair-bucket classification).
#include <algorithm>

#include "common.hpp"

namespace tgs {

namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 16;
constexpr int kPerBlock = kThreads * kRounds;
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;

__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t* lds) {
    constexpr int NW = kThreads / kWave;
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v += shfl_xor_u32(v, m);
    if (lane() == 0) lds[threadIdx.x / kWave] = v;
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s += lds[i];
    __syncthreads();
    return s;
}

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* lds) {
    constexpr int NW = kThreads / kWave;
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        const uint32_t lo = shfl_xor_u32((uint32_t)v, m), hi = shfl_xor_u32((uint32_t)(v >> 32), m);
        v += ((uint64_t)hi << 32) | lo;
    }
    if (lane() == 0) lds[threadIdx.x / kWave] = v;
    __syncthreads();
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s += lds[i];
    __syncthreads();
    return s;
}

// Exclusive scan of one uint32 per thread across the workgroup; *total
// receives the sum. Ends with a barrier, so lds is reusable.
__device__ __forceinline__ uint32_t block_excl_u32(uint32_t v, uint32_t* lds, uint32_t* total) {
    constexpr int NW = kThreads / kWave;
    const int w = threadIdx.x / kWave, l = lane();
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = shfl_up_u32(inc, d);
        if (l >= d) inc += o;
    }
    if (l == kWave - 1) lds[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const uint32_t t = lds[i];
        before += i < w ? t : 0u;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__device__ __forceinline__ uint64_t status_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void status_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of the values of workgroups 0..b-1. Waits only on workgroups with a
// smaller ticket, which are running or done, and stops at the first
// inclusive prefix (workgroup 0 always publishes one).
__device__ uint64_t look_back(const uint64_t* status, int64_t b) {
    uint64_t prefix = 0;
    for (int64_t p = b - 1; p >= 0; --p) {
        uint64_t s;
        do {
            s = status_load(&status[p]);
        } while ((s >> 62) == 0);
        prefix += s & kValMask;
        if ((s & ~kValMask) == kFlagInc) break;
    }
    return prefix;
}

// Publishes the aggregate, looks back and publishes the inclusive prefix;
// returns the exclusive prefix of workgroup b (thread 0 only).
__device__ __forceinline__ uint64_t publish_and_look_back(uint64_t* status, int64_t b, uint64_t agg) {
    if (b == 0) {
        status_store(&status[0], kFlagInc | agg);
        return 0;
    }
    status_store(&status[b], kFlagAgg | agg);
    const uint64_t prefix = look_back(status, b);
    status_store(&status[b], kFlagInc | ((prefix + agg) & kValMask));
    return prefix;
}

// ---- entry-emission scan ---------------------------------------------------
// Per Gaussian: x = number of tiles (entries), y = 1 if visible. Writes
// emit_off[g] (exclusive prefix of x), vis_ids[rank] = g for visible g, and
// counters[0] = M, counters[1] = V, counters[2] = M > capacity.

__global__ void __launch_bounds__(kThreads) emit_scan_kernel(const uint4* __restrict__ info, int64_t n, int tiles_x,
                                                             int tiles_y, uint32_t* __restrict__ emit_off,
                                                             uint32_t* __restrict__ vis_ids, uint32_t* ticket,
                                                             uint64_t* status_x, uint64_t* status_y,
                                                             int64_t* __restrict__ counters, int64_t capacity) {
    __shared__ uint32_t tk;
    __shared__ uint64_t lds64[kThreads / kWave];
    __shared__ uint32_t lds32[kThreads / kWave];
    __shared__ uint64_t pre[2];
    if (threadIdx.x == 0) tk = atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t b = tk;
    const int64_t nb = gridDim.x;
    const int64_t base = b * kPerBlock;
    uint32_t nt[kRounds];
    uint64_t sx = 0;
    uint32_t sy = 0;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t g = base + r * kThreads + threadIdx.x;
        int x0, y0, x1, y1;
        nt[r] = g < n ? (uint32_t)rect_of(info[g], tiles_x, tiles_y, x0, y0, x1, y1) : 0u;
        sx += nt[r];
        sy += nt[r] ? 1u : 0u;
    }
    const uint64_t ax = block_sum_u64(sx, lds64);
    const uint32_t ay = block_sum_u32(sy, lds32);
    if (threadIdx.x == 0) {
        pre[0] = publish_and_look_back(status_x, b, ax);
    } else if (threadIdx.x == kWave) {
        pre[1] = publish_and_look_back(status_y, b, ay);
    }
    __syncthreads();
    uint64_t cx = pre[0];
    uint32_t cy = (uint32_t)pre[1];
    if (b == nb - 1 && threadIdx.x == 0) {
        counters[0] = (int64_t)(cx + ax);
        counters[1] = (int64_t)(cy + ay);
        counters[2] = (int64_t)(cx + ax) > capacity ? 1 : 0;
        counters[3] = 0;
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t g = base + r * kThreads + threadIdx.x;
        uint32_t tx_, ty_;
        const uint32_t ex = block_excl_u32(nt[r], lds32, &tx_);
        const uint32_t ey = block_excl_u32(nt[r] ? 1u : 0u, lds32, &ty_);
        if (g < n) {
            emit_off[g] = (uint32_t)(cx + ex);
            if (nt[r]) vis_ids[cy + ey] = (uint32_t)g;
        }
        cx += tx_;
        cy += ty_;
    }
}

// ---- bin offsets from the per-XCD count copies ---------------------------

__host__ __device__ __forceinline__ int64_t blocks_for(int64_t n) {
    const int64_t b = (n + kPerBlock - 1) / kPerBlock;
    return b > 0 ? b : 1;
}

__device__ __forceinline__ uint32_t seg_total(const uint32_t* __restrict__ count, int64_t nseg, int64_t s) {
    uint32_t t = 0;
    if (s < nseg)
#pragma unroll
        for (int x = 0; x < kXcc; ++x) t += count[(int64_t)x * nseg + s];
    return t;
}

// bin_off[s] = exclusive prefix of the summed copies (bin_off[nseg] = M);
// count[x][s] becomes bin_off[s] + the counts of copies 0..x-1 in segment
// s. Every segment with two or more entries is appended to the list of its
// repair bucket (aggregated per wavefront and per workgroup: one global
// atomic per bucket and workgroup). Nothing is queued when the stream
// overflowed (counters[2]). With nseg_dev, the number of segments (and the
// stride of the count copies) is *nseg_dev and the grid is sized for its
// upper bound: workgroups past the last needed one leave after their ticket.
__global__ void __launch_bounds__(kThreads) bin_offsets_kernel(uint32_t* __restrict__ count, int64_t nseg_max,
                                                               const uint32_t* __restrict__ nseg_dev,
                                                               uint32_t* __restrict__ bin_off, uint32_t* ticket,
                                                               uint64_t* status, uint32_t* __restrict__ lists,
                                                               uint32_t* __restrict__ bucket_count,
                                                               const int64_t* __restrict__ counters) {
    __shared__ uint32_t tk;
    __shared__ uint32_t lds32[kThreads / kWave];
    __shared__ uint64_t pre;
    __shared__ uint32_t lcount[kBuckets], lbase[kBuckets];
    if (threadIdx.x == 0) tk = atomicAdd(ticket, 1u);
    if (threadIdx.x < kBuckets) lcount[threadIdx.x] = 0;
    __syncthreads();
    const int64_t b = tk;
    const int64_t nseg = nseg_dev ? (int64_t)*nseg_dev : nseg_max;
    const int64_t nb = blocks_for(nseg);
    if (b >= nb) return;
    const int64_t base = b * kPerBlock;
    const bool queue = counters[2] == 0;
    uint32_t v[kRounds];
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        v[r] = seg_total(count, nseg, base + r * kThreads + threadIdx.x);
        s += v[r];
    }
    const uint32_t agg = block_sum_u32(s, lds32);
    if (threadIdx.x == 0) pre = publish_and_look_back(status, b, agg);
    __syncthreads();
    uint32_t carry = (uint32_t)pre;
    if (b == nb - 1 && threadIdx.x == 0) bin_off[nseg] = carry + agg;
    int bk[kRounds];
    uint32_t slot[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t sg = base + r * kThreads + threadIdx.x;
        uint32_t tot;
        uint32_t run = carry + block_excl_u32(v[r], lds32, &tot);
        carry += tot;
        bk[r] = -1;
        slot[r] = 0;
        if (sg < nseg) {
            bin_off[sg] = run;
#pragma unroll
            for (int x = 0; x < kXcc; ++x) {
                uint32_t* c = count + (int64_t)x * nseg + sg;
                const uint32_t cv = *c;
                *c = run;
                run += cv;
            }
            if (queue) bk[r] = bucket_of(v[r]);
        }
        if (ballot(bk[r] >= 0) == 0) continue;
#pragma unroll
        for (int k = 0; k < kBuckets; ++k) {
            const uint64_t m = ballot(bk[r] == k);
            if (m == 0) continue;
            const int leader = __builtin_ctzll(m);
            uint32_t b0 = 0;
            if (lane() == leader) b0 = atomicAdd(&lcount[k], (uint32_t)__builtin_popcountll(m));
            b0 = shfl_u32(b0, leader);
            if (bk[r] == k) slot[r] = b0 + rank_in(m);
        }
    }
    __syncthreads();
    if (threadIdx.x < kBuckets)
        lbase[threadIdx.x] = lcount[threadIdx.x] ? atomicAdd(&bucket_count[threadIdx.x], lcount[threadIdx.x]) : 0u;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        if (bk[r] < 0) continue;
        const int64_t sg = base + r * kThreads + threadIdx.x;
        lists[(int64_t)bk[r] * nseg_max + lbase[bk[r]] + slot[r]] = (uint32_t)sg;
    }
}

// ---- per-tile segment bases -------------------------------------------------
// seg_base[t] = exclusive prefix of the per-tile bin counts, each clamped to
// 1..kmax and rounded down to a power of two; seg_base[T] = S.

__device__ __forceinline__ uint32_t pow2_bins(int32_t k, int kmax) {
    const uint32_t c = (uint32_t)(k < 1 ? 1 : (k > kmax ? kmax : k));
    return 1u << (31 - __builtin_clz(c));
}

__global__ void __launch_bounds__(kThreads) seg_base_kernel(const int32_t* __restrict__ kt, int64_t T, int kmax,
                                                            uint32_t* __restrict__ seg_base, uint2* __restrict__ tile_seg,
                                                            uint32_t* ticket, uint64_t* status) {
    __shared__ uint32_t tk;
    __shared__ uint32_t lds32[kThreads / kWave];
    __shared__ uint64_t pre;
    if (threadIdx.x == 0) tk = atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t b = tk;
    const int64_t nb = gridDim.x;
    const int64_t base = b * kPerBlock;
    uint32_t v[kRounds];
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t t = base + r * kThreads + threadIdx.x;
        v[r] = t < T ? pow2_bins(kt[t], kmax) : 0u;
        sum += v[r];
    }
    const uint32_t agg = block_sum_u32(sum, lds32);
    if (threadIdx.x == 0) pre = publish_and_look_back(status, b, agg);
    __syncthreads();
    uint32_t carry = (uint32_t)pre;
    if (b == nb - 1 && threadIdx.x == 0) seg_base[T] = carry + agg;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t t = base + r * kThreads + threadIdx.x;
        uint32_t tot;
        const uint32_t ex = block_excl_u32(v[r], lds32, &tot);
        if (t < T) {
            seg_base[t] = carry + ex;
            tile_seg[t] = make_uint2(carry + ex, 32u - (uint32_t)__builtin_ctz(v[r]));
        }
        carry += tot;
    }
}

__global__ void fill_u32_dyn_kernel(uint32_t* p, uint32_t v, const uint32_t* n_dev, int mult) {
    const int64_t n = (int64_t)*n_dev * mult;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

int64_t scan_blocks(int64_t n) { return n > 0 ? (n + kPerBlock - 1) / kPerBlock : 1; }

hipError_t launch_emit_scan(const uint32_t* info, int64_t n, int tiles_x, int tiles_y, uint32_t* emit_off,
                            uint32_t* vis_ids, uint32_t* ticket, uint64_t* status_x, uint64_t* status_y,
                            int64_t* counters, int64_t capacity, hipStream_t s) {
    hipLaunchKernelGGL(emit_scan_kernel, dim3((unsigned)scan_blocks(n)), dim3(kThreads), 0, s,
                       reinterpret_cast<const uint4*>(info), n, tiles_x, tiles_y, emit_off, vis_ids, ticket, status_x,
                       status_y, counters, capacity);
    return hipGetLastError();
}

hipError_t launch_bin_offsets(uint32_t* count, int64_t nseg, const uint32_t* nseg_dev, uint32_t* bin_off,
                              uint32_t* ticket, uint64_t* status, uint32_t* lists, uint32_t* bucket_count,
                              const int64_t* counters, hipStream_t s) {
    hipLaunchKernelGGL(bin_offsets_kernel, dim3((unsigned)scan_blocks(nseg)), dim3(kThreads), 0, s, count, nseg,
                       nseg_dev, bin_off, ticket, status, lists, bucket_count, counters);
    return hipGetLastError();
}

hipError_t launch_seg_base(const int32_t* per_tile_bins, int64_t T, int kmax, uint32_t* seg_base, uint2* tile_seg,
                           uint32_t* ticket, uint64_t* status, hipStream_t s) {
    hipLaunchKernelGGL(seg_base_kernel, dim3((unsigned)scan_blocks(T)), dim3(kThreads), 0, s, per_tile_bins, T, kmax,
                       seg_base, tile_seg, ticket, status);
    return hipGetLastError();
}

hipError_t launch_fill_u32_dyn(uint32_t* p, uint32_t v, const uint32_t* n_dev, int mult, int64_t max_n,
                               hipStream_t s) {
    if (max_n <= 0) return hipSuccess;
    int64_t grid = (max_n + 255) / 256;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(fill_u32_dyn_kernel, dim3((unsigned)grid), dim3(256), 0, s, p, v, n_dev, mult);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t grid = (n + 255) / 256;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)grid), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace tgs
