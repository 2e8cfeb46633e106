// Exclusive prefix sums, two launches each: (1) per-block partial sums, the
// last block to finish scanning the partials; (2) per-block apply. Items are
// read in coalesced rounds of 256 per workgroup. Used for the per-Gaussian
// entry offsets (fused with the visible-Gaussian ranks and the depth-range
// sampling) and for the (tile, bin) counts -> bin offsets (fused with the
// per-XCD bases and the repair-bucket classification).
#include "common.hpp"

namespace tgs {

namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 16;
constexpr int kPerBlock = kThreads * kRounds;

struct U64x2 {
    uint64_t x, y;
};
__device__ __forceinline__ U64x2 operator+(U64x2 a, U64x2 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ U64x2 operator-(U64x2 a, U64x2 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ void set_zero(uint32_t& v) { v = 0u; }
__device__ __forceinline__ void set_zero(U64x2& v) { v.x = 0ull; v.y = 0ull; }

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int d) {
    uint32_t lo = shfl_up_u32((uint32_t)v, d), hi = shfl_up_u32((uint32_t)(v >> 32), d);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t shfl_up_v(uint32_t v, int d) { return shfl_up_u32(v, d); }
__device__ __forceinline__ U64x2 shfl_up_v(U64x2 v, int d) { return {shfl_up_u64(v.x, d), shfl_up_u64(v.y, d)}; }

template <typename V>
__device__ __forceinline__ V wave_incl(V v) {
    const int l = lane();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        V o = shfl_up_v(v, d);
        if (l >= d) v = v + o;
    }
    return v;
}

// Exclusive scan of one value per thread across the workgroup (NT threads).
// Returns the thread's exclusive prefix; *total receives the workgroup sum.
// lds must hold NT / 64 + 1 values. Ends with a barrier, so lds is reusable.
template <typename V, int NT>
__device__ __forceinline__ V block_excl(V v, V* lds, V* total) {
    constexpr int NW = NT / kWave;
    const int w = threadIdx.x / kWave;
    const V inc = wave_incl(v);
    if (lane() == kWave - 1) lds[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        V acc;
        set_zero(acc);
        for (int i = 0; i < NW; ++i) {
            V t = lds[i];
            lds[i] = acc;
            acc = acc + t;
        }
        lds[NW] = acc;
    }
    __syncthreads();
    const V r = lds[w] + (inc - v);
    *total = lds[NW];
    __syncthreads();
    return r;
}

// Called by every block after writing its partial: the block that finishes
// last replaces the partials by their exclusive scan, writes the total and
// resets the done counter for the next launch. The device-scope fences make
// the partials of all XCDs visible to it.
template <typename V>
__device__ __forceinline__ bool last_block_scan(V* partials, int64_t nb, uint32_t* done, V* lds, V* total_out) {
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) is_last = atomicAdd(done, 1u) == (uint32_t)(nb - 1);
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    V carry;
    set_zero(carry);
    for (int64_t base = 0; base < nb; base += kThreads) {
        const int64_t i = base + threadIdx.x;
        V v;
        set_zero(v);
        if (i < nb) v = partials[i];
        V tot;
        const V ex = block_excl<V, kThreads>(v, lds, &tot);
        if (i < nb) partials[i] = carry + ex;
        carry = carry + tot;
    }
    if (threadIdx.x == 0) {
        *total_out = carry;
        *done = 0;
    }
    return true;
}

// ---- entry-emission scan over the info array --------------------------------
// x: number of tiles (entries) per Gaussian, y: 1 if visible.

__device__ __forceinline__ U64x2 emit_val(const uint4* info, int64_t g, int64_t n, int tiles_x, int tiles_y) {
    U64x2 r;
    set_zero(r);
    if (g < n) {
        int x0, y0, x1, y1;
        const int nt = rect_of(info[g], tiles_x, tiles_y, x0, y0, x1, y1);
        r.x = (uint64_t)nt;
        r.y = nt > 0 ? 1ull : 0ull;
    }
    return r;
}

// Also clears the `zero_words` control words (count copies, repair queues)
// that later kernels of the same tgs_bin call accumulate into.
__global__ void __launch_bounds__(kThreads) emit_reduce(const uint4* __restrict__ info, int64_t n, int tiles_x,
                                                        int tiles_y, U64x2* __restrict__ partials, uint32_t* done,
                                                        int64_t* __restrict__ counters, int64_t capacity,
                                                        uint32_t* __restrict__ zero, int64_t zero_words) {
    __shared__ U64x2 lds[kThreads / kWave + 1];
    const int64_t nb = gridDim.x;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < zero_words; i += (int64_t)gridDim.x * kThreads)
        zero[i] = 0u;
    U64x2 s;
    set_zero(s);
    const int64_t base = (int64_t)blockIdx.x * kPerBlock;
    for (int r = 0; r < kRounds; ++r) s = s + emit_val(info, base + r * kThreads + threadIdx.x, n, tiles_x, tiles_y);
    U64x2 total;
    (void)block_excl<U64x2, kThreads>(s, lds, &total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
    U64x2 all;
    if (last_block_scan(partials, nb, done, lds, &all) && threadIdx.x == 0) {
        counters[0] = (int64_t)all.x;
        counters[1] = (int64_t)all.y;
        counters[2] = (int64_t)all.x > capacity ? 1 : 0;
        counters[3] = 0;
    }
}

// Writes emit_off[g] and the depth-range samples. With V visible Gaussians
// and S samples: all visible depths when V <= S (sample[rank] = depth),
// otherwise the visible Gaussians at ranks floor(i V / S), i < S, each
// stored at its i. A rank r is such a rank iff i = ceil(r S / V) < S and
// floor(i V / S) == r.
__global__ void __launch_bounds__(kThreads) emit_apply(const uint4* __restrict__ info, int64_t n, int tiles_x,
                                                       int tiles_y, uint32_t* __restrict__ emit_off,
                                                       const U64x2* __restrict__ block_off,
                                                       const int64_t* __restrict__ counters,
                                                       uint32_t* __restrict__ sample, int S) {
    __shared__ U64x2 lds[kThreads / kWave + 1];
    const int64_t V = counters[1];
    U64x2 carry = block_off[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kPerBlock;
    for (int r = 0; r < kRounds; ++r) {
        if (base + (int64_t)r * kThreads >= n) break;  // uniform across the workgroup
        const int64_t g = base + r * kThreads + threadIdx.x;
        const U64x2 v = emit_val(info, g, n, tiles_x, tiles_y);
        U64x2 tot;
        const U64x2 run = carry + block_excl<U64x2, kThreads>(v, lds, &tot);
        carry = carry + tot;
        if (g < n) {
            emit_off[g] = (uint32_t)run.x;
            if (v.y) {
                const int64_t rk = (int64_t)run.y;
                int64_t i = -1;
                if (V <= S) {
                    i = rk;
                } else {
                    const int64_t c = (rk * S + V - 1) / V;
                    if (c < S && (c * V) / S == rk) i = c;
                }
                if (i >= 0) sample[i] = info[g].x;
            }
        }
    }
}

// ---- bin offsets from the per-XCD count copies ---------------------------

__device__ __forceinline__ uint32_t seg_total(const uint32_t* __restrict__ count, int64_t nseg, int64_t s) {
    uint32_t t = 0;
    if (s < nseg)
#pragma unroll
        for (int x = 0; x < kXcc; ++x) t += count[(int64_t)x * nseg + s];
    return t;
}

__global__ void __launch_bounds__(kThreads) bo_reduce(const uint32_t* __restrict__ count, int64_t nseg,
                                                      uint32_t* __restrict__ partials, uint32_t* done,
                                                      uint32_t* __restrict__ total_out) {
    __shared__ uint32_t lds[kThreads / kWave + 1];
    const int64_t nb = gridDim.x;
    const int64_t base = (int64_t)blockIdx.x * kPerBlock;
    uint32_t s = 0;
    for (int r = 0; r < kRounds; ++r) s += seg_total(count, nseg, base + r * kThreads + threadIdx.x);
    uint32_t total;
    (void)block_excl<uint32_t, kThreads>(s, lds, &total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
    (void)last_block_scan(partials, nb, done, lds, total_out);
}

// bin_off[s] = exclusive prefix of the summed copies; count[x][s] becomes
// bin_off[s] + the counts of copies 0..x-1 in segment s. Every segment with
// two or more entries is appended to the list of its repair bucket
// (aggregated per wavefront and per workgroup: one global atomic per bucket
// and workgroup). Nothing is queued when the stream overflowed (counters[2]).
__global__ void __launch_bounds__(kThreads) bo_apply(uint32_t* __restrict__ count, int64_t nseg,
                                                     uint32_t* __restrict__ bin_off,
                                                     const uint32_t* __restrict__ block_off,
                                                     uint32_t* __restrict__ lists, uint32_t* __restrict__ bucket_count,
                                                     const int64_t* __restrict__ counters) {
    __shared__ uint32_t lds[kThreads / kWave + 1];
    __shared__ uint32_t lcount[kBuckets], lbase[kBuckets];
    if (threadIdx.x < kBuckets) lcount[threadIdx.x] = 0;
    const bool queue = counters[2] == 0;
    uint32_t carry = block_off[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kPerBlock;
    int bk[kRounds];
    uint32_t slot[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t s = base + r * kThreads + threadIdx.x;
        const uint32_t v = seg_total(count, nseg, s);
        uint32_t tot;
        uint32_t run = carry + block_excl<uint32_t, kThreads>(v, lds, &tot);
        carry += tot;
        bk[r] = -1;
        slot[r] = 0;
        if (s < nseg) {
            bin_off[s] = run;
#pragma unroll
            for (int x = 0; x < kXcc; ++x) {
                uint32_t* c = count + (int64_t)x * nseg + s;
                const uint32_t cv = *c;
                *c = run;
                run += cv;
            }
            if (queue) bk[r] = bucket_of(v);
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
        const int64_t s = base + r * kThreads + threadIdx.x;
        lists[(int64_t)bk[r] * nseg + lbase[bk[r]] + slot[r]] = (uint32_t)s;
    }
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

size_t scan_tmp_words(int64_t n) {
    const int64_t nb = (n + kPerBlock - 1) / kPerBlock;
    return (size_t)(4 * (nb + 1) + 64);  // U64x2 partials
}

hipError_t launch_emit_scan(const uint32_t* info, int64_t n, int tiles_x, int tiles_y, uint32_t* emit_off,
                            uint32_t* tmp, uint32_t* done, int64_t* counters, int64_t capacity, uint32_t* sample, int S,
                            uint32_t* zero, int64_t zero_words, hipStream_t s) {
    const int64_t nb = n > 0 ? (n + kPerBlock - 1) / kPerBlock : 1;
    U64x2* partials = reinterpret_cast<U64x2*>(tmp);
    hipLaunchKernelGGL(emit_reduce, dim3((unsigned)nb), dim3(kThreads), 0, s, reinterpret_cast<const uint4*>(info), n,
                       tiles_x, tiles_y, partials, done, counters, capacity, zero, zero_words);
    if (n > 0)
        hipLaunchKernelGGL(emit_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, reinterpret_cast<const uint4*>(info),
                           n, tiles_x, tiles_y, emit_off, partials, counters, sample, S);
    return hipGetLastError();
}

hipError_t launch_bin_offsets(uint32_t* count, int64_t nseg, uint32_t* bin_off, uint32_t* tmp, uint32_t* done,
                              uint32_t* lists, uint32_t* bucket_count, const int64_t* counters, hipStream_t s) {
    const int64_t nb = nseg > 0 ? (nseg + kPerBlock - 1) / kPerBlock : 1;
    hipLaunchKernelGGL(bo_reduce, dim3((unsigned)nb), dim3(kThreads), 0, s, count, nseg, tmp, done, bin_off + nseg);
    hipLaunchKernelGGL(bo_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, count, nseg, bin_off, tmp, lists,
                       bucket_count, counters);
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
