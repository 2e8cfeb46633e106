// Exclusive prefix sums: reduce -> scan of block sums -> apply, with
// wavefront shuffles inside a workgroup. Used for the per-Gaussian entry
// offsets (fused with the visible-Gaussian ranks and the depth-range
// sampling) and for the (tile, bin) counts -> bin offsets.
#include "common.hpp"

namespace tgs {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kPerBlock = kThreads * kItems;
constexpr int kTopThreads = 1024;

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

// ---- generic uint32 scan -------------------------------------------------

__global__ void __launch_bounds__(kThreads) u32_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                       uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t lds[kThreads / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kPerBlock + (int64_t)threadIdx.x * kItems;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (base + k < n) s += in[base + k];
    uint32_t total;
    (void)block_excl<uint32_t, kThreads>(s, lds, &total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Single workgroup: exclusive scan of the block sums in place; *total = sum.
__global__ void __launch_bounds__(kTopThreads) u32_top(uint32_t* __restrict__ block_sums, int64_t nb,
                                                       uint32_t* __restrict__ total_out) {
    __shared__ uint32_t lds[kTopThreads / kWave + 1];
    uint32_t carry = 0;
    for (int64_t base = 0; base < nb; base += kTopThreads) {
        const int64_t i = base + threadIdx.x;
        const uint32_t v = i < nb ? block_sums[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl<uint32_t, kTopThreads>(v, lds, &tot);
        if (i < nb) block_sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ void __launch_bounds__(kThreads) u32_apply(const uint32_t* in, uint32_t* out, int64_t n,
                                                      const uint32_t* __restrict__ block_off) {
    __shared__ uint32_t lds[kThreads / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kPerBlock + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint32_t run = block_off[blockIdx.x] + block_excl<uint32_t, kThreads>(s, lds, &total);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

// ---- entry-emission scan over the info array --------------------------------
// x: number of tiles (entries) per Gaussian, y: 1 if visible.

__device__ __forceinline__ U64x2 emit_val(const uint32_t* info, int64_t g, int64_t n, int tiles_x, int tiles_y) {
    U64x2 r;
    set_zero(r);
    if (g < n) {
        const uint4 in = reinterpret_cast<const uint4*>(info)[g];
        int x0, y0, x1, y1;
        const int nt = rect_of(in, tiles_x, tiles_y, x0, y0, x1, y1);
        r.x = (uint64_t)nt;
        r.y = nt > 0 ? 1ull : 0ull;
    }
    return r;
}

__global__ void __launch_bounds__(kThreads) emit_reduce(const uint32_t* __restrict__ info, int64_t n, int tiles_x,
                                                        int tiles_y, U64x2* __restrict__ block_sums) {
    __shared__ U64x2 lds[kThreads / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kPerBlock + (int64_t)threadIdx.x * kItems;
    U64x2 s;
    set_zero(s);
#pragma unroll
    for (int k = 0; k < kItems; ++k) s = s + emit_val(info, base + k, n, tiles_x, tiles_y);
    U64x2 total;
    (void)block_excl<U64x2, kThreads>(s, lds, &total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kTopThreads) emit_top(U64x2* __restrict__ block_sums, int64_t nb,
                                                        int64_t* __restrict__ counters, int64_t capacity) {
    __shared__ U64x2 lds[kTopThreads / kWave + 1];
    U64x2 carry;
    set_zero(carry);
    for (int64_t base = 0; base < nb; base += kTopThreads) {
        const int64_t i = base + threadIdx.x;
        U64x2 v;
        set_zero(v);
        if (i < nb) v = block_sums[i];
        U64x2 tot;
        const U64x2 ex = block_excl<U64x2, kTopThreads>(v, lds, &tot);
        if (i < nb) block_sums[i] = carry + ex;
        carry = carry + tot;
    }
    if (threadIdx.x == 0) {
        counters[0] = (int64_t)carry.x;
        counters[1] = (int64_t)carry.y;
        counters[2] = (int64_t)carry.x > capacity ? 1 : 0;
        counters[3] = 0;
    }
}

// Writes emit_off[g] and the depth-range samples. With V visible Gaussians
// and S samples: all visible depths when V <= S (sample[rank] = depth),
// otherwise the visible Gaussians at ranks floor(i V / S), i < S, each
// stored at its i. A rank r is such a rank iff i = ceil(r S / V) < S and
// floor(i V / S) == r.
__global__ void __launch_bounds__(kThreads) emit_apply(const uint32_t* __restrict__ info, int64_t n, int tiles_x,
                                                       int tiles_y, uint32_t* __restrict__ emit_off,
                                                       const U64x2* __restrict__ block_off,
                                                       const int64_t* __restrict__ counters,
                                                       uint32_t* __restrict__ sample, int S) {
    __shared__ U64x2 lds[kThreads / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kPerBlock + (int64_t)threadIdx.x * kItems;
    U64x2 v[kItems];
    U64x2 s;
    set_zero(s);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        v[k] = emit_val(info, base + k, n, tiles_x, tiles_y);
        s = s + v[k];
    }
    U64x2 total;
    U64x2 run = block_off[blockIdx.x] + block_excl<U64x2, kThreads>(s, lds, &total);
    const int64_t V = counters[1];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t g = base + k;
        if (g < n) {
            emit_off[g] = (uint32_t)run.x;
            if (v[k].y) {
                const int64_t r = (int64_t)run.y;
                int64_t i = -1;
                if (V <= S) {
                    i = r;
                } else {
                    const int64_t c = (r * S + V - 1) / V;
                    if (c < S && (c * V) / S == r) i = c;
                }
                if (i >= 0) sample[i] = info[4 * g];
            }
        }
        run = run + v[k];
    }
}

// ---- bin offsets from the per-XCD count copies ---------------------------

__global__ void __launch_bounds__(kThreads) bo_reduce(const uint32_t* __restrict__ count, int64_t nseg,
                                                      uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t lds[kThreads / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kPerBlock + (int64_t)threadIdx.x * kItems;
    uint32_t s = 0;
    for (int x = 0; x < kXcc; ++x) {
        const uint32_t* c = count + (int64_t)x * nseg;
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (base + k < nseg) s += c[base + k];
    }
    uint32_t total;
    (void)block_excl<uint32_t, kThreads>(s, lds, &total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// bin_off[s] = exclusive prefix of the summed copies; count[x][s] is then
// replaced by bin_off[s] + the counts of copies 0..x-1 in segment s.
__global__ void __launch_bounds__(kThreads) bo_apply(uint32_t* __restrict__ count, int64_t nseg,
                                                     uint32_t* __restrict__ bin_off,
                                                     const uint32_t* __restrict__ block_off) {
    __shared__ uint32_t lds[kThreads / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kPerBlock + (int64_t)threadIdx.x * kItems;
    uint32_t tot[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) tot[k] = 0;
    for (int x = 0; x < kXcc; ++x) {
        const uint32_t* c = count + (int64_t)x * nseg;
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (base + k < nseg) tot[k] += c[base + k];
    }
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) s += tot[k];
    uint32_t total;
    uint32_t run = block_off[blockIdx.x] + block_excl<uint32_t, kThreads>(s, lds, &total);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (base + k < nseg) {
            bin_off[base + k] = run;
            uint32_t r = run;
            for (int x = 0; x < kXcc; ++x) {
                uint32_t* c = count + (int64_t)x * nseg + base + k;
                const uint32_t v = *c;
                *c = r;
                r += v;
            }
        }
        run += tot[k];
    }
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

size_t scan_tmp_words(int64_t n) {
    const int64_t nb = (n + kPerBlock - 1) / kPerBlock;
    // room for U64x2 block sums (4 words each) plus alignment
    return (size_t)(4 * (nb + 1) + 16);
}

hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, uint32_t* total,
                           hipStream_t s) {
    if (n <= 0) return total ? launch_fill_u32(total, 0u, 1, s) : hipSuccess;
    const int64_t nb = (n + kPerBlock - 1) / kPerBlock;
    hipLaunchKernelGGL(u32_reduce, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, tmp);
    hipLaunchKernelGGL(u32_top, dim3(1), dim3(kTopThreads), 0, s, tmp, nb, total);
    hipLaunchKernelGGL(u32_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, in, out, n, tmp);
    return hipGetLastError();
}

hipError_t launch_emit_scan(const uint32_t* info, int64_t n, int tiles_x, int tiles_y, uint32_t* emit_off,
                            uint32_t* tmp, int64_t* counters, int64_t capacity, uint32_t* sample, int S,
                            hipStream_t s) {
    const int64_t nb = n > 0 ? (n + kPerBlock - 1) / kPerBlock : 0;
    U64x2* bs = reinterpret_cast<U64x2*>(tmp);
    if (nb > 0) hipLaunchKernelGGL(emit_reduce, dim3((unsigned)nb), dim3(kThreads), 0, s, info, n, tiles_x, tiles_y, bs);
    hipLaunchKernelGGL(emit_top, dim3(1), dim3(kTopThreads), 0, s, bs, nb, counters, capacity);
    if (nb > 0)
        hipLaunchKernelGGL(emit_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, info, n, tiles_x, tiles_y, emit_off,
                           bs, counters, sample, S);
    return hipGetLastError();
}

size_t bin_offsets_tmp_words(int64_t nseg) { return (size_t)((nseg + kPerBlock - 1) / kPerBlock + 16); }

hipError_t launch_bin_offsets(uint32_t* count, int64_t nseg, uint32_t* bin_off, uint32_t* tmp, hipStream_t s) {
    if (nseg <= 0) return launch_fill_u32(bin_off, 0u, 1, s);
    const int64_t nb = (nseg + kPerBlock - 1) / kPerBlock;
    hipLaunchKernelGGL(bo_reduce, dim3((unsigned)nb), dim3(kThreads), 0, s, count, nseg, tmp);
    hipLaunchKernelGGL(u32_top, dim3(1), dim3(kTopThreads), 0, s, tmp, nb, bin_off + nseg);
    hipLaunchKernelGGL(bo_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, count, nseg, bin_off, tmp);
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
