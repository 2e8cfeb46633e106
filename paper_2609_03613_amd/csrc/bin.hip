// Ordering stages.
//
// BINNED (the paper's tile-local path):
//   depth_range  robust [zmin, zmax] from exact order statistics of the
//                sampled depths (supplement, Algorithm "Robust depth-range
//                estimation"), one workgroup, LDS radix select;
//   bin_count    log-depth bin of each Gaussian and an atomic count per
//                (tile, bin); the returned old count is the entry's rank in
//                its segment (Algorithm "Tile-local bin construction");
//   bin_scatter  pair = depth bits << 32 | id written at bin offset + rank;
//   repair       every (tile, bin) segment with two or more entries is sorted
//                by its unique 64-bit pair, routed by length to a wavefront
//                register sort (<= 64), workgroup LDS sorts (<= 512, 2048,
//                8192) or a global-memory tail sort (section "Repair for
//                correctness": length buckets, local and broader exact
//                paths);
//   pack         per-entry records at their final stream positions.
// GLOBAL (the comparator): one (tile << 32 | depth bits, id) key-value pair
// per entry, a device radix sort, and per-tile ranges by binary search.
#include "common.hpp"

namespace tgs {

namespace {

// ---------------------------------------------------------------------------
// depth range
// ---------------------------------------------------------------------------

constexpr int kRangeThreads = 1024;
constexpr int kMaxSamples = 8192;

// Selects, for two ranks at once, the key with that 0-based rank among
// keys[0..n) (LDS) by four 8-bit radix passes.
__global__ void __launch_bounds__(kRangeThreads) depth_range_kernel(const uint32_t* __restrict__ sample,
                                                                   const int64_t* __restrict__ counters, int S,
                                                                   float p_lo, float p_hi, float pad, float znear,
                                                                   float zfar, float* __restrict__ zrange) {
#pragma clang fp contract(off)
    __shared__ uint32_t keys[kMaxSamples];
    __shared__ uint32_t hist[2][256];
    __shared__ uint32_t sel[2][3];  // prefix, mask, remaining rank
    const int64_t V = counters[1];
    const int n = (int)(V < S ? V : S);
    if (n == 0) {
        if (threadIdx.x == 0) {
            zrange[0] = znear;
            zrange[1] = zfar;
        }
        return;
    }
    for (int i = threadIdx.x; i < n; i += kRangeThreads) keys[i] = sample[i];
    if (threadIdx.x < 2) {
        int64_t k = threadIdx.x == 0 ? (int64_t)floor((double)p_lo / 100.0 * (double)(n - 1))
                                     : (int64_t)ceil((double)p_hi / 100.0 * (double)(n - 1));
        if (k < 0) k = 0;
        if (k > n - 1) k = n - 1;
        sel[threadIdx.x][0] = 0;
        sel[threadIdx.x][1] = 0;
        sel[threadIdx.x][2] = (uint32_t)k;
    }
    __syncthreads();
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int i = threadIdx.x; i < 512; i += kRangeThreads) hist[i >> 8][i & 255] = 0;
        __syncthreads();
        const uint32_t pre0 = sel[0][0], msk0 = sel[0][1], pre1 = sel[1][0], msk1 = sel[1][1];
        for (int i = threadIdx.x; i < n; i += kRangeThreads) {
            const uint32_t k = keys[i];
            const uint32_t d = (k >> shift) & 255u;
            if ((k & msk0) == pre0) atomicAdd(&hist[0][d], 1u);
            if ((k & msk1) == pre1) atomicAdd(&hist[1][d], 1u);
        }
        __syncthreads();
        // waves 0 and 1 each resolve one rank: lane l owns bins 4l..4l+3
        const int w = threadIdx.x / kWave;
        if (w < 2) {
            const int l = lane();
            const uint32_t h0 = hist[w][4 * l], h1 = hist[w][4 * l + 1], h2 = hist[w][4 * l + 2],
                           h3 = hist[w][4 * l + 3];
            const uint32_t own = h0 + h1 + h2 + h3;
            const uint32_t inc = wave_inclusive_sum(own);
            const uint32_t exc = inc - own;
            const uint32_t r = sel[w][2];
            const bool here = (exc <= r) && (r < inc);
            if (here) {
                uint32_t rr = r - exc;
                int d = 4 * l;
                if (rr >= h0) { rr -= h0; d++;
                    if (rr >= h1) { rr -= h1; d++;
                        if (rr >= h2) { rr -= h2; d++; } } }
                sel[w][0] |= (uint32_t)d << shift;
                sel[w][1] |= 255u << shift;
                sel[w][2] = rr;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float zlo = __uint_as_float(sel[0][0]);
        const float zhi = __uint_as_float(sel[1][0]);
        const float diff = zhi - zlo;
        const float span = diff > 1e-6f ? diff : 1e-6f;
        const float padv = pad * span;
        const float lo = zlo - padv;
        const float hi = zhi + padv;
        zrange[0] = lo > znear ? lo : znear;
        zrange[1] = hi < zfar ? hi : zfar;
    }
}

// Log-depth bin: the clamped log-space map floor(K u), realised with the
// IEEE-754 bit pattern of the binary32 depth as the logarithm (monotone,
// piecewise-linear log2), evaluated exactly in integers.
__device__ __forceinline__ int bin_of(uint32_t L, uint32_t Lmin, uint32_t Lmax, int K) {
    if (Lmax <= Lmin || L <= Lmin) return 0;
    if (L >= Lmax) return K - 1;
    const uint64_t b = ((uint64_t)K * (uint64_t)(L - Lmin)) / (uint64_t)(Lmax - Lmin);
    return b > (uint64_t)(K - 1) ? K - 1 : (int)b;
}

__global__ void __launch_bounds__(256) bin_count_kernel(const uint4* __restrict__ info, int64_t n,
                                                        const uint32_t* __restrict__ emit_off,
                                                        const float* __restrict__ zrange, int K, int tiles_x,
                                                        int tiles_y, uint32_t* __restrict__ count,
                                                        uint32_t* __restrict__ entry_rank, int64_t capacity) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const uint4 in = info[g];
    int x0, y0, x1, y1;
    if (rect_of(in, tiles_x, tiles_y, x0, y0, x1, y1) == 0) return;
    const int b = bin_of(in.x, __float_as_uint(zrange[0]), __float_as_uint(zrange[1]), K);
    int64_t e = emit_off[g];
    for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x, ++e) {
            const uint32_t r = atomicAdd(&count[(int64_t)(y * tiles_x + x) * K + b], 1u);
            if (e < capacity) entry_rank[e] = r;
        }
}

__global__ void __launch_bounds__(256) bin_scatter_kernel(const uint4* __restrict__ info, int64_t n,
                                                          const uint32_t* __restrict__ emit_off,
                                                          const float* __restrict__ zrange, int K, int tiles_x,
                                                          int tiles_y, const uint32_t* __restrict__ bin_off,
                                                          const uint32_t* __restrict__ entry_rank,
                                                          uint64_t* __restrict__ pairs, int64_t capacity) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const uint4 in = info[g];
    int x0, y0, x1, y1;
    if (rect_of(in, tiles_x, tiles_y, x0, y0, x1, y1) == 0) return;
    const int b = bin_of(in.x, __float_as_uint(zrange[0]), __float_as_uint(zrange[1]), K);
    const uint64_t pair = ((uint64_t)in.x << 32) | (uint64_t)g;
    int64_t e = emit_off[g];
    for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x, ++e) {
            if (e >= capacity) return;
            const int64_t p = (int64_t)bin_off[(int64_t)(y * tiles_x + x) * K + b] + entry_rank[e];
            if (p < capacity) pairs[p] = pair;
        }
}

// ---------------------------------------------------------------------------
// exact repair
// ---------------------------------------------------------------------------

// Length buckets: 2..64 (one wavefront), 65..512, 513..2048, 2049..8192
// (one workgroup, LDS), > 8192 (one workgroup, in place in global memory).
__device__ __forceinline__ int bucket_of(uint32_t len) {
    if (len <= 1) return -1;
    if (len <= 64) return 0;
    if (len <= 512) return 1;
    if (len <= 2048) return 2;
    if (len <= 8192) return 3;
    return 4;
}

// Nothing is queued when the stream overflowed its buffers (counters[2]).
__global__ void __launch_bounds__(256) classify_kernel(const uint32_t* __restrict__ bin_off, int64_t nseg,
                                                       uint32_t* __restrict__ lists,
                                                       uint32_t* __restrict__ bucket_count,
                                                       const int64_t* __restrict__ counters) {
    if (counters[2]) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int b = -1;
    if (s < nseg) b = bucket_of(bin_off[s + 1] - bin_off[s]);
#pragma unroll
    for (int k = 0; k < kBuckets; ++k) {
        const uint64_t m = ballot(b == k);
        if (m == 0) continue;
        uint32_t base = 0;
        const int leader = __builtin_ctzll(m);
        if (lane() == leader) base = atomicAdd(&bucket_count[k], (uint32_t)__builtin_popcountll(m));
        base = shfl_u32(base, leader);
        if (b == k) lists[(int64_t)k * nseg + base + rank_in(m)] = (uint32_t)s;
    }
}

// Segments of 2..64 entries: one wavefront per segment, bitonic network in
// registers, partners exchanged with lane shuffles.
__global__ void __launch_bounds__(256) sort_wave_kernel(const uint32_t* __restrict__ bin_off,
                                                        const uint32_t* __restrict__ list,
                                                        const uint32_t* __restrict__ bucket_count,
                                                        uint64_t* __restrict__ pairs) {
    const int waves = gridDim.x * (blockDim.x / kWave);
    const int wid = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const uint32_t cnt = bucket_count[0];
    const int l = lane();
    for (uint32_t i = wid; i < cnt; i += waves) {
        const uint32_t s = list[i];
        const uint32_t begin = bin_off[s], len = bin_off[s + 1] - begin;
        uint64_t v = l < (int)len ? pairs[begin + l] : ~0ull;
#pragma unroll
        for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                const uint64_t o = shfl_xor_u64(v, j);
                const bool up = (l & k) == 0;
                const bool lower = (l & j) == 0;
                const uint64_t mn = v < o ? v : o, mx = v < o ? o : v;
                v = (lower == up) ? mn : mx;
            }
        }
        if (l < (int)len) pairs[begin + l] = v;
    }
}

// Segments up to CAP entries: one workgroup per segment, bitonic network in
// LDS over the next power of two, padded with the maximum key.
template <int NT, int CAP>
__global__ void __launch_bounds__(NT) sort_lds_kernel(const uint32_t* __restrict__ bin_off,
                                                      const uint32_t* __restrict__ list,
                                                      const uint32_t* __restrict__ bucket_count, int bucket,
                                                      uint64_t* __restrict__ pairs) {
    __shared__ uint64_t buf[CAP];
    const uint32_t cnt = bucket_count[bucket];
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        const uint32_t s = list[i];
        const uint32_t begin = bin_off[s], len = bin_off[s + 1] - begin;
        uint32_t P = 1;
        while (P < len) P <<= 1;
        for (uint32_t e = threadIdx.x; e < P; e += NT) buf[e] = e < len ? pairs[begin + e] : ~0ull;
        __syncthreads();
        for (uint32_t k = 2; k <= P; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t e = threadIdx.x; e < P; e += NT) {
                    const uint32_t p = e ^ j;
                    if (p > e) {
                        const uint64_t a = buf[e], b = buf[p];
                        const bool up = (e & k) == 0;
                        if ((a > b) == up) {
                            buf[e] = b;
                            buf[p] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t e = threadIdx.x; e < len; e += NT) pairs[begin + e] = buf[e];
        __syncthreads();
    }
}

// Segments above 8192 entries: one workgroup sorts the segment in place in
// global memory. Bitonic network in the form whose every comparator puts
// the smaller key at the lower index (each merge starts by comparing
// mirrored positions), so positions at or beyond the segment length act as
// +infinity and are never touched.
__global__ void __launch_bounds__(1024) sort_tail_kernel(const uint32_t* __restrict__ bin_off,
                                                         const uint32_t* __restrict__ list,
                                                         const uint32_t* __restrict__ bucket_count,
                                                         uint64_t* pairs) {
    const uint32_t cnt = bucket_count[4];
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        const uint32_t s = list[i];
        const uint32_t begin = bin_off[s], len = bin_off[s + 1] - begin;
        uint64_t* a = pairs + begin;
        uint32_t P = 1;
        while (P < len) P <<= 1;
        for (uint32_t k = 2; k <= P; k <<= 1) {
            const uint32_t h = k >> 1;
            for (uint32_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
                const uint32_t blk = t / h, off = t % h;
                const uint32_t lo = blk * k + off, hi = blk * k + k - 1 - off;
                if (hi < len) {
                    const uint64_t x = a[lo], y = a[hi];
                    if (x > y) {
                        a[lo] = y;
                        a[hi] = x;
                    }
                }
            }
            __syncthreads();
            for (uint32_t j = k >> 2; j > 0; j >>= 1) {
                for (uint32_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
                    const uint32_t lo = (t / j) * 2 * j + (t % j), hi = lo + j;
                    if (hi < len) {
                        const uint64_t x = a[lo], y = a[hi];
                        if (x > y) {
                            a[lo] = y;
                            a[hi] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
}

// ---------------------------------------------------------------------------
// packed per-entry records
// ---------------------------------------------------------------------------

// One wavefront per tile: record p = splat of the entry's Gaussian with the
// mean relative to the tile origin, computed as (hi - origin) + lo.
__global__ void __launch_bounds__(256) pack_kernel(const uint64_t* __restrict__ pairs,
                                                   const uint32_t* __restrict__ bin_off, int K, int tiles_x,
                                                   int64_t T, const float4* __restrict__ splats,
                                                   float4* __restrict__ records,
                                                   const int64_t* __restrict__ counters, int64_t capacity) {
#pragma clang fp contract(off)
    if (counters[2]) return;
    const int waves = gridDim.x * (blockDim.x / kWave);
    const int wid = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int l = lane();
    for (int64_t t = wid; t < T; t += waves) {
        const uint32_t begin = bin_off[t * K], end = bin_off[t * K + K];
        const float ox = (float)((t % tiles_x) * kTile), oy = (float)((t / tiles_x) * kTile);
        for (uint32_t p = begin + l; p < end; p += kWave) {
            const uint32_t gid = (uint32_t)pairs[p];
            const float4 a = splats[3 * (int64_t)gid], b = splats[3 * (int64_t)gid + 1],
                         c = splats[3 * (int64_t)gid + 2];
            float4* r = records + 3 * (int64_t)p;
            r[0] = make_float4((a.x - ox) + a.z, (a.y - oy) + a.w, b.x, b.y);
            r[1] = make_float4(b.z, b.w, c.x, c.y);
            r[2] = make_float4(c.z, __uint_as_float(gid), 0.f, 0.f);
        }
    }
}

// ---------------------------------------------------------------------------
// global-sort comparator
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) emit_keys_kernel(const uint4* __restrict__ info, int64_t n,
                                                        const uint32_t* __restrict__ emit_off, int tiles_x,
                                                        int tiles_y, uint64_t* __restrict__ keys,
                                                        uint32_t* __restrict__ vals, int64_t capacity) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const uint4 in = info[g];
    int x0, y0, x1, y1;
    if (rect_of(in, tiles_x, tiles_y, x0, y0, x1, y1) == 0) return;
    int64_t e = emit_off[g];
    for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x, ++e) {
            if (e >= capacity) return;
            keys[e] = ((uint64_t)(y * tiles_x + x) << 32) | in.x;
            vals[e] = (uint32_t)g;
        }
}

// tile_off[t] = first position whose tile is >= t (t = 0..T).
__global__ void __launch_bounds__(256) tile_ranges_kernel(const uint64_t* __restrict__ keys, int64_t m, int64_t T,
                                                          uint32_t* __restrict__ tile_off) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > T) return;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)(keys[mid] >> 32) < t)
            lo = mid + 1;
        else
            hi = mid;
    }
    tile_off[t] = (uint32_t)lo;
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hipError_t launch_depth_range(const uint32_t* sample, const int64_t* counters, int S, float p_lo, float p_hi,
                              float pad, float znear, float zfar, float* zrange, hipStream_t s) {
    hipLaunchKernelGGL(depth_range_kernel, dim3(1), dim3(kRangeThreads), 0, s, sample, counters, S, p_lo, p_hi, pad,
                       znear, zfar, zrange);
    return hipGetLastError();
}

hipError_t launch_bin_count(const uint32_t* info, int64_t n, const uint32_t* emit_off, const float* zrange, int K,
                            int tiles_x, int tiles_y, uint32_t* count, uint32_t* entry_rank, int64_t capacity,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(bin_count_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       reinterpret_cast<const uint4*>(info), n, emit_off, zrange, K, tiles_x, tiles_y, count,
                       entry_rank, capacity);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(const uint32_t* info, int64_t n, const uint32_t* emit_off, const float* zrange, int K,
                              int tiles_x, int tiles_y, const uint32_t* bin_off, const uint32_t* entry_rank,
                              uint64_t* pairs, int64_t capacity, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(bin_scatter_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       reinterpret_cast<const uint4*>(info), n, emit_off, zrange, K, tiles_x, tiles_y, bin_off,
                       entry_rank, pairs, capacity);
    return hipGetLastError();
}

hipError_t launch_repair(const uint32_t* bin_off, int64_t nseg, uint64_t* pairs, uint32_t* seg_lists,
                         uint32_t* bucket_count, const int64_t* counters, hipStream_t s) {
    if (nseg == 0) return hipSuccess;
    hipError_t e = launch_fill_u32(bucket_count, 0u, kBuckets, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(classify_kernel, dim3(grid_for(nseg, 256)), dim3(256), 0, s, bin_off, nseg, seg_lists,
                       bucket_count, counters);
    hipLaunchKernelGGL(sort_wave_kernel, dim3(2048), dim3(256), 0, s, bin_off, seg_lists, bucket_count, pairs);
    hipLaunchKernelGGL((sort_lds_kernel<256, 512>), dim3(1024), dim3(256), 0, s, bin_off, seg_lists + nseg,
                       bucket_count, 1, pairs);
    hipLaunchKernelGGL((sort_lds_kernel<1024, 2048>), dim3(512), dim3(1024), 0, s, bin_off, seg_lists + 2 * nseg,
                       bucket_count, 2, pairs);
    hipLaunchKernelGGL((sort_lds_kernel<1024, 8192>), dim3(256), dim3(1024), 0, s, bin_off, seg_lists + 3 * nseg,
                       bucket_count, 3, pairs);
    hipLaunchKernelGGL(sort_tail_kernel, dim3(64), dim3(1024), 0, s, bin_off, seg_lists + 4 * nseg, bucket_count,
                       pairs);
    return hipGetLastError();
}

hipError_t launch_pack(const uint64_t* pairs, const uint32_t* bin_off, int K, int tiles_x, int64_t T,
                       const float* splats, float* records, const int64_t* counters, int64_t capacity,
                       hipStream_t s) {
    if (T == 0) return hipSuccess;
    int64_t blocks = (T + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)blocks), dim3(256), 0, s, pairs, bin_off, K, tiles_x, T,
                       reinterpret_cast<const float4*>(splats), reinterpret_cast<float4*>(records), counters,
                       capacity);
    return hipGetLastError();
}

hipError_t launch_emit_keys(const uint32_t* info, int64_t n, const uint32_t* emit_off, int tiles_x, int tiles_y,
                            uint64_t* keys, uint32_t* vals, int64_t capacity, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(emit_keys_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       reinterpret_cast<const uint4*>(info), n, emit_off, tiles_x, tiles_y, keys, vals, capacity);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint64_t* keys, int64_t m, int64_t T, uint32_t* tile_off, hipStream_t s) {
    hipLaunchKernelGGL(tile_ranges_kernel, dim3(grid_for(T + 1, 256)), dim3(256), 0, s, keys, m, T, tile_off);
    return hipGetLastError();
}

}  // namespace tgs
