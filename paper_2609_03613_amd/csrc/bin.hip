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
//   records      packed per-entry records written where each entry becomes
//                final (the scatter for one-entry segments, the repair
//                sorts for the others).
// GLOBAL (the comparator): one (tile << 32 | depth bits, id) key-value pair
// per entry, a device radix sort, and per-tile ranges by binary search.
#include <algorithm>

#include "common.hpp"

namespace tgs {

namespace {

// ---------------------------------------------------------------------------
// depth range
// ---------------------------------------------------------------------------

constexpr int kRangeThreads = 1024;
constexpr int kMaxSamples = 8192;
constexpr int kDigit = 11;
constexpr int kBinsR = 1 << kDigit;

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v = min(v, shfl_xor_u32(v, m));
    return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v = max(v, shfl_xor_u32(v, m));
    return v;
}

// Exact order statistics of the sampled depths (binary32 bits; depths are
// positive so the bit order is the value order). Both ranks are selected
// together by radix passes of 11 bits over key - min(key), which spreads the
// histogram even when all depths share their top bits.
__global__ void __launch_bounds__(kRangeThreads) depth_range_kernel(const uint32_t* __restrict__ sample,
                                                                   const int64_t* __restrict__ counters, int S,
                                                                   float p_lo, float p_hi, float pad, float znear,
                                                                   float zfar, float* __restrict__ zrange) {
#pragma clang fp contract(off)
    __shared__ uint32_t keys[kMaxSamples];
    __shared__ uint32_t hist[2][kBinsR];
    __shared__ uint32_t sel[2][3];  // prefix (relative), mask, remaining rank
    __shared__ uint32_t red[2][kRangeThreads / kWave];
    const int64_t V = counters[1];
    const int n = (int)(V < S ? V : S);
    if (n == 0) {
        if (threadIdx.x == 0) {
            zrange[0] = znear;
            zrange[1] = zfar;
        }
        return;
    }
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (int i = threadIdx.x; i < n; i += kRangeThreads) {
        const uint32_t k = sample[i];
        keys[i] = k;
        lo = min(lo, k);
        hi = max(hi, k);
    }
    lo = wave_min_u32(lo);
    hi = wave_max_u32(hi);
    const int w = threadIdx.x / kWave;
    if (lane() == 0) {
        red[0][w] = lo;
        red[1][w] = hi;
    }
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
    uint32_t kmin = red[0][0], kmax = red[1][0];
    for (int i = 1; i < kRangeThreads / kWave; ++i) {
        kmin = min(kmin, red[0][i]);
        kmax = max(kmax, red[1][i]);
    }
    const uint32_t span_bits = kmax - kmin;
    const int L = span_bits == 0 ? 0 : 32 - __builtin_clz(span_bits);
    for (int top = L; top > 0; top -= kDigit) {
        const int shift = top > kDigit ? top - kDigit : 0;
        for (int i = threadIdx.x; i < 2 * kBinsR; i += kRangeThreads) hist[i / kBinsR][i % kBinsR] = 0;
        __syncthreads();
        const uint32_t pre0 = sel[0][0], msk0 = sel[0][1], pre1 = sel[1][0], msk1 = sel[1][1];
        for (int i = threadIdx.x; i < n; i += kRangeThreads) {
            const uint32_t k = keys[i] - kmin;
            const uint32_t d = (k >> shift) & (kBinsR - 1);
            if ((k & msk0) == pre0) atomicAdd(&hist[0][d], 1u);
            if ((k & msk1) == pre1) atomicAdd(&hist[1][d], 1u);
        }
        __syncthreads();
        // waves 0 and 1 each resolve one rank: lane l owns 32 consecutive bins
        if (w < 2) {
            const int l = lane();
            constexpr int per = kBinsR / kWave;
            uint32_t own = 0;
            for (int j = 0; j < per; ++j) own += hist[w][l * per + j];
            const uint32_t inc = wave_inclusive_sum(own);
            const uint32_t exc = inc - own;
            const uint32_t r = sel[w][2];
            if (exc <= r && r < inc) {
                uint32_t rr = r - exc;
                int d = l * per;
                while (rr >= hist[w][d]) {
                    rr -= hist[w][d];
                    ++d;
                }
                sel[w][0] |= (uint32_t)d << shift;
                sel[w][1] |= (uint32_t)(kBinsR - 1) << shift;
                sel[w][2] = rr;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float zlo = __uint_as_float(sel[0][0] + kmin);
        const float zhi = __uint_as_float(sel[1][0] + kmin);
        const float diff = zhi - zlo;
        const float span = diff > 1e-6f ? diff : 1e-6f;
        const float padv = pad * span;
        const float a = zlo - padv;
        const float b = zhi + padv;
        zrange[0] = a > znear ? a : znear;
        zrange[1] = b < zfar ? b : zfar;
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

// Atomic count per (tile, bin) into the calling XCD's copy of the counts.
// All atomics on copy x come from XCD x, so they are carried out in that
// XCD's L2 (workgroup scope) instead of at the memory side; the returned old
// value is the entry's rank inside its copy.
__global__ void __launch_bounds__(256) bin_count_kernel(const uint4* __restrict__ info, int64_t n,
                                                        const uint32_t* __restrict__ emit_off,
                                                        const float* __restrict__ zrange, int K, int tiles_x,
                                                        int tiles_y, uint32_t* __restrict__ count, int64_t nseg,
                                                        uint32_t* __restrict__ entry_rank, int64_t capacity) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const uint4 in = info[g];
    int x0, y0, x1, y1;
    if (rect_of(in, tiles_x, tiles_y, x0, y0, x1, y1) == 0) return;
    const int b = bin_of(in.x, __float_as_uint(zrange[0]), __float_as_uint(zrange[1]), K);
    const uint32_t x = (uint32_t)xcc_id();
    uint32_t* cnt = count + (int64_t)x * nseg;
    int64_t e = emit_off[g];
    for (int y = y0; y < y1; ++y)
        for (int xx = x0; xx < x1; ++xx, ++e) {
            const uint32_t r = __hip_atomic_fetch_add(&cnt[(int64_t)(y * tiles_x + xx) * K + b], 1u,
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (e < capacity) entry_rank[e] = (r & 0x1FFFFFFFu) | (x << 29);
        }
}

// pair = depth bits << 32 | id at base[copy][segment] + rank. An entry that
// is alone in its segment is final here, so its packed record is written
// too; longer segments get theirs from the repair sorts.
__global__ void __launch_bounds__(256) bin_scatter_kernel(const uint4* __restrict__ info, int64_t n,
                                                          const uint32_t* __restrict__ emit_off,
                                                          const float* __restrict__ zrange, int K, int tiles_x,
                                                          int tiles_y, const uint32_t* __restrict__ bin_off,
                                                          const uint32_t* __restrict__ base, int64_t nseg,
                                                          const uint32_t* __restrict__ entry_rank,
                                                          uint64_t* __restrict__ pairs, int64_t capacity,
                                                          RecordSink rs) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const uint4 in = info[g];
    int x0, y0, x1, y1;
    if (rect_of(in, tiles_x, tiles_y, x0, y0, x1, y1) == 0) return;
    const int b = bin_of(in.x, __float_as_uint(zrange[0]), __float_as_uint(zrange[1]), K);
    const uint64_t pair = ((uint64_t)in.x << 32) | (uint64_t)g;
    int64_t e = emit_off[g];
    for (int y = y0; y < y1; ++y)
        for (int xx = x0; xx < x1; ++xx, ++e) {
            if (e >= capacity) return;
            const uint32_t rk = entry_rank[e];
            const int64_t sg = (int64_t)(y * tiles_x + xx) * K + b;
            const int64_t p = (int64_t)base[(int64_t)(rk >> 29) * nseg + sg] + (rk & 0x1FFFFFFFu);
            if (p >= capacity) continue;
            pairs[p] = pair;
            if (rs.records && bin_off[sg + 1] - bin_off[sg] == 1) rs.put((uint32_t)sg, (uint32_t)p, pair);
        }
}

// ---------------------------------------------------------------------------
// exact repair
// ---------------------------------------------------------------------------

// Length buckets: 2..64, 65..128, 129..256, 257..512 (one wavefront, 1, 2,
// 4 or 8 keys per lane in registers), 513..4096, 4097..8192 (one workgroup,
// LDS), > 8192 (one workgroup, in place in global memory).
__device__ __forceinline__ int bucket_of(uint32_t len) {
    if (len <= 1) return -1;
    if (len <= 64) return 0;
    if (len <= 128) return 1;
    if (len <= 256) return 2;
    if (len <= 512) return 3;
    if (len <= 4096) return 4;
    if (len <= 8192) return 5;
    return 6;
}

constexpr int kClassifyItems = 8;

// Appends every segment of two or more entries to its bucket list. Counts
// are aggregated per wavefront (ballot) and per workgroup (LDS) so that each
// workgroup issues one global atomic per bucket. Nothing is queued when the
// stream overflowed its buffers (counters[2]).
__global__ void __launch_bounds__(256) classify_kernel(const uint32_t* __restrict__ bin_off, int64_t nseg,
                                                       uint32_t* __restrict__ lists,
                                                       uint32_t* __restrict__ bucket_count,
                                                       const int64_t* __restrict__ counters) {
    __shared__ uint32_t lcount[kBuckets], lbase[kBuckets];
    if (counters[2]) return;
    if (threadIdx.x < kBuckets) lcount[threadIdx.x] = 0;
    __syncthreads();
    const int64_t first = (int64_t)blockIdx.x * 256 * kClassifyItems;
    int bk[kClassifyItems];
    uint32_t slot[kClassifyItems];
#pragma unroll
    for (int i = 0; i < kClassifyItems; ++i) {
        const int64_t s = first + (int64_t)i * 256 + threadIdx.x;
        bk[i] = s < nseg ? bucket_of(bin_off[s + 1] - bin_off[s]) : -1;
        slot[i] = 0;
        if (ballot(bk[i] >= 0) == 0) continue;
#pragma unroll
        for (int k = 0; k < kBuckets; ++k) {
            const uint64_t m = ballot(bk[i] == k);
            if (m == 0) continue;
            const int leader = __builtin_ctzll(m);
            uint32_t b0 = 0;
            if (lane() == leader) b0 = atomicAdd(&lcount[k], (uint32_t)__builtin_popcountll(m));
            b0 = shfl_u32(b0, leader);
            if (bk[i] == k) slot[i] = b0 + rank_in(m);
        }
    }
    __syncthreads();
    if (threadIdx.x < kBuckets)
        lbase[threadIdx.x] = lcount[threadIdx.x] ? atomicAdd(&bucket_count[threadIdx.x], lcount[threadIdx.x]) : 0u;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kClassifyItems; ++i) {
        if (bk[i] < 0) continue;
        const int64_t s = first + (int64_t)i * 256 + threadIdx.x;
        lists[(int64_t)bk[i] * nseg + lbase[bk[i]] + slot[i]] = (uint32_t)s;
    }
}

// One wavefront per segment of at most 64 E keys; lane l holds keys
// l E .. l E + E - 1 in registers. Bitonic network: partners at distance
// j >= E are in lane l ^ (j / E) (lane shuffle), closer ones in the same lane.
template <int E>
__global__ void __launch_bounds__(256) sort_wave_kernel(const uint32_t* __restrict__ bin_off,
                                                        const uint32_t* __restrict__ list,
                                                        const uint32_t* __restrict__ bucket_count, int bucket,
                                                        uint64_t* __restrict__ pairs, RecordSink rs) {
    constexpr int N = kWave * E;
    const int waves = gridDim.x * (blockDim.x / kWave);
    const int wid = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const uint32_t cnt = bucket_count[bucket];
    const int l = lane();
    for (uint32_t i = wid; i < cnt; i += waves) {
        const uint32_t s = list[i];
        const uint32_t begin = bin_off[s], len = bin_off[s + 1] - begin;
        uint64_t v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t idx = (uint32_t)(l * E + e);
            v[e] = idx < len ? pairs[begin + idx] : ~0ull;
        }
#pragma unroll
        for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                if (j >= E) {
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int idx = l * E + e;
                        const uint64_t o = shfl_xor_u64(v[e], j / E);
                        const bool up = (idx & k) == 0, lower = (idx & j) == 0;
                        const uint64_t mn = v[e] < o ? v[e] : o, mx = v[e] < o ? o : v[e];
                        v[e] = (lower == up) ? mn : mx;
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        if (e & j) continue;
                        const int idx = l * E + e;
                        const bool up = (idx & k) == 0;
                        const uint64_t a = v[e], b = v[e ^ j];
                        if ((a > b) == up) {
                            v[e] = b;
                            v[e ^ j] = a;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t idx = (uint32_t)(l * E + e);
            if (idx < len) {
                pairs[begin + idx] = v[e];
                rs.put(s, begin + idx, v[e]);
            }
        }
    }
}

// Segments up to CAP keys: one workgroup per segment, bitonic network in
// LDS over the next power of two, padded with the maximum key.
template <int NT, int CAP>
__global__ void __launch_bounds__(NT) sort_lds_kernel(const uint32_t* __restrict__ bin_off,
                                                      const uint32_t* __restrict__ list,
                                                      const uint32_t* __restrict__ bucket_count, int bucket,
                                                      uint64_t* __restrict__ pairs, RecordSink rs) {
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
        for (uint32_t e = threadIdx.x; e < len; e += NT) {
            pairs[begin + e] = buf[e];
            rs.put(s, begin + e, buf[e]);
        }
        __syncthreads();
    }
}

// Segments above 8192 keys: one workgroup sorts the segment in place in
// global memory. Bitonic network in the form whose every comparator puts
// the smaller key at the lower index (each merge starts by comparing
// mirrored positions), so positions at or beyond the segment length act as
// +infinity and are never touched.
__global__ void __launch_bounds__(1024) sort_tail_kernel(const uint32_t* __restrict__ bin_off,
                                                         const uint32_t* __restrict__ list,
                                                         const uint32_t* __restrict__ bucket_count, int bucket,
                                                         uint64_t* pairs, RecordSink rs) {
    const uint32_t cnt = bucket_count[bucket];
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
        for (uint32_t e = threadIdx.x; e < len; e += blockDim.x) rs.put(s, begin + e, a[e]);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// heaviest-first tile order
// ---------------------------------------------------------------------------

constexpr int kOrderBuckets = 33;

__global__ void __launch_bounds__(1024) tile_order_kernel(const uint32_t* __restrict__ offsets, int stride,
                                                          int64_t T, uint32_t* __restrict__ order) {
    __shared__ uint32_t hist[kOrderBuckets], cur[kOrderBuckets];
    if (threadIdx.x < kOrderBuckets) hist[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < T; t += blockDim.x) {
        const uint32_t c = offsets[(t + 1) * stride] - offsets[t * stride];
        const int b = 32 - (c ? 32 - __builtin_clz(c) : 0);
        atomicAdd(&hist[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int b = 0; b < kOrderBuckets; ++b) {
            cur[b] = acc;
            acc += hist[b];
        }
    }
    __syncthreads();
    for (int64_t t = threadIdx.x; t < T; t += blockDim.x) {
        const uint32_t c = offsets[(t + 1) * stride] - offsets[t * stride];
        const int b = 32 - (c ? 32 - __builtin_clz(c) : 0);
        order[atomicAdd(&cur[b], 1u)] = (uint32_t)t;
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
                            int tiles_x, int tiles_y, uint32_t* count, int64_t nseg, uint32_t* entry_rank,
                            int64_t capacity, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(bin_count_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       reinterpret_cast<const uint4*>(info), n, emit_off, zrange, K, tiles_x, tiles_y, count, nseg,
                       entry_rank, capacity);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(const uint32_t* info, int64_t n, const uint32_t* emit_off, const float* zrange, int K,
                              int tiles_x, int tiles_y, const uint32_t* bin_off, const uint32_t* base, int64_t nseg,
                              const uint32_t* entry_rank, uint64_t* pairs, int64_t capacity, RecordSink rs,
                              hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(bin_scatter_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       reinterpret_cast<const uint4*>(info), n, emit_off, zrange, K, tiles_x, tiles_y, bin_off, base,
                       nseg, entry_rank, pairs, capacity, rs);
    return hipGetLastError();
}

hipError_t launch_repair(const uint32_t* bin_off, int64_t nseg, uint64_t* pairs, uint32_t* seg_lists,
                         uint32_t* bucket_count, const int64_t* counters, RecordSink rs, hipStream_t s) {
    if (nseg == 0) return hipSuccess;
    hipError_t e = launch_fill_u32(bucket_count, 0u, kBuckets, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(classify_kernel, dim3(grid_for(nseg, 256 * kClassifyItems)), dim3(256), 0, s, bin_off, nseg,
                       seg_lists, bucket_count, counters);
    const unsigned wave_blocks = (unsigned)std::min<int64_t>(std::max<int64_t>((nseg + 3) / 4, 1), 8192);
    hipLaunchKernelGGL((sort_wave_kernel<1>), dim3(wave_blocks), dim3(256), 0, s, bin_off, seg_lists, bucket_count, 0,
                       pairs, rs);
    hipLaunchKernelGGL((sort_wave_kernel<2>), dim3(std::min(wave_blocks, 4096u)), dim3(256), 0, s, bin_off,
                       seg_lists + nseg, bucket_count, 1, pairs, rs);
    hipLaunchKernelGGL((sort_wave_kernel<4>), dim3(std::min(wave_blocks, 2048u)), dim3(256), 0, s, bin_off,
                       seg_lists + 2 * nseg, bucket_count, 2, pairs, rs);
    hipLaunchKernelGGL((sort_wave_kernel<8>), dim3(std::min(wave_blocks, 2048u)), dim3(256), 0, s, bin_off,
                       seg_lists + 3 * nseg, bucket_count, 3, pairs, rs);
    hipLaunchKernelGGL((sort_lds_kernel<1024, 4096>), dim3(512), dim3(1024), 0, s, bin_off, seg_lists + 4 * nseg,
                       bucket_count, 4, pairs, rs);
    hipLaunchKernelGGL((sort_lds_kernel<1024, 8192>), dim3(256), dim3(1024), 0, s, bin_off, seg_lists + 5 * nseg,
                       bucket_count, 5, pairs, rs);
    hipLaunchKernelGGL(sort_tail_kernel, dim3(64), dim3(1024), 0, s, bin_off, seg_lists + 6 * nseg, bucket_count, 6,
                       pairs, rs);
    return hipGetLastError();
}

hipError_t launch_tile_order(const uint32_t* offsets, int stride, int64_t T, uint32_t* order, hipStream_t s) {
    if (T == 0) return hipSuccess;
    hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(1024), 0, s, offsets, stride, T, order);
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
