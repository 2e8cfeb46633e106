// Ordering stages.
//
// BINNED (the paper's tile-local path):
//   depth_range  robust [zmin, zmax] from exact order statistics of the
//                sampled depths (supplement, Algorithm "Robust depth-range
//                estimation"): the samples are gathered by many workgroups,
//                the LDS radix select runs in one workgroup (beside the
//                group count when binning is grouped);
//   grouped      the count / scan / scatter of Algorithm "Tile-local bin
//                construction" in two levels: entries are counted and
//                scattered per group of consecutive tiles with LDS counters
//                and one global atomic per (workgroup, group), then each
//                group is counting-sorted by (tile, bin[, sub-bin]) in LDS;
//                per-entry global atomics on scattered counters run at
//                ~25 G/s on this GPU and would dominate the stage;
//   bin_count    (group shapes beyond the LDS counters) log-depth bin of each
//                Gaussian and an atomic count per (tile, bin) in the XCD's
//                copy; the returned old count is the entry's rank;
//   bin_scatter  pair = depth bits << 32 | id written at bin offset + rank;
//   repair       every (tile, bin) segment with two or more entries is sorted
//                by its unique 64-bit pair (with sub-bins: every sub-segment),
//                routed by length to wavefront register sorts (<= 64 in lane
//                groups, <= 512 with 2-8 keys per lane), workgroup LDS sorts
//                (<= 8192) or a global-memory tail sort (section "Repair for
//                correctness": length buckets, local and broader exact
//                paths);
//   records      packed per-entry records written where each entry becomes
//                final (the group sort or scatter for one-entry segments,
//                the repair sorts for the others).
// GLOBAL (the comparator): one (tile << 32 | depth bits, id) key-value pair
// per entry, a device radix sort, and per-tile ranges by binary search.
#include <algorithm>

#include "common.hpp"
#include "wave_sort.hpp"

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

// LDS of one depth-range workgroup.
struct RangeLds {
    uint32_t keys[kMaxSamples];
    uint32_t hist[2][kBinsR];
    uint32_t sel[2][3];  // prefix (relative), mask, remaining rank
    uint32_t red[2][kRangeThreads / kWave];
};

// Exact order statistics of the sampled binning keys (binary32 bits of the
// depth or of the near-depth key; both are positive, so the bit order is the
// value order). Both ranks are selected together by radix passes of 11 bits
// over key - min(key), which spreads the histogram even when all depths
// share their top bits; while both ranks share their prefix (always in the
// first pass) one histogram serves both. Run by one workgroup of
// kRangeThreads threads.
// Binning key of depth sample i < n = min(V, S): the visible Gaussian at
// rank floor(i V / S) (rank i when V <= S).
__device__ __forceinline__ uint32_t sample_key(const uint4* __restrict__ info, const uint32_t* __restrict__ vis_ids,
                                               const NearKey& nk, int64_t V, int S, int i) {
    const int64_t r = V <= S ? (int64_t)i : ((int64_t)i * V) / S;
    const uint32_t g = vis_ids[r];
    const uint32_t key = info[g].x;
    return nk.splats ? nk(key, g) : key;
}

// The sample keys gathered by many workgroups into samples[0 .. n): the
// random reads of one workgroup alone would take longer than the selection.
__global__ void __launch_bounds__(256) range_samples_kernel(const uint4* __restrict__ info,
                                                            const uint32_t* __restrict__ vis_ids,
                                                            const int64_t* __restrict__ counters, NearKey nk, int S,
                                                            uint32_t* __restrict__ samples) {
#pragma clang fp contract(off)
    const int64_t V = counters[1];
    const int n = (int)(V < S ? V : S);
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) samples[i] = sample_key(info, vis_ids, nk, V, S, i);
}

// samples: the keys from range_samples_kernel, or null to gather them here.
__device__ __forceinline__ void depth_range_block(const uint4* __restrict__ info, const uint32_t* __restrict__ vis_ids,
                                                  const int64_t* __restrict__ counters, const NearKey& nk, int S,
                                                  float p_lo, float p_hi, float pad, float znear, float zfar,
                                                  float* __restrict__ zrange, const uint32_t* __restrict__ samples,
                                                  RangeLds& R) {
#pragma clang fp contract(off)
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
    constexpr int kPer = kMaxSamples / kRangeThreads;
    uint32_t key[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = j * kRangeThreads + threadIdx.x;
        key[j] = i >= n ? 0u : samples ? samples[i] : sample_key(info, vis_ids, nk, V, S, i);
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = j * kRangeThreads + threadIdx.x;
        if (i < n) {
            R.keys[i] = key[j];
            lo = min(lo, key[j]);
            hi = max(hi, key[j]);
        }
    }
    lo = wave_min_u32(lo);
    hi = wave_max_u32(hi);
    const int w = threadIdx.x / kWave;
    if (lane() == 0) {
        R.red[0][w] = lo;
        R.red[1][w] = hi;
    }
    if (threadIdx.x < 2) {
        int64_t k = threadIdx.x == 0 ? (int64_t)floor((double)p_lo / 100.0 * (double)(n - 1))
                                     : (int64_t)ceil((double)p_hi / 100.0 * (double)(n - 1));
        if (k < 0) k = 0;
        if (k > n - 1) k = n - 1;
        R.sel[threadIdx.x][0] = 0;
        R.sel[threadIdx.x][1] = 0;
        R.sel[threadIdx.x][2] = (uint32_t)k;
    }
    __syncthreads();
    uint32_t kmin = R.red[0][0], kmax = R.red[1][0];
    for (int i = 1; i < kRangeThreads / kWave; ++i) {
        kmin = min(kmin, R.red[0][i]);
        kmax = max(kmax, R.red[1][i]);
    }
    const uint32_t span_bits = kmax - kmin;
    const int L = span_bits == 0 ? 0 : 32 - __builtin_clz(span_bits);
    for (int top = L; top > 0; top -= kDigit) {
        const int shift = top > kDigit ? top - kDigit : 0;
        const uint32_t pre0 = R.sel[0][0], msk0 = R.sel[0][1], pre1 = R.sel[1][0], msk1 = R.sel[1][1];
        const bool same = pre0 == pre1 && msk0 == msk1;
        for (int i = threadIdx.x; i < (same ? 1 : 2) * kBinsR; i += kRangeThreads) R.hist[i / kBinsR][i % kBinsR] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += kRangeThreads) {
            const uint32_t k = R.keys[i] - kmin;
            const uint32_t d = (k >> shift) & (kBinsR - 1);
            if ((k & msk0) == pre0) atomicAdd(&R.hist[0][d], 1u);
            if (!same && (k & msk1) == pre1) atomicAdd(&R.hist[1][d], 1u);
        }
        __syncthreads();
        // both ranks are resolved by one workgroup scan over the bins:
        // thread t owns bins 2t and 2t + 1 of each rank's histogram
        static_assert(kBinsR == 2 * kRangeThreads, "two bins per thread");
        const uint32_t* h0 = R.hist[0];
        const uint32_t* h1 = R.hist[same ? 0 : 1];
        const int t2 = 2 * (int)threadIdx.x;
        const uint32_t a0 = h0[t2], a1 = h0[t2 + 1], b0 = h1[t2], b1 = h1[t2 + 1];
        const uint32_t r0 = R.sel[0][2], r1 = R.sel[1][2];
        const uint32_t ia = wave_inclusive_sum(a0 + a1), ib = wave_inclusive_sum(b0 + b1);
        if (lane() == kWave - 1) {
            R.red[0][w] = ia;
            R.red[1][w] = ib;
        }
        __syncthreads();
        uint32_t ea = ia - (a0 + a1), eb = ib - (b0 + b1);
        for (int i = 0; i < w; ++i) {
            ea += R.red[0][i];
            eb += R.red[1][i];
        }
        auto resolve = [&](int q, uint32_t e, uint32_t c0, uint32_t c1, uint32_t r) {
            if (r < e || r >= e + c0 + c1) return;
            const bool first = r < e + c0;
            R.sel[q][0] |= (uint32_t)(first ? t2 : t2 + 1) << shift;
            R.sel[q][1] |= (uint32_t)(kBinsR - 1) << shift;
            R.sel[q][2] = first ? r - e : r - e - c0;
        };
        resolve(0, ea, a0, a1, r0);
        resolve(1, eb, b0, b1, r1);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float zlo = __uint_as_float(R.sel[0][0] + kmin);
        const float zhi = __uint_as_float(R.sel[1][0] + kmin);
        const float diff = zhi - zlo;
        const float span = diff > 1e-6f ? diff : 1e-6f;
        const float padv = pad * span;
        const float a = zlo - padv;
        const float b = zhi + padv;
        zrange[0] = a > znear ? a : znear;
        zrange[1] = b < zfar ? b : zfar;
    }
}

__global__ void __launch_bounds__(kRangeThreads) depth_range_kernel(const uint4* __restrict__ info,
                                                                   const uint32_t* __restrict__ vis_ids,
                                                                   const int64_t* __restrict__ counters, NearKey nk,
                                                                   int S, float p_lo, float p_hi, float pad,
                                                                   float znear, float zfar, float* __restrict__ zrange,
                                                                   const uint32_t* __restrict__ samples) {
    __shared__ RangeLds R;
    depth_range_block(info, vis_ids, counters, nk, S, p_lo, p_hi, pad, znear, zfar, zrange, samples, R);
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

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wavefront LDS view of its 64 Gaussians for the entry expansion.
struct WaveGauss {
    uint32_t excl[kWave];  // first entry of each Gaussian, relative to the wavefront
    uint32_t rect[kWave];  // x0 | y0 << 16
    uint32_t width[kWave];
    uint32_t key[kWave];   // depth bits
    uint32_t bin[kWave];
};

// Position of depth bits L in the depth range as a 32-bit fraction,
// floor(2^32 (L - Lmin) / (Lmax - Lmin)), clamped to [0, 2^32 - 1]. For K =
// 2^k bins, frac >> (32 - k) equals bin_of(L, Lmin, Lmax, K) exactly (floor
// of a floor divided by an integer), which lets each tile pick its own
// power-of-two bin count from one per-Gaussian value.
__device__ __forceinline__ uint32_t depth_frac(uint32_t L, uint32_t Lmin, uint32_t Lmax) {
    if (Lmax <= Lmin || L <= Lmin) return 0u;
    if (L >= Lmax) return 0xFFFFFFFFu;
    return (uint32_t)(((uint64_t)(L - Lmin) << 32) / (uint64_t)(Lmax - Lmin));
}

// Segment of an entry of tile t whose Gaussian has bin value bv (the bin
// for uniform K; for per-tile bin counts the depth fraction, whose top
// log2 K_t bits are the bin: shift = 32 - log2 K_t, 32 for one bin).
template <bool VAR>
__device__ __forceinline__ int64_t segment_of(const SegMap& sm, int64_t t, uint32_t bv) {
    if (!VAR) return t * sm.K + bv;
    const uint2 ts = sm.tile_seg[t];
    return (int64_t)ts.x + (int64_t)((uint64_t)bv >> ts.y);
}

// One (Gaussian, tile) entry of a wavefront's expansion; ok = false for the
// lanes past the wavefront's last entry.
struct Ent {
    int64_t gid, e;
    int tx, ty;
    uint32_t key, bin;
    bool ok;
};

// Load-balanced expansion of the (Gaussian, tile) entries of a wavefront's
// 64 consecutive Gaussians: the entries are enumerated 64 at a time, one per
// lane, and each lane finds its Gaussian by binary search over the
// wavefront's exclusive entry counts. Entries of consecutive Gaussians are
// consecutive in the global entry order, so entry e = emit_off[first] + k.
// f(en) receives R rounds (R x 64 entries) at once, so that it can issue the
// memory operations of all R rounds before waiting for any of them.
template <int R, bool WITH_BIN, bool VAR, class F>
__device__ __forceinline__ void for_wave_entries_at(int64_t g0, const uint4* __restrict__ info, int64_t n,
                                                    const uint32_t* __restrict__ emit_off, int tiles_x, int tiles_y,
                                                    const float* __restrict__ zrange, const NearKey& nk, int K,
                                                    WaveGauss* W, F&& f) {
    const int l = lane();
    if (g0 >= n) return;
    const int64_t g = g0 + l;
    int cnt = 0, x0 = 0, y0 = 0, x1 = 0, y1 = 0;
    uint32_t key = 0;
    if (g < n) {
        const uint4 in = info[g];
        cnt = rect_of(in, tiles_x, tiles_y, x0, y0, x1, y1);
        key = in.x;
    }
    const uint32_t incl = wave_inclusive_sum((uint32_t)cnt);
    const uint32_t total = shfl_u32(incl, kWave - 1);
    if (total == 0) return;
    W->excl[l] = incl - (uint32_t)cnt;
    W->rect[l] = (uint32_t)x0 | ((uint32_t)y0 << 16);
    W->width[l] = (uint32_t)(x1 - x0);
    W->key[l] = key;
    if (WITH_BIN) {
        const uint32_t Lmin = __float_as_uint(zrange[0]), Lmax = __float_as_uint(zrange[1]);
        const uint32_t bk = cnt ? nk(key, g) : 0u;
        W->bin[l] = !cnt ? 0u : VAR ? depth_frac(bk, Lmin, Lmax) : (uint32_t)bin_of(bk, Lmin, Lmax, K);
    }
    const int64_t ebase = emit_off[g0];
    wave_sync();
    for (uint32_t base = 0; base < total; base += R * kWave) {
        Ent en[R];
        int lo[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = base + (uint32_t)(r * kWave + l);
            en[r].ok = k < total;
            en[r].e = ebase + k;
            lo[r] = 0;
        }
        // the R searches are independent; interleaved, their LDS reads overlap
#pragma unroll
        for (int step = kWave / 2; step > 0; step >>= 1)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t k = base + (uint32_t)(r * kWave + l);
                if (W->excl[lo[r] + step] <= k) lo[r] += step;
            }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t k = base + (uint32_t)(r * kWave + l);
            const uint32_t j = k - W->excl[lo[r]], w = W->width[lo[r]], rc = W->rect[lo[r]];
            // lanes past the end hold lo = 63 with a width that may be 0
            const uint32_t ws = w ? w : 1u;
            en[r].tx = (int)(rc & 0xFFFFu) + (int)(j % ws);
            en[r].ty = (int)(rc >> 16) + (int)(j / ws);
            en[r].gid = g0 + lo[r];
            en[r].key = W->key[lo[r]];
            en[r].bin = WITH_BIN ? W->bin[lo[r]] : 0u;
        }
        f(en);
    }
}

// The wavefront's 64 Gaussians of a one-Gaussian-per-thread grid.
template <int R, bool WITH_BIN, bool VAR, class F>
__device__ __forceinline__ void for_wave_entries(const uint4* __restrict__ info, int64_t n,
                                                 const uint32_t* __restrict__ emit_off, int tiles_x, int tiles_y,
                                                 const float* __restrict__ zrange, const NearKey& nk, int K,
                                                 WaveGauss* W, F&& f) {
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1));
    for_wave_entries_at<R, WITH_BIN, VAR>(g0, info, n, emit_off, tiles_x, tiles_y, zrange, nk, K, W, f);
}

constexpr int kExpandRounds = 4;

// Atomic count per (tile, bin) into the calling XCD's copy of the counts.
// All atomics on copy x come from XCD x, so they are carried out in that
// XCD's L2 (workgroup scope) instead of at the memory side; the returned old
// value is the entry's rank inside its copy.
template <bool VAR>
__global__ void __launch_bounds__(256) bin_count_kernel(const uint4* __restrict__ info, int64_t n,
                                                        const uint32_t* __restrict__ emit_off,
                                                        const float* __restrict__ zrange, NearKey nk, SegMap sm,
                                                        int tiles_x, int tiles_y, uint32_t* __restrict__ count,
                                                        int64_t nseg,
                                                        uint32_t* __restrict__ entry_rank, int64_t capacity) {
    __shared__ WaveGauss wg[4];
    const uint32_t x = (uint32_t)xcc_id() % (uint32_t)kCopies;
    const int64_t S = VAR ? (int64_t)sm.seg_base[(int64_t)tiles_x * tiles_y] : nseg;
    uint32_t* cnt = count + (int64_t)x * S;
    constexpr int R = kExpandRounds;
    for_wave_entries<R, true, VAR>(info, n, emit_off, tiles_x, tiles_y, zrange, nk, sm.K, &wg[threadIdx.x / kWave],
                                   [&](const Ent (&en)[R]) {
                                       uint32_t rk[R];
#pragma unroll
                                       for (int r = 0; r < R; ++r) {
                                           rk[r] = 0;
                                           if (en[r].ok) {
                                               const int64_t sg =
                                                   segment_of<VAR>(sm, (int64_t)en[r].ty * tiles_x + en[r].tx, en[r].bin);
                                               rk[r] = __hip_atomic_fetch_add(&cnt[sg], 1u, __ATOMIC_RELAXED,
                                                                              __HIP_MEMORY_SCOPE_WORKGROUP);
                                           }
                                       }
#pragma unroll
                                       for (int r = 0; r < R; ++r)
                                           if (en[r].ok && en[r].e < capacity)
                                               entry_rank[en[r].e] = (rk[r] & 0x1FFFFFFFu) | (x << 29);
                                   });
}

// pair = depth bits << 32 | id at base[copy][segment] + rank. An entry that
// is alone in its segment is final here, so its packed record is written
// too; longer segments get theirs from the repair sorts.
template <bool VAR>
__global__ void __launch_bounds__(256) bin_scatter_kernel(const uint4* __restrict__ info, int64_t n,
                                                          const uint32_t* __restrict__ emit_off,
                                                          const float* __restrict__ zrange, NearKey nk, SegMap sm,
                                                          int tiles_x, int tiles_y,
                                                          const uint32_t* __restrict__ bin_off,
                                                          const uint32_t* __restrict__ base, int64_t nseg,
                                                          const uint32_t* __restrict__ entry_rank,
                                                          uint64_t* __restrict__ pairs, int64_t capacity,
                                                          RecordSink rs) {
    __shared__ WaveGauss wg[4];
    const int64_t S = VAR ? (int64_t)sm.seg_base[(int64_t)tiles_x * tiles_y] : nseg;
    constexpr int R = kExpandRounds;
    for_wave_entries<R, true, VAR>(info, n, emit_off, tiles_x, tiles_y, zrange, nk, sm.K, &wg[threadIdx.x / kWave],
                                   [&](const Ent (&en)[R]) {
                                       bool ok[R];
                                       uint32_t rk[R];
#pragma unroll
                                       for (int r = 0; r < R; ++r) {
                                           ok[r] = en[r].ok && en[r].e < capacity;
                                           rk[r] = ok[r] ? entry_rank[en[r].e] : 0u;
                                       }
                                       int64_t sg[R];
                                       uint32_t bs[R];
#pragma unroll
                                       for (int r = 0; r < R; ++r) {
                                           sg[r] = ok[r] ? segment_of<VAR>(sm, (int64_t)en[r].ty * tiles_x + en[r].tx,
                                                                           en[r].bin)
                                                         : 0;
                                           bs[r] = ok[r] ? base[(int64_t)(rk[r] >> 29) * S + sg[r]] : 0u;
                                       }
#pragma unroll
                                       for (int r = 0; r < R; ++r) {
                                           const int64_t p = (int64_t)bs[r] + (rk[r] & 0x1FFFFFFFu);
                                           if (!ok[r] || p >= capacity) continue;
                                           const uint64_t pair = ((uint64_t)en[r].key << 32) | (uint64_t)en[r].gid;
                                           pairs[p] = pair;
                                           if (rs.masks && bin_off[sg[r] + 1] - bin_off[sg[r]] == 1)
                                               rs.put((uint32_t)sg[r], (uint32_t)p, pair);
                                       }
                                   });
}

// ---------------------------------------------------------------------------
// grouped binning (uniform K): the same count / scan / scatter, done in two
// levels so that no per-entry global atomic is needed. Groups are runs of
// GT consecutive tiles, i.e. contiguous ranges of GS = GT K segments.
//   group_count    each workgroup expands the entries of kGroupChunk
//                  Gaussians, counts them per group in LDS and reserves its
//                  slice of every group it touches with one global atomic
//                  per (workgroup, group): wgbase[wg][g];
//   group_scan     exclusive prefix of the group totals;
//   group_scatter  the same workgroups expand their entries again and write
//                  (pair, segment within the group) at group offset + slice
//                  base + an LDS rank;
//   group_sort     one workgroup per group: LDS counting sort of its entries
//                  by segment, bin offsets, repair queues.
// ---------------------------------------------------------------------------

constexpr int kCountThreads = kRangeThreads;

struct CountLds {
    uint32_t hist[kMaxGroups];
    WaveGauss wg[kCountThreads / kWave];
};

// Workgroup 0: the depth range. Workgroups 1..: the group count of chunk
// blockIdx.x - 1 (kGroupChunk Gaussians, 16 wavefronts).
__global__ void __launch_bounds__(kCountThreads) group_count_kernel(const uint4* __restrict__ info, int64_t n,
                                                                    const uint32_t* __restrict__ emit_off, GroupMap gm,
                                                                    int tiles_x, int tiles_y,
                                                                    uint32_t* __restrict__ gcount,
                                                                    uint32_t* __restrict__ wgbase, RangeArgs ra) {
    __shared__ union {
        CountLds c;
        RangeLds r;
    } U;
    if (blockIdx.x == 0) {
        depth_range_block(info, ra.vis_ids, ra.counters, ra.nk, ra.S, ra.p_lo, ra.p_hi, ra.pad, ra.znear, ra.zfar,
                          ra.zrange, ra.samples, U.r);
        return;
    }
    const int64_t chunk = blockIdx.x - 1;
    uint32_t* hist = U.c.hist;
    for (int g = threadIdx.x; g < gm.G; g += kCountThreads) hist[g] = 0;
    __syncthreads();
    const int w = threadIdx.x / kWave;
    constexpr int NW = kCountThreads / kWave;
    const int64_t first = chunk * kGroupChunk;
    constexpr int R = kExpandRounds;
    for (int it = 0; it < kGroupChunk / kCountThreads; ++it) {
        const int64_t g0 = first + (int64_t)(it * NW + w) * kWave;
        for_wave_entries_at<R, false, false>(g0, info, n, emit_off, tiles_x, tiles_y, nullptr, NearKey{}, gm.K,
                                             &U.c.wg[w], [&](const Ent (&en)[R]) {
#pragma unroll
                                                 for (int r = 0; r < R; ++r)
                                                     if (en[r].ok)
                                                         atomicAdd(&hist[(uint32_t)(en[r].ty * tiles_x + en[r].tx) /
                                                                         (uint32_t)gm.GT],
                                                                   1u);
                                             });
    }
    __syncthreads();
    uint32_t* row = wgbase + chunk * gm.G;
    for (int g = threadIdx.x; g < gm.G; g += kCountThreads) {
        const uint32_t h = hist[g];
        if (h) row[g] = atomicAdd(&gcount[g], h);
    }
}

#ifndef TGS_SCATTER_THREADS
#define TGS_SCATTER_THREADS 512
#endif
constexpr int kScatterThreads = TGS_SCATTER_THREADS;  // threads of a group-scatter workgroup

template <bool VAR>
__global__ void __launch_bounds__(kScatterThreads) group_scatter_kernel(const uint4* __restrict__ info, int64_t n,
                                                            const uint32_t* __restrict__ emit_off,
                                                            const float* __restrict__ zrange, NearKey nk, GroupMap gm,
                                                            int tiles_x, int tiles_y,
                                                            const uint32_t* __restrict__ group_off,
                                                            const uint32_t* __restrict__ wgbase,
                                                            uint64_t* __restrict__ tmp_pair,
                                                            uint16_t* __restrict__ tmp_code, int64_t capacity) {
    constexpr int NT = kScatterThreads, NW = NT / kWave;
    static_assert(kGroupChunk % NT == 0, "whole wavefront slabs per chunk");
    __shared__ WaveGauss wg[NW];
    __shared__ uint32_t cursor[kMaxGroups];
    const uint32_t* row = wgbase + (int64_t)blockIdx.x * gm.G;
    // slots of groups this workgroup does not touch hold stale values and
    // are never used
    for (int g = threadIdx.x; g < gm.G; g += NT) cursor[g] = group_off[g] + row[g];
    __syncthreads();
    const int w = threadIdx.x / kWave;
    const int64_t first = (int64_t)blockIdx.x * kGroupChunk;
    constexpr int R = kExpandRounds;
    for (int it = 0; it < kGroupChunk / NT; ++it) {
        const int64_t g0 = first + (int64_t)(it * NW + w) * kWave;
        for_wave_entries_at<R, true, VAR>(
            g0, info, n, emit_off, tiles_x, tiles_y, zrange, nk, gm.K * gm.SB, &wg[w], [&](const Ent (&en)[R]) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (!en[r].ok) continue;
                    const uint32_t t = (uint32_t)(en[r].ty * tiles_x + en[r].tx);
                    const uint32_t grp = t / (uint32_t)gm.GT;
                    uint32_t code;
                    if (VAR) {
                        // en.bin is the depth fraction: bin = frac >> shift, then
                        // the next log2 SB_g bits are the sub-bin
                        const uint2 ts = gm.tile_seg[t];
                        const uint4 gi = gm.ginfo[grp];
                        const uint64_t f = en[r].bin;
                        const uint32_t seg = ts.x + (uint32_t)(f >> ts.y) - gi.x;
                        const uint32_t sub = (uint32_t)(f >> (ts.y - gi.z)) & ((1u << gi.z) - 1u);
                        code = (seg << gi.z) + sub;
                    } else {
                        // en.bin is the bin at K SB bins: (bin, sub) = (bin / SB, bin % SB)
                        code = (t - grp * (uint32_t)gm.GT) * (uint32_t)(gm.K * gm.SB) + en[r].bin;
                    }
                    const uint32_t pos = atomicAdd(&cursor[grp], 1u);
                    if (pos >= capacity) continue;
                    tmp_pair[pos] = ((uint64_t)en[r].key << 32) | (uint64_t)en[r].gid;
                    tmp_code[pos] = (uint16_t)code;
                }
            });
    }
}

// ---------------------------------------------------------------------------
// exact repair
// ---------------------------------------------------------------------------

// A queued segment: its id s (for the records) and position. The lists
// hold segment ids located by bin_off, or (DESC) {begin, length} pairs of
// sub-segments, which carry no records.
template <bool DESC>
__device__ __forceinline__ void locate(const uint32_t* __restrict__ bin_off, uint2 entry, uint32_t& s,
                                       uint32_t& begin, uint32_t& len) {
    if (DESC) {
        s = 0;
        begin = entry.x;
        len = entry.y;
    } else {
        s = entry.x;
        begin = bin_off[s];
        len = bin_off[s + 1] - begin;
    }
}

// Buckets 0..4 in one launch. The wavefront jobs of all five buckets form
// one list, longest first (bucket 4: one 65..512 segment per wavefront job,
// 2, 4 or 8 keys per lane; buckets 3..0: 1, 2, 4, 8 segments of 64 / G
// lanes each), which every wavefront strides through, so that no wavefront
// gets a job of every bucket. Each bucket's stretch of the list is its own
// loop with the group size fixed at compile time.
struct SmallSort {
    const uint32_t* bin_off;
    const uint32_t* lists;
    int64_t nseg;
    uint64_t* pairs;
    uint32_t waves, wid;
};

// The first job >= a of wavefront wid (jobs wid, wid + waves, ...).
__device__ __forceinline__ uint32_t first_job(const SmallSort& S, uint32_t a) {
    return a + (S.wid + S.waves - a % S.waves) % S.waves;
}

// Jobs [j_begin, j_end) of bucket b (list entries from (j - j_begin) (64 /
// G)): 64 / G segments of at most G keys per job, G lanes each.
template <int G, bool DESC>
__device__ __forceinline__ void sort_groups(const SmallSort& S, int b, uint32_t j_begin, uint32_t j_end, uint32_t cnt,
                                            const RecordSink& rs) {
    const int l = lane(), li = l & (G - 1);
    const uint32_t sub = (uint32_t)(l / G);
    for (uint32_t j = first_job(S, j_begin); j < j_end; j += S.waves) {
        const uint32_t i = (j - j_begin) * (uint32_t)(kWave / G) + sub;
        uint32_t sg = 0, begin = 0, len = 0;
        if (i < cnt) {
            const int64_t at = (int64_t)b * S.nseg + i;
            locate<DESC>(S.bin_off, DESC ? reinterpret_cast<const uint2*>(S.lists)[at] : make_uint2(S.lists[at], 0u),
                         sg, begin, len);
        }
        uint64_t* seg = S.pairs + begin;
        uint64_t v = (uint32_t)li < len ? seg[li] : ~0ull;
        v = group_bitonic<G>(v, li);
        if ((uint32_t)li < len) {
            seg[li] = v;
            if (!DESC) rs.put(sg, begin + li, v);
        }
    }
}

template <bool DESC>
__global__ void __launch_bounds__(256) sort_small_kernel(const uint32_t* __restrict__ bin_off,
                                                         const uint32_t* __restrict__ lists, int64_t nseg,
                                                         const uint32_t* __restrict__ bucket_count,
                                                         uint64_t* __restrict__ pairs, RecordSink rs) {
    const SmallSort S{bin_off, lists, nseg, pairs, gridDim.x * (blockDim.x / kWave),
                      blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave};
    const uint32_t c0 = bucket_count[0], c1 = bucket_count[1], c2 = bucket_count[2], c3 = bucket_count[3],
                   c4 = bucket_count[4];
    // job counts and their running sums, bucket 4 first
    const uint32_t j4 = c4, j3 = j4 + c3, j2 = j3 + (c2 + 1) / 2, j1 = j2 + (c1 + 3) / 4, j0 = j1 + (c0 + 7) / 8;
    if (S.wid >= j0) return;
    for (uint32_t j = first_job(S, 0); j < j4; j += S.waves) {
        uint32_t sg = 0, begin = 0, len = 0;
        const int64_t at = (int64_t)4 * nseg + j;
        locate<DESC>(bin_off, DESC ? reinterpret_cast<const uint2*>(lists)[at] : make_uint2(lists[at], 0u), sg,
                     begin, len);
        if (len <= 2 * kWave)
            sort_wave_reg<2, !DESC>(pairs + begin, sg, begin, len, rs);
        else if (len <= 4 * kWave)
            sort_wave_reg<4, !DESC>(pairs + begin, sg, begin, len, rs);
        else
            sort_wave_reg<8, !DESC>(pairs + begin, sg, begin, len, rs);
    }
    sort_groups<64, DESC>(S, 3, j4, j3, c3, rs);
    sort_groups<32, DESC>(S, 2, j3, j2, c2, rs);
    sort_groups<16, DESC>(S, 1, j2, j1, c1, rs);
    sort_groups<8, DESC>(S, 0, j1, j0, c0, rs);
}

// Buckets 5..7: one workgroup per segment. 513..8192 keys: bitonic network
// in LDS over the next power of two, padded with the maximum key. Above
// 8192: in place in global memory, with the network in the form whose every
// comparator puts the smaller key at the lower index (each merge starts by
// comparing mirrored positions), so positions at or beyond the segment
// length act as +infinity and are never touched.
constexpr int kLargeThreads = 512;
constexpr int kLargeCap = 8192;

constexpr int kOrderBuckets = 33;  // tile order buckets: bit lengths 32 .. 0 of the entry count
template <int NT>
__device__ __forceinline__ void tile_place_chunk(const TileOrder& to, int64_t chunk, uint32_t* h, uint32_t* base);

// One segment of 513..8192 keys by the workgroup: coalesced load into LDS
// (padded slots), E keys per thread into registers, the register / lane /
// LDS bitonic network of sort_block_reg, and a coalesced store (with the
// records when !DESC).
template <int E, bool DESC>
__device__ __forceinline__ void sort_large_block(uint64_t* pairs, uint32_t s, uint32_t begin, uint32_t len,
                                                 const RecordSink& rs, uint64_t* buf) {
    constexpr uint32_t P = (uint32_t)kLargeThreads * E;
    for (uint32_t e = threadIdx.x; e < P; e += kLargeThreads) buf[block_slot<E>(e)] = e < len ? pairs[begin + e] : ~0ull;
    __syncthreads();
    uint64_t v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = buf[block_slot<E>((uint32_t)(threadIdx.x * E + k))];
    __syncthreads();
    sort_block_reg<E, kLargeThreads>(v, buf);
#pragma unroll
    for (int k = 0; k < E; ++k) buf[block_slot<E>((uint32_t)(threadIdx.x * E + k))] = v[k];
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < len; e += kLargeThreads) {
        const uint64_t x = buf[block_slot<E>(e)];
        pairs[begin + e] = x;
        if (!DESC) rs.put(s, begin + e, x);
    }
    __syncthreads();
}

template <bool DESC>
__global__ void __launch_bounds__(kLargeThreads) sort_large_kernel(const uint32_t* __restrict__ bin_off,
                                                                   const uint32_t* __restrict__ lists, int64_t nseg,
                                                                   const uint32_t* __restrict__ bucket_count,
                                                                   uint64_t* pairs, RecordSink rs, TileOrder to) {
    __shared__ uint64_t buf[kLargeCap + kLargeThreads];  // block_slot<E> of P = 512 E keys: at most 8192 + 512
    auto entry = [&](int bucket, uint32_t i) {
        const int64_t at = (int64_t)bucket * nseg + i;
        return DESC ? reinterpret_cast<const uint2*>(lists)[at] : make_uint2(lists[at], 0u);
    };
    for (int bucket = 5; bucket <= 6; ++bucket) {
        const uint32_t cnt = bucket_count[bucket];
        for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
            uint32_t s, begin, len;
            locate<DESC>(bin_off, entry(bucket, i), s, begin, len);
            uint32_t P = 1;
            while (P < len) P <<= 1;
            // E = P / kLargeThreads keys per thread (P = 1024 .. 8192)
            if (P <= 1024)
                sort_large_block<2, DESC>(pairs, s, begin, len, rs, buf);
            else if (P <= 2048)
                sort_large_block<4, DESC>(pairs, s, begin, len, rs, buf);
            else if (P <= 4096)
                sort_large_block<8, DESC>(pairs, s, begin, len, rs, buf);
            else
                sort_large_block<16, DESC>(pairs, s, begin, len, rs, buf);
        }
    }
    const uint32_t cnt = bucket_count[7];
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        uint32_t s, begin, len;
        locate<DESC>(bin_off, entry(7, i), s, begin, len);
        uint64_t* a = pairs + begin;
        uint32_t P = 1;
        while (P < len) P <<= 1;
        for (uint32_t k = 2; k <= P; k <<= 1) {
            const uint32_t h = k >> 1;
            for (uint32_t t = threadIdx.x; t < P / 2; t += kLargeThreads) {
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
                for (uint32_t t = threadIdx.x; t < P / 2; t += kLargeThreads) {
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
        if (!DESC)
            for (uint32_t e = threadIdx.x; e < len; e += kLargeThreads) rs.put(s, begin + e, a[e]);
        __syncthreads();
    }
    // the tile order's placement, by the last workgroups (the first ones
    // take the long segments)
    if (to.order) {
        __shared__ uint32_t oh[kOrderBuckets], ob[kOrderBuckets];
        const int64_t chunks = (to.T + kLargeThreads - 1) / kLargeThreads;
        for (int64_t c = (int64_t)gridDim.x - 1 - blockIdx.x; c < chunks; c += gridDim.x)
            tile_place_chunk<kLargeThreads>(to, c, oh, ob);
    }
}

// ---------------------------------------------------------------------------
// heaviest-first tile order
// ---------------------------------------------------------------------------

__device__ __forceinline__ int order_bucket(uint32_t c) { return c ? __builtin_clz(c) : 32; }

// Counts per bucket are aggregated per wavefront (one LDS atomic per
// distinct bucket value in the wavefront) before the LDS atomics.
__device__ __forceinline__ uint32_t wave_aggregated_add(uint32_t* ctr, int b, bool active) {
    uint32_t slot = 0;
    uint64_t pending = ballot(active);
    while (pending) {
        const int leader = __builtin_ctzll(pending);
        const int lb = (int)shfl_u32((uint32_t)b, leader);
        const uint64_t m = ballot(active && b == lb);
        uint32_t base = 0;
        if (lane() == leader) base = atomicAdd(&ctr[lb], (uint32_t)__builtin_popcountll(m));
        base = shfl_u32(base, leader);
        if (active && b == lb) slot = base + rank_in(m);
        pending &= ~m;
    }
    return slot;
}

// Two launches over all tiles: (1) bucket histogram (per-workgroup LDS,
// then one global atomic per bucket and workgroup), (2) placement: every
// workgroup scans the global histogram and reserves its slots per bucket
// with one global atomic per bucket. Order inside a bucket is arbitrary.
__device__ __forceinline__ uint32_t tile_count(const uint32_t* offsets, const SegMap& sm, int64_t t) {
    return offsets[sm.first(t + 1)] - offsets[sm.first(t)];
}

__global__ void __launch_bounds__(256) tile_hist_kernel(const uint32_t* __restrict__ offsets, SegMap sm, int64_t T,
                                                        uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[kOrderBuckets];
    if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = t < T;
    (void)wave_aggregated_add(h, act ? order_bucket(tile_count(offsets, sm, t)) : 0, act);
    __syncthreads();
    if (threadIdx.x < kOrderBuckets && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Placement of tiles [chunk NT, chunk NT + NT) by a workgroup of NT
// threads; h, base: LDS [kOrderBuckets]. Ends with a barrier.
template <int NT>
__device__ __forceinline__ void tile_place_chunk(const TileOrder& to, int64_t chunk, uint32_t* h, uint32_t* base) {
    const uint32_t* hist = to.hist;
    uint32_t* cursor = to.hist + kOrderBuckets;
    const int64_t T = to.T;
    if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t = chunk * NT + threadIdx.x;
    const bool act = t < T;
    const int b = act ? order_bucket(tile_count(to.offsets, to.sm, t)) : 0;
    const uint32_t slot = wave_aggregated_add(h, b, act);
    __syncthreads();
    if (threadIdx.x < kOrderBuckets) {
        uint32_t start = 0;
        for (int k = 0; k < (int)threadIdx.x; ++k) start += hist[k];
        base[threadIdx.x] = h[threadIdx.x] ? start + atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]) : 0u;
    }
    __syncthreads();
    if (act) to.order[base[b] + slot] = (uint32_t)t;
    if (chunk == 0 && threadIdx.x == 0) {
        // counts >= 2^h have a bit length > h: buckets 0 .. 31 - h. The
        // threshold is the smallest power of two >= split and >= `factor`
        // times the mean count of the non-empty tiles that leaves at most
        // kSplitTiles tiles above it, so the split set is a union of whole
        // buckets (independent of the order inside a bucket). Only tiles
        // far longer than the typical walk are on the critical path, and
        // only when the longest reach at least twice that bound (a long
        // tail): where every tile is long the quad walk's extra
        // instructions per entry cost more than its shorter walks gain.
        uint32_t nh = 0, thr = 0;
        if (to.split > 0) {
            const uint64_t m = to.offsets[to.sm.first(T)];
            const uint64_t nonempty = (uint64_t)T - hist[32];
            // with fewer block wavefronts than the CUs hold (256 x 32), the
            // quad walks run on otherwise idle SIMDs: no bound from the mean
            const bool filled = 4 * nonempty >= (uint64_t)kFillWaves;
            const uint64_t rel = nonempty && filled ? (uint64_t)to.factor * m / nonempty : 0;
            int top = 0;  // bucket of the longest tiles
            while (top < 32 && hist[top] == 0) ++top;
            const uint64_t longest = top < 32 ? (uint64_t)1 << (31 - top) : 0;  // their lower bound
            int h0 = rel == 0 || longest >= 2 * rel ? 31 - __builtin_clz((uint32_t)to.split) : 32;
            while (h0 < 31 && ((uint64_t)1 << h0) < rel) ++h0;
            for (int h = h0; h <= 31; ++h) {
                uint32_t c = 0;
                for (int k = 0; k <= 31 - h; ++k) c += hist[k];
                if (c <= (uint32_t)kSplitTiles) {
                    nh = c;
                    thr = 1u << h;
                    break;
                }
            }
        }
        to.order[T] = nh;
        to.order[T + 1] = thr;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(256) tile_place_kernel(TileOrder to) {
    __shared__ uint32_t h[kOrderBuckets], base[kOrderBuckets];
    tile_place_chunk<256>(to, blockIdx.x, h, base);
}

// ---------------------------------------------------------------------------
// global-sort comparator
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) emit_keys_kernel(const uint4* __restrict__ info, int64_t n,
                                                        const uint32_t* __restrict__ emit_off, int tiles_x,
                                                        int tiles_y, uint64_t* __restrict__ keys,
                                                        uint32_t* __restrict__ vals, int64_t capacity) {
    __shared__ WaveGauss wg[4];
    constexpr int R = kExpandRounds;
    for_wave_entries<R, false, false>(info, n, emit_off, tiles_x, tiles_y, nullptr, NearKey{}, 1,
                                      &wg[threadIdx.x / kWave], [&](const Ent (&en)[R]) {
#pragma unroll
                                          for (int r = 0; r < R; ++r) {
                                              if (!en[r].ok || en[r].e >= capacity) continue;
                                              keys[en[r].e] = ((uint64_t)(en[r].ty * tiles_x + en[r].tx) << 32) |
                                                              en[r].key;
                                              vals[en[r].e] = (uint32_t)en[r].gid;
                                          }
                                      });
}

// Without a host-side entry count the sort runs over all `capacity` slots:
// the slots past the device count M get keys of tile T (past the last
// tile), which sort after every real entry and which tile_ranges_kernel
// leaves out (tile_off[T] = M).
__global__ void __launch_bounds__(256) pad_keys_kernel(uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                       const int64_t* __restrict__ counters, int64_t capacity,
                                                       uint64_t pad) {
    const int64_t m = counters[0];
    for (int64_t i = (m > 0 ? m : 0) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < capacity;
         i += (int64_t)gridDim.x * blockDim.x) {
        keys[i] = pad;
        vals[i] = 0u;
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

hipError_t launch_depth_range(const uint32_t* info, const uint32_t* vis_ids, const int64_t* counters, NearKey nk,
                              int S, float p_lo, float p_hi, float pad, float znear, float zfar, float* zrange,
                              uint32_t* samples, hipStream_t s) {
    const auto* in = reinterpret_cast<const uint4*>(info);
    hipLaunchKernelGGL(range_samples_kernel, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, s, in, vis_ids, counters,
                       nk, S, samples);
    hipLaunchKernelGGL(depth_range_kernel, dim3(1), dim3(kRangeThreads), 0, s, in, vis_ids, counters, nk, S, p_lo, p_hi,
                       pad, znear, zfar, zrange, samples);
    return hipGetLastError();
}

hipError_t launch_bin_count(const uint32_t* info, int64_t n, const uint32_t* emit_off, const float* zrange,
                            NearKey nk, SegMap sm, int tiles_x, int tiles_y, uint32_t* count, int64_t nseg,
                            uint32_t* entry_rank, int64_t capacity, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const auto* in = reinterpret_cast<const uint4*>(info);
    if (sm.seg_base)
        hipLaunchKernelGGL(bin_count_kernel<true>, dim3(grid_for(n, 256)), dim3(256), 0, s, in, n, emit_off, zrange,
                           nk, sm, tiles_x, tiles_y, count, nseg, entry_rank, capacity);
    else
        hipLaunchKernelGGL(bin_count_kernel<false>, dim3(grid_for(n, 256)), dim3(256), 0, s, in, n, emit_off, zrange,
                           nk, sm, tiles_x, tiles_y, count, nseg, entry_rank, capacity);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(const uint32_t* info, int64_t n, const uint32_t* emit_off, const float* zrange,
                              NearKey nk, SegMap sm, int tiles_x, int tiles_y, const uint32_t* bin_off,
                              const uint32_t* base, int64_t nseg, const uint32_t* entry_rank, uint64_t* pairs,
                              int64_t capacity, RecordSink rs, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const auto* in = reinterpret_cast<const uint4*>(info);
    if (sm.seg_base)
        hipLaunchKernelGGL(bin_scatter_kernel<true>, dim3(grid_for(n, 256)), dim3(256), 0, s, in, n, emit_off, zrange,
                           nk, sm, tiles_x, tiles_y, bin_off, base, nseg, entry_rank, pairs, capacity, rs);
    else
        hipLaunchKernelGGL(bin_scatter_kernel<false>, dim3(grid_for(n, 256)), dim3(256), 0, s, in, n, emit_off,
                           zrange, nk, sm, tiles_x, tiles_y, bin_off, base, nseg, entry_rank, pairs, capacity, rs);
    return hipGetLastError();
}

hipError_t launch_repair(const uint32_t* bin_off, int64_t nseg, uint64_t* pairs, const uint32_t* seg_lists,
                         const uint32_t* bucket_count, RecordSink rs, bool desc, const TileOrder& to, hipStream_t s) {
    if (nseg == 0) return launch_tile_place(to, s);
    const unsigned small_blocks = (unsigned)std::min<int64_t>(std::max<int64_t>((nseg + 31) / 32, 1), 4096);
    if (desc) {
        hipLaunchKernelGGL(sort_small_kernel<true>, dim3(small_blocks), dim3(256), 0, s, bin_off, seg_lists, nseg,
                           bucket_count, pairs, rs);
        hipLaunchKernelGGL(sort_large_kernel<true>, dim3(512), dim3(kLargeThreads), 0, s, bin_off, seg_lists, nseg,
                           bucket_count, pairs, rs, to);
    } else {
        hipLaunchKernelGGL(sort_small_kernel<false>, dim3(small_blocks), dim3(256), 0, s, bin_off, seg_lists, nseg,
                           bucket_count, pairs, rs);
        hipLaunchKernelGGL(sort_large_kernel<false>, dim3(512), dim3(kLargeThreads), 0, s, bin_off, seg_lists, nseg,
                           bucket_count, pairs, rs, to);
    }
    return hipGetLastError();
}

hipError_t launch_tile_order(const uint32_t* offsets, SegMap sm, int64_t T, uint32_t* hist, uint32_t* order, int split,
                             int factor, hipStream_t s) {
    if (T == 0) return hipSuccess;
    hipLaunchKernelGGL(tile_hist_kernel, dim3(grid_for(T, 256)), dim3(256), 0, s, offsets, sm, T, hist);
    hipLaunchKernelGGL(tile_place_kernel, dim3(grid_for(T, 256)), dim3(256), 0, s,
                       TileOrder{offsets, sm, T, hist, order, split, factor});
    return hipGetLastError();
}

hipError_t launch_tile_place(const TileOrder& to, hipStream_t s) {
    if (to.T == 0 || !to.order) return hipSuccess;
    hipLaunchKernelGGL(tile_place_kernel, dim3(grid_for(to.T, 256)), dim3(256), 0, s, to);
    return hipGetLastError();
}

GroupMap group_map(int64_t T, int K, int sub) {
    GroupMap gm{K, 1, 0, 0, 1, T, nullptr, nullptr, nullptr};
    if (T <= 0 || K <= 0) return gm;
    int64_t gt = K >= kGroupSegTarget ? 1 : kGroupSegTarget / K;
    while ((T + gt - 1) / gt > kMaxGroups) gt *= 2;
    if (gt * K > kMaxGroupSegs) return gm;
    gm.GT = (int)gt;
    gm.G = (int)((T + gt - 1) / gt);
    gm.GS = (int)(gt * K);
    if (sub > 1 && (int64_t)gm.GS * sub <= kMaxGroupSegs) gm.SB = sub;
    return gm;
}

GroupMap group_map_var(int64_t T, int K, int sub) {
    GroupMap gm{K, 1, 0, 0, 1, T, nullptr, nullptr, nullptr};
    if (T <= 0 || K <= 0 || K > kMaxGroupSegs) return gm;
    int64_t gt = std::min<int64_t>(8, kMaxGroupSegs / K);
    while ((T + gt - 1) / gt > kMaxGroups) gt *= 2;
    if (gt * K > kMaxGroupSegs) return gm;
    gm.GT = (int)gt;
    gm.G = (int)((T + gt - 1) / gt);
    gm.GS = (int)(gt * K);
    gm.SB = sub > 1 ? sub : 1;
    return gm;
}

hipError_t launch_group_count(const uint32_t* info, int64_t n, const uint32_t* emit_off, GroupMap gm, int tiles_x,
                              int tiles_y, uint32_t* gcount, uint32_t* wgbase, const RangeArgs& ra, hipStream_t s) {
    static_assert(kGroupChunk % kCountThreads == 0, "whole wavefront slabs per chunk");
    if (ra.samples)
        hipLaunchKernelGGL(range_samples_kernel, dim3((unsigned)((ra.S + 255) / 256)), dim3(256), 0, s,
                           reinterpret_cast<const uint4*>(info), ra.vis_ids, ra.counters, ra.nk, ra.S, ra.samples);
    const int64_t chunks = (n + kGroupChunk - 1) / kGroupChunk;
    hipLaunchKernelGGL(group_count_kernel, dim3((unsigned)(chunks + 1)), dim3(kCountThreads), 0, s,
                       reinterpret_cast<const uint4*>(info), n, emit_off, gm, tiles_x, tiles_y, gcount, wgbase, ra);
    return hipGetLastError();
}

hipError_t launch_group_scatter(const uint32_t* info, int64_t n, const uint32_t* emit_off, const float* zrange,
                                NearKey nk, GroupMap gm, int tiles_x, int tiles_y, const uint32_t* group_off,
                                const uint32_t* wgbase, uint64_t* tmp_pair, uint16_t* tmp_code, int64_t capacity,
                                hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + kGroupChunk - 1) / kGroupChunk;
    if (gm.seg_base)
        hipLaunchKernelGGL(group_scatter_kernel<true>, dim3((unsigned)blocks), dim3(kScatterThreads), 0, s,
                           reinterpret_cast<const uint4*>(info), n, emit_off, zrange, nk, gm, tiles_x, tiles_y,
                           group_off, wgbase, tmp_pair, tmp_code, capacity);
    else
        hipLaunchKernelGGL(group_scatter_kernel<false>, dim3((unsigned)blocks), dim3(kScatterThreads), 0, s,
                           reinterpret_cast<const uint4*>(info), n, emit_off, zrange, nk, gm, tiles_x, tiles_y,
                           group_off, wgbase, tmp_pair, tmp_code, capacity);
    return hipGetLastError();
}

hipError_t launch_emit_keys(const uint32_t* info, int64_t n, const uint32_t* emit_off, int tiles_x, int tiles_y,
                            uint64_t* keys, uint32_t* vals, int64_t capacity, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(emit_keys_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       reinterpret_cast<const uint4*>(info), n, emit_off, tiles_x, tiles_y, keys, vals, capacity);
    return hipGetLastError();
}

hipError_t launch_pad_keys(uint64_t* keys, uint32_t* vals, const int64_t* counters, int64_t capacity, int64_t T,
                           hipStream_t s) {
    if (capacity <= 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<int64_t>((capacity + 255) / 256, 2048);
    hipLaunchKernelGGL(pad_keys_kernel, dim3(grid), dim3(256), 0, s, keys, vals, counters, capacity,
                       (uint64_t)T << 32);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint64_t* keys, int64_t m, int64_t T, uint32_t* tile_off, hipStream_t s) {
    hipLaunchKernelGGL(tile_ranges_kernel, dim3(grid_for(T + 1, 256)), dim3(256), 0, s, keys, m, T, tile_off);
    return hipGetLastError();
}

}  // namespace tgs
