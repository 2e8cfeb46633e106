// Single-pass exclusive prefix sums with decoupled look-back: each workgroup
// takes a ticket (so every workgroup it waits on is already running),
// publishes its aggregate, adds the aggregates / inclusive prefixes of its
// predecessors (a status word per workgroup: 2 flag bits + 62 value bits,
// exchanged with agent-scope relaxed atomics), publishes its inclusive
// prefix and writes its outputs. Items are read in coalesced rounds of 256.
// Used for the per-Gaussian entry offsets (fused with the visible-Gaussian
// list), the per-tile segment bases, the rule-based repair selection and, on
// the per-entry atomic path, the (tile, bin) counts -> bin offsets (fused
// with the per-XCD bases and the repair-bucket classification). Also here:
// the group scan and the per-group counting sort of grouped binning.
#include <algorithm>

#include "common.hpp"

namespace tgs {

namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 8;
constexpr int kPerBlock = kThreads * kRounds;
#ifndef TGS_EMIT_THREADS
#define TGS_EMIT_THREADS 1024
#endif
#ifndef TGS_EMIT_ROUNDS
#define TGS_EMIT_ROUNDS 4
#endif
constexpr int kEmitThreads = TGS_EMIT_THREADS;  // threads of an emit-scan workgroup
constexpr int kEmitRounds = TGS_EMIT_ROUNDS;    // items per thread of the emit scan
constexpr int kEmitPerBlock = kEmitThreads * kEmitRounds;
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;

template <int NT = kThreads>
__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t* lds) {
    constexpr int NW = NT / kWave;
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
template <int NT = kThreads>
__device__ __forceinline__ uint32_t block_excl_u32(uint32_t v, uint32_t* lds, uint32_t* total) {
    constexpr int NW = NT / kWave;
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

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        const uint32_t lo = shfl_xor_u32((uint32_t)v, m), hi = shfl_xor_u32((uint32_t)(v >> 32), m);
        v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

// Sum of the values of workgroups 0..b-1, by one whole wavefront: each
// lane reads one status word of a window of 64 predecessors (nearest in lane
// 0) and waits until it is published; the window's values up to the nearest
// inclusive prefix are summed, else the whole window is added and the next
// window further back is read. Waits only on workgroups with a smaller
// ticket, which are running or done; workgroup 0 always publishes an
// inclusive prefix, and positions before it count as an inclusive zero.
__device__ uint64_t look_back(const uint64_t* status, int64_t b) {
    uint64_t prefix = 0;
    for (int64_t hi = b - 1;; hi -= kWave) {
        const int64_t p = hi - lane();
        uint64_t s = kFlagInc;
        if (p >= 0) {
            do {
                s = status_load(&status[p]);
            } while ((s >> 62) == 0);
        }
        const uint64_t inc = ballot((s & ~kValMask) == kFlagInc);
        const int stop = inc ? __builtin_ctzll(inc) : kWave - 1;
        prefix += wave_sum_u64(lane() <= stop ? (s & kValMask) : 0ull);
        if (inc) return prefix;
    }
}

// Called by every lane of one wavefront: publishes the aggregate, looks
// back and publishes the inclusive prefix; returns the exclusive prefix of
// workgroup b (in every lane).
__device__ __forceinline__ uint64_t publish_and_look_back(uint64_t* status, int64_t b, uint64_t agg) {
    if (b == 0) {
        if (lane() == 0) status_store(&status[0], kFlagInc | agg);
        return 0;
    }
    if (lane() == 0) status_store(&status[b], kFlagAgg | agg);
    const uint64_t prefix = look_back(status, b);
    if (lane() == 0) status_store(&status[b], kFlagInc | ((prefix + agg) & kValMask));
    return prefix;
}

// Exclusive scan of one uint64 per thread across the workgroup; *total
// receives the sum. Ends with a barrier, so lds is reusable.
template <int NT = kThreads>
__device__ __forceinline__ uint64_t block_excl_u64(uint64_t v, uint64_t* lds, uint64_t* total) {
    constexpr int NW = NT / kWave;
    const int w = threadIdx.x / kWave, l = lane();
    uint64_t inc = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t lo = shfl_up_u32((uint32_t)inc, d), hi = shfl_up_u32((uint32_t)(inc >> 32), d);
        if (l >= d) inc += ((uint64_t)hi << 32) | lo;
    }
    if (l == kWave - 1) lds[w] = inc;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const uint64_t t = lds[i];
        before += i < w ? t : 0ull;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// ---- entry-emission scan ---------------------------------------------------
// Per Gaussian: x = number of tiles (entries), y = 1 if visible. Writes
// emit_off[g] (exclusive prefix of x), vis_ids[rank] = g for visible g, and
// counters[0] = M, counters[1] = V, counters[2] = M > capacity.
// Items are loaded and stored in coalesced rounds; in between they pass
// through LDS so that each thread scans kEmitRounds consecutive items and one
// workgroup scan of the packed pair (x << 24 | y; y <= kEmitPerBlock) serves
// both prefixes.

__global__ void __launch_bounds__(kEmitThreads) emit_scan_kernel(const uint4* __restrict__ info, int64_t n, int tiles_x,
                                                             int tiles_y, uint32_t* __restrict__ emit_off,
                                                             uint32_t* __restrict__ vis_ids, uint32_t* ticket,
                                                             uint64_t* status_x, uint64_t* status_y,
                                                             int64_t* __restrict__ counters, int64_t capacity) {
    static_assert(kEmitRounds % 4 == 0 && kEmitPerBlock < (1 << 24), "packed pair layout");
    __shared__ uint32_t tk;
    __shared__ __align__(16) uint32_t item_x[kEmitPerBlock];  // tile counts, then exclusive x
    __shared__ __align__(16) uint32_t item_y[kEmitPerBlock];  // exclusive y | visible << 31
    __shared__ uint64_t lds64[kEmitThreads / kWave];
    __shared__ uint64_t pre[2];
    if (threadIdx.x == 0) tk = atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t b = tk;
    const int64_t nb = gridDim.x;
    const int64_t base = b * kEmitPerBlock;
#pragma unroll
    for (int r = 0; r < kEmitRounds; ++r) {
        const int64_t g = base + r * kEmitThreads + threadIdx.x;
        int x0, y0, x1, y1;
        item_x[r * kEmitThreads + threadIdx.x] = g < n ? (uint32_t)rect_of(info[g], tiles_x, tiles_y, x0, y0, x1, y1) : 0u;
    }
    __syncthreads();
    constexpr int kVec = kEmitRounds / 4;
    const uint4* own = reinterpret_cast<const uint4*>(item_x) + kVec * threadIdx.x;
    uint32_t c[kEmitRounds];
#pragma unroll
    for (int q = 0; q < kVec; ++q) {
        const uint4 cq = own[q];
        c[4 * q] = cq.x;
        c[4 * q + 1] = cq.y;
        c[4 * q + 2] = cq.z;
        c[4 * q + 3] = cq.w;
    }
    uint32_t ex[kEmitRounds], ey[kEmitRounds];
    uint64_t sx = 0;
    uint32_t sy = 0;
#pragma unroll
    for (int i = 0; i < kEmitRounds; ++i) {
        ex[i] = (uint32_t)sx;
        ey[i] = sy;
        sx += c[i];
        sy += c[i] ? 1u : 0u;
    }
    uint64_t tot;
    const uint64_t tex = block_excl_u64<kEmitThreads>((sx << 24) | sy, lds64, &tot);
    const uint64_t ax = tot >> 24;
    const uint32_t ay = (uint32_t)(tot & 0xFFFFFFu);
    const uint32_t tx0 = (uint32_t)(tex >> 24), ty0 = (uint32_t)(tex & 0xFFFFFFu);
    uint4* own_x = reinterpret_cast<uint4*>(item_x) + kVec * threadIdx.x;
    uint4* own_y = reinterpret_cast<uint4*>(item_y) + kVec * threadIdx.x;
    auto vy = [&](int i) { return (ty0 + ey[i]) | (c[i] ? 0x80000000u : 0u); };
#pragma unroll
    for (int q = 0; q < kVec; ++q) {
        own_x[q] = make_uint4(tx0 + ex[4 * q], tx0 + ex[4 * q + 1], tx0 + ex[4 * q + 2], tx0 + ex[4 * q + 3]);
        own_y[q] = make_uint4(vy(4 * q), vy(4 * q + 1), vy(4 * q + 2), vy(4 * q + 3));
    }
    if (threadIdx.x < kWave) {
        const uint64_t px = publish_and_look_back(status_x, b, ax);
        if (threadIdx.x == 0) pre[0] = px;
    } else if (threadIdx.x < 2 * kWave) {
        const uint64_t py = publish_and_look_back(status_y, b, ay);
        if (threadIdx.x == kWave) pre[1] = py;
    }
    __syncthreads();
    const uint64_t cx = pre[0];
    const uint32_t cy = (uint32_t)pre[1];
    if (b == nb - 1 && threadIdx.x == 0) {
        counters[0] = (int64_t)(cx + ax);
        counters[1] = (int64_t)(cy + ay);
        counters[2] = (int64_t)(cx + ax) > capacity ? 1 : 0;
        counters[3] = 0;
    }
#pragma unroll
    for (int r = 0; r < kEmitRounds; ++r) {
        const int64_t g = base + r * kEmitThreads + threadIdx.x;
        if (g < n) {
            const int i = r * kEmitThreads + threadIdx.x;
            emit_off[g] = (uint32_t)(cx + item_x[i]);
            const uint32_t y = item_y[i];
            if (y >> 31) vis_ids[cy + (y & 0x7FFFFFFFu)] = (uint32_t)g;
        }
    }
}

// ---- bin offsets from the per-XCD count copies ---------------------------

__host__ __device__ __forceinline__ int64_t blocks_for(int64_t n) {
    const int64_t b = (n + kPerBlock - 1) / kPerBlock;
    return b > 0 ? b : 1;
}

// Appends value(r) of the items with bk[r] >= 0 (one per thread and round)
// to the list of their repair bucket: aggregated per wavefront and per
// workgroup, one global atomic per bucket and workgroup. lcount / lbase: LDS
// [kBuckets], lcount zeroed before the first round.
template <int R, int NT, class E, class V>
__device__ __forceinline__ void queue_values(const int (&bk)[R], V&& value, int64_t list_stride, uint32_t* lcount,
                                             uint32_t* lbase, E* __restrict__ lists,
                                             uint32_t* __restrict__ bucket_count) {
    uint32_t slot[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        slot[r] = 0;
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
    for (int r = 0; r < R; ++r) {
        if (bk[r] < 0) continue;
        lists[(int64_t)bk[r] * list_stride + lbase[bk[r]] + slot[r]] = value(r);
    }
}

// The same with the segment ids base + r NT + threadIdx.x as the values.
template <int R, int NT = kThreads>
__device__ __forceinline__ void queue_segments(const int (&bk)[R], int64_t base, int64_t list_stride,
                                               uint32_t* lcount, uint32_t* lbase, uint32_t* __restrict__ lists,
                                               uint32_t* __restrict__ bucket_count) {
    queue_values<R, NT>(
        bk, [&](int r) { return (uint32_t)(base + r * NT + threadIdx.x); }, list_stride, lcount, lbase, lists,
        bucket_count);
}

// bin_off[s] = exclusive prefix of the summed copies (bin_off[nseg] = M);
// count[x][s] becomes bin_off[s] + the counts of copies 0..x-1 in segment
// s. With queue_all, every segment with two or more entries is appended to
// the list of its repair bucket and its entries are added to counters[3];
// nothing is queued when the stream overflowed (counters[2]). repaired[s]
// (optional) records whether segment s was queued. With nseg_dev, the
// number of segments (and the stride of the count copies) is *nseg_dev and
// the grid is sized for its upper bound: workgroups past the last needed one
// leave after their ticket.
__global__ void __launch_bounds__(kThreads) bin_offsets_kernel(uint32_t* __restrict__ count, int64_t nseg_max,
                                                               const uint32_t* __restrict__ nseg_dev,
                                                               uint32_t* __restrict__ bin_off, uint32_t* ticket,
                                                               uint64_t* status, uint32_t* __restrict__ lists,
                                                               uint32_t* __restrict__ bucket_count,
                                                               int64_t* __restrict__ counters, bool queue_all,
                                                               uint8_t* __restrict__ repaired) {
    __shared__ uint32_t tk;
    __shared__ uint32_t lds32[kThreads / kWave];
    __shared__ uint64_t pre;
    __shared__ uint32_t lcount[kBuckets], lbase[kBuckets];
    __shared__ __align__(16) uint32_t tots[kPerBlock];  // segment totals, then block-exclusive prefixes
    if (threadIdx.x == 0) tk = atomicAdd(ticket, 1u);
    if (threadIdx.x < kBuckets) lcount[threadIdx.x] = 0;
    __syncthreads();
    const int64_t b = tk;
    const int64_t nseg = nseg_dev ? (int64_t)*nseg_dev : nseg_max;
    const int64_t nb = blocks_for(nseg);
    if (b >= nb) return;
    const int64_t base = b * kPerBlock;
    const bool queue = queue_all && counters[2] == 0;
    // the copies' counts stay in registers for the base pass below
    uint32_t cv[kRounds][kCopies];
    uint32_t v[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t sg = base + r * kThreads + threadIdx.x;
        v[r] = 0;
#pragma unroll
        for (int x = 0; x < kCopies; ++x) {
            cv[r][x] = sg < nseg ? count[(int64_t)x * nseg + sg] : 0u;
            v[r] += cv[r][x];
        }
        tots[r * kThreads + threadIdx.x] = v[r];
    }
    __syncthreads();
    // each thread scans kRounds consecutive segment totals
    uint4* own = reinterpret_cast<uint4*>(tots) + 2 * threadIdx.x;
    const uint4 t0 = own[0], t1 = own[1];
    const uint32_t c[kRounds] = {t0.x, t0.y, t0.z, t0.w, t1.x, t1.y, t1.z, t1.w};
    uint32_t ex[kRounds], s = 0;
#pragma unroll
    for (int i = 0; i < kRounds; ++i) {
        ex[i] = s;
        s += c[i];
    }
    uint32_t agg;
    const uint32_t tex = block_excl_u32(s, lds32, &agg);
    own[0] = make_uint4(tex + ex[0], tex + ex[1], tex + ex[2], tex + ex[3]);
    own[1] = make_uint4(tex + ex[4], tex + ex[5], tex + ex[6], tex + ex[7]);
    if (threadIdx.x < kWave) {
        const uint64_t pv = publish_and_look_back(status, b, agg);
        if (threadIdx.x == 0) pre = pv;
    }
    __syncthreads();
    const uint32_t carry = (uint32_t)pre;
    if (b == nb - 1 && threadIdx.x == 0) bin_off[nseg] = carry + agg;
    int bk[kRounds];
    uint32_t queued = 0;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t sg = base + r * kThreads + threadIdx.x;
        uint32_t run = carry + tots[r * kThreads + threadIdx.x];
        bk[r] = -1;
        if (sg < nseg) {
            bin_off[sg] = run;
#pragma unroll
            for (int x = 0; x < kCopies; ++x) {
                count[(int64_t)x * nseg + sg] = run;
                run += cv[r][x];
            }
            if (queue) bk[r] = bucket_of(v[r]);
            if (repaired) repaired[sg] = bk[r] >= 0 ? 1 : 0;
            if (bk[r] >= 0) queued += v[r];
        }
    }
    if (!queue) return;
    queue_segments(bk, base, nseg_max, lcount, lbase, lists, bucket_count);
    const uint32_t qsum = block_sum_u32(queued, lds32);
    if (threadIdx.x == 0 && qsum)
        atomicAdd(reinterpret_cast<unsigned long long*>(&counters[3]), (unsigned long long)qsum);
}

// ---- rule-based repair selection -------------------------------------------
// Table "Exact-repair selection rules" and the supplement's Algorithm
// "Selective repair selection and local exact sorting": a segment of length
// l >= 2, bin b, in a tile of l_tile entries is kept when l >= 320, l > 512,
// 100 l >= 45 l_tile, 129 <= l <= 256 and 100 l >= 10 l_tile, or b < 2 and
// l >= 16; kept segments are selected in (tile, bin) order while the
// selected entries fit the budget B (first fit). Kept length of segment q
// (0 when not kept or past the end).
__device__ __forceinline__ uint32_t kept_length(const uint32_t* __restrict__ bin_off, int64_t q, int K,
                                                int64_t nseg) {
    if (q >= nseg) return 0u;
    const int64_t t = q / K;
    const int b = (int)(q - t * K);
    const uint32_t len = bin_off[q + 1] - bin_off[q];
    if (len <= 1) return 0u;
    const uint64_t tl = bin_off[t * K + K] - bin_off[t * K];
    const uint64_t l100 = 100ull * len;
    const bool keep = len >= 320u || len > 512u || l100 >= 45ull * tl || (len >= 129u && len <= 256u && l100 >= 10ull * tl) ||
                      (b < 2 && len >= 16u);
    return keep ? len : 0u;
}

__device__ __forceinline__ uint64_t budget_of(float frac, uint32_t M) {
    return (uint64_t)floor((double)frac * (double)M);
}

// Pass 1: prefix of the kept lengths by a single-pass scan. A kept segment
// whose inclusive prefix is within B is selected (all kept segments before
// it were selected and fit). The one kept segment whose prefix first
// exceeds B is rejected; it leaves ctl = {its index + 1, B - the exclusive
// prefix} for the sequential continuation. When everything fits,
// counters[3] = the kept total.
__global__ void __launch_bounds__(kThreads) select_prefix_kernel(const uint32_t* __restrict__ bin_off, int64_t nseg,
                                                                 int K, float budget, uint32_t* ticket,
                                                                 uint64_t* status, uint32_t* __restrict__ ctl,
                                                                 uint32_t* __restrict__ lists,
                                                                 uint32_t* __restrict__ bucket_count,
                                                                 int64_t* __restrict__ counters,
                                                                 uint8_t* __restrict__ repaired) {
    __shared__ uint32_t tk;
    __shared__ uint32_t lds32[kThreads / kWave];
    __shared__ uint64_t pre;
    __shared__ uint32_t lcount[kBuckets], lbase[kBuckets];
    if (threadIdx.x == 0) tk = atomicAdd(ticket, 1u);
    if (threadIdx.x < kBuckets) lcount[threadIdx.x] = 0;
    __syncthreads();
    const int64_t b = tk;
    const int64_t nb = blocks_for(nseg);
    if (b >= nb) return;
    const int64_t base = b * kPerBlock;
    const bool queue = counters[2] == 0;
    const uint64_t B = budget_of(budget, bin_off[nseg]);
    uint32_t v[kRounds];
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        v[r] = kept_length(bin_off, base + r * kThreads + threadIdx.x, K, nseg);
        s += v[r];
    }
    const uint32_t agg = block_sum_u32(s, lds32);
    if (threadIdx.x < kWave) {
        const uint64_t pv = publish_and_look_back(status, b, agg);
        if (threadIdx.x == 0) pre = pv;
    }
    __syncthreads();
    uint64_t carry = pre;
    if (b == nb - 1 && threadIdx.x == 0 && carry + agg <= B) counters[3] = (int64_t)(carry + agg);
    int bk[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t sg = base + r * kThreads + threadIdx.x;
        uint32_t tot;
        const uint64_t excl = carry + block_excl_u32(v[r], lds32, &tot);
        carry += tot;
        const uint64_t incl = excl + v[r];
        const bool sel = v[r] != 0 && incl <= B;
        if (v[r] != 0 && incl > B && excl <= B) {
            ctl[0] = (uint32_t)(sg + 1);
            ctl[1] = (uint32_t)(B - excl);
        }
        if (repaired && sg < nseg) repaired[sg] = sel ? 1 : 0;
        bk[r] = queue && sel ? bucket_of(v[r]) : -1;
    }
    queue_segments(bk, base, nseg, lcount, lbase, lists, bucket_count);
}

constexpr int kTailThreads = 1024;

// Exclusive scan over a workgroup of kTailThreads; *total gets the sum.
// Ends with a barrier.
__device__ __forceinline__ uint32_t tail_excl_u32(uint32_t v, uint32_t* lds, uint32_t* total) {
    constexpr int NW = kTailThreads / kWave;
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

// Pass 2 (one workgroup): first fit over the segments after the first
// rejected one, with the remaining budget R, 1024 segments at a time. In a
// chunk, candidates are the kept segments with length <= R; the longest run
// of candidates whose running sum fits R is selected, the candidate that
// ends it is rejected, R drops by the run's sum and the candidates after it
// are filtered against the new R, until none is left. Stops once R < 2 (a
// kept segment has two or more entries). counters[3] = B - R at the end.
__global__ void __launch_bounds__(kTailThreads) select_tail_kernel(const uint32_t* __restrict__ bin_off,
                                                                   int64_t nseg, int K, float budget,
                                                                   const uint32_t* __restrict__ ctl,
                                                                   uint32_t* __restrict__ lists,
                                                                   uint32_t* __restrict__ bucket_count,
                                                                   int64_t* __restrict__ counters,
                                                                   uint8_t* __restrict__ repaired) {
    __shared__ uint32_t lds[kTailThreads / kWave];
    __shared__ uint32_t first, rem;
    if (ctl[0] == 0 || counters[2] != 0) return;
    const uint64_t B = budget_of(budget, bin_off[nseg]);
    uint32_t R = ctl[1];
    for (int64_t base = ctl[0]; base < nseg && R >= 2u; base += kTailThreads) {
        const int64_t q = base + threadIdx.x;
        const uint32_t kl = kept_length(bin_off, q, K, nseg);
        bool cand = kl != 0u && kl <= R;
        bool sel = false;
        while (__syncthreads_or(cand)) {
            uint32_t tot;
            const uint32_t excl = tail_excl_u32(cand ? kl : 0u, lds, &tot);
            if (threadIdx.x == 0) first = 0xFFFFFFFFu;
            __syncthreads();
            if (cand && excl + kl > R) atomicMin(&first, (uint32_t)threadIdx.x);
            __syncthreads();
            const uint32_t f = first;
            if (f == 0xFFFFFFFFu) {
                sel = sel || cand;
                cand = false;
                R -= tot;
            } else {
                if (threadIdx.x == f) rem = R - excl;
                __syncthreads();
                if (cand && threadIdx.x < f) sel = true;
                if (threadIdx.x <= f) cand = false;
                R = rem;
                cand = cand && kl <= R;
            }
        }
        if (sel) {
            if (repaired) repaired[q] = 1;
            const int bk = bucket_of(kl);
            const uint32_t at = atomicAdd(&bucket_count[bk], 1u);
            lists[(int64_t)bk * nseg + at] = (uint32_t)q;
        }
    }
    if (threadIdx.x == 0) counters[3] = (int64_t)(B - R);
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
    if (threadIdx.x < kWave) {
        const uint64_t pv = publish_and_look_back(status, b, agg);
        if (threadIdx.x == 0) pre = pv;
    }
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

// ---- grouped binning: group prefix and per-group counting sort ---------------

// group_off[g] = exclusive prefix of gcount over g < G, group_off[G] = total
// (one workgroup; G <= kMaxGroups = 8 per thread), and order[0 .. G) = the
// groups by decreasing floor(log2(count)) (empty groups last; arbitrary
// inside a class), so that the group sort starts the longest groups first.
__global__ void __launch_bounds__(kTailThreads) group_scan_kernel(const uint32_t* __restrict__ gcount, GroupMap gm,
                                                                  uint32_t* __restrict__ group_off,
                                                                  uint32_t* __restrict__ order) {
    const int G = gm.G;
    // per-tile bin counts: each group's first segment, segment count and the
    // most sub-bins (up to SB) whose codes fit the group sort's counters
    if (gm.seg_base) {
        for (int g = threadIdx.x; g < G; g += kTailThreads) {
            const int64_t t0 = (int64_t)g * gm.GT, t1 = min(t0 + gm.GT, gm.T);
            const uint32_t first = gm.seg_base[t0], segs = gm.seg_base[t1] - first;
            uint32_t lg = 0;
            while ((2u << lg) <= (uint32_t)gm.SB && (uint64_t)segs << (lg + 1) <= (uint64_t)kMaxGroupSegs) ++lg;
            gm.ginfo[g] = make_uint4(first, segs, lg, 0u);
        }
    }
    static_assert(kMaxGroups <= 8 * kTailThreads, "eight groups per thread");
    constexpr int kClasses = 33;  // class 31 - floor(log2 count) for count > 0, 32 for empty
    __shared__ uint32_t lds[kTailThreads / kWave];
    __shared__ uint32_t chist[kClasses], cbase[kClasses];
    if (threadIdx.x < kClasses) chist[threadIdx.x] = 0;
    const int i0 = 8 * threadIdx.x;
    uint32_t v[8], s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        v[j] = i0 + j < G ? gcount[i0 + j] : 0u;
        s += v[j];
    }
    uint32_t total;
    uint32_t run = tail_excl_u32(s, lds, &total);  // ends with a barrier: chist is cleared
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (i0 + j < G) {
            group_off[i0 + j] = run;
            atomicAdd(&chist[v[j] ? __builtin_clz(v[j]) : 32], 1u);
        }
        run += v[j];
    }
    if (threadIdx.x == 0) group_off[G] = total;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = 0;
        for (int c = 0; c < kClasses; ++c) {
            cbase[c] = b;
            b += chist[c];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (i0 + j < G) order[atomicAdd(&cbase[v[j] ? __builtin_clz(v[j]) : 32], 1u)] = (uint32_t)(i0 + j);
}

#ifndef TGS_SORT_THREADS
#define TGS_SORT_THREADS 512
#endif
#ifndef TGS_SORT_BATCH
#define TGS_SORT_BATCH (8192 / TGS_SORT_THREADS)
#endif
#ifndef TGS_SORT_WAVES_PER_EU
#define TGS_SORT_WAVES_PER_EU 0
#endif
#if TGS_SORT_WAVES_PER_EU > 0
#define TGS_SORT_ATTR __attribute__((amdgpu_waves_per_eu(TGS_SORT_WAVES_PER_EU, TGS_SORT_WAVES_PER_EU)))
#else
#define TGS_SORT_ATTR
#endif
constexpr int kSortThreads = TGS_SORT_THREADS;  // threads of a group-sort workgroup
constexpr int kSortBatch = TGS_SORT_BATCH;      // entries per thread and sweep step, loaded before any is used
constexpr int kTileBuckets = 33;                  // tile order buckets: bit lengths 32 .. 0 of the entry count

// Staging of the group sort's output when the lists hold sub-segment
// descriptors (SB > 1: exact repair, no records) and the group has at most
// kStage entries: they are placed at their code offsets in LDS, each
// sub-segment of 2..kRankMax entries is put in pair order there (an entry's
// rank among its sub-segment's pairs, ties by slot), and the group is
// written out in order: the output is written in runs instead of one
// scattered 8-byte store per entry, and the short sub-segments need no
// repair pass.
#ifndef TGS_RANK_MAX
#define TGS_RANK_MAX 128
#endif
#ifndef TGS_STAGE
#define TGS_STAGE 4096
#endif
constexpr int kStage = TGS_STAGE;
constexpr int kRankMax = TGS_RANK_MAX;

// One workgroup per group: its entries [group_off[g], group_off[g + 1])
// (clipped to the capacity) are counted per code (segment, or sub-segment
// when SB > 1) in LDS, the code offsets follow by a workgroup scan, and a
// second sweep places every entry at its code offset + an LDS rank (staged
// as above when SB > 1). Also writes bin_off for the group's segments,
// queues the repair segments (as bin_offsets_kernel; sub-segments as
// {begin, length} when SB > 1, without those the staging ordered), and
// writes the records of single-entry segments.
__global__ void __launch_bounds__(kSortThreads) TGS_SORT_ATTR group_sort_kernel(
    const uint64_t* __restrict__ tmp_pair, const uint16_t* __restrict__ tmp_code, const uint32_t* __restrict__ group_off,
    const uint32_t* __restrict__ order, GroupMap gm, int64_t nseg, int64_t capacity, uint64_t* __restrict__ pairs,
    uint32_t* __restrict__ bin_off, uint32_t* __restrict__ lists, int64_t list_stride,
    uint32_t* __restrict__ bucket_count, int64_t* __restrict__ counters, bool queue_all, uint8_t* __restrict__ repaired,
    RecordSink rs, uint32_t* __restrict__ tile_hist) {
    constexpr int NT = kSortThreads;
    constexpr int kMaxPer = kMaxGroupSegs / NT;
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    __shared__ uint32_t hist[kMaxGroupSegs];
    __shared__ uint32_t cur[kMaxGroupSegs];
    __shared__ uint32_t lds32[NT / kWave];
    __shared__ uint32_t lcount[kBuckets], lbase[kBuckets];
    __shared__ uint32_t thist[kTileBuckets];
    __shared__ uint64_t stage[kStage];
    __shared__ uint16_t scode[kStage];
    const int g = (int)order[blockIdx.x];
    const int64_t cap = capacity;
    const uint32_t lo = (uint32_t)min((int64_t)group_off[g], cap);
    const uint32_t hi = (uint32_t)min((int64_t)group_off[g + 1], cap);
    // the group's segments [sbase, sbase + segs), sub-bins SB, codes segs SB
    int64_t sbase, segs;
    int SB;
    if (gm.seg_base) {
        const uint4 gi = gm.ginfo[g];
        sbase = gi.x;
        segs = gi.y;
        SB = 1 << gi.z;
        nseg = gm.seg_base[gm.T];
    } else {
        sbase = (int64_t)g * gm.GS;
        segs = min((int64_t)gm.GS, nseg - sbase);
        SB = gm.SB;
    }
    const int codes = (int)(segs * SB);
    const int per = (codes + NT - 1) / NT;  // codes per thread, <= kMaxPer
    for (int c = threadIdx.x; c < per * NT; c += NT) hist[c] = 0;
    if (threadIdx.x < kBuckets) lcount[threadIdx.x] = 0;
    if (threadIdx.x < kTileBuckets) thist[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t base = lo; base < hi; base += NT * kSortBatch) {
        uint32_t c[kSortBatch];
#pragma unroll
        for (int j = 0; j < kSortBatch; ++j) {
            const uint32_t e = base + (uint32_t)(j * NT) + threadIdx.x;
            c[j] = e < hi ? (uint32_t)tmp_code[e] : kNone;
        }
#pragma unroll
        for (int j = 0; j < kSortBatch; ++j)
            if (c[j] != kNone) atomicAdd(&hist[c[j]], 1u);
    }
    __syncthreads();
    // exclusive prefix of the code counts: thread i owns codes i per ..
    uint32_t ex[kMaxPer], sum = 0;
#pragma unroll
    for (int j = 0; j < kMaxPer; ++j) {
        ex[j] = sum;
        if (j < per) sum += hist[threadIdx.x * per + j];
    }
    uint32_t agg;
    const uint32_t tex = block_excl_u32<NT>(sum, lds32, &agg);
#pragma unroll
    for (int j = 0; j < kMaxPer; ++j)
        if (j < per) cur[threadIdx.x * per + j] = tex + ex[j];
    __syncthreads();
    if (tile_hist) {
        // entries per tile of the group (tiles g GT ..): difference of the
        // exclusive prefixes at the tiles' first codes, as the bin offsets
        // will give them; bucket = bit length of the count
        const int64_t t0 = (int64_t)g * gm.GT, t1 = min(t0 + gm.GT, (int64_t)gm.T);
        auto first_code = [&](int64_t t) -> uint32_t {
            if (t >= t1) return hi - lo;
            const int64_t c = gm.seg_base ? ((int64_t)gm.seg_base[t] - sbase) * SB : (t - t0) * gm.K * SB;
            return c < codes ? cur[c] : hi - lo;
        };
        for (int64_t t = t0 + threadIdx.x; t < t1; t += NT) {
            const uint32_t cnt = first_code(t + 1) - first_code(t);
            atomicAdd(&thist[cnt ? __builtin_clz(cnt) : 32], 1u);
        }
    }
    const bool queue = queue_all && counters[2] == 0;
    const int64_t cbase = sbase * gm.SB;  // id of the group's first code
    const uint32_t n = hi - lo;
    const bool staged = gm.SB > 1 && n <= (uint32_t)kStage;
    // sub-segments the staging puts in order (none with an overflow)
    const uint32_t local_max = staged && queue ? (uint32_t)kRankMax : 1u;
    // repair queues per code (segments when SB == 1, sub-segments otherwise)
    int bk[kMaxPer];
#pragma unroll
    for (int r = 0; r < kMaxPer; ++r) {
        const int c = r * NT + threadIdx.x;
        bk[r] = -1;
        if (r < per && c < codes) {
            if (queue && hist[c] > local_max) bk[r] = bucket_of(hist[c]);
        }
    }
    // offsets, repair flags and repaired entries per segment
    uint32_t queued = 0;
    for (int c = threadIdx.x; c < segs; c += NT) {
        const int64_t sg = sbase + c;
        uint32_t len = 0;
        for (int k = 0; k < SB; ++k) len += hist[c * SB + k];
        bin_off[sg] = lo + cur[c * SB];
        const bool rep = queue && len >= 2;
        if (repaired) repaired[sg] = rep ? 1 : 0;
        if (rep) queued += len;
    }
    if (g == gm.G - 1 && threadIdx.x == 0) bin_off[nseg] = hi;
    if (gm.SB > 1)
        // sub-segments are queued as {begin, length}: the repair needs no offset lookup
        queue_values<kMaxPer, NT>(
            bk,
            [&](int r) {
                const int c = r * NT + threadIdx.x;
                return make_uint2(lo + cur[c], hist[c]);
            },
            list_stride, lcount, lbase, reinterpret_cast<uint2*>(lists), bucket_count);
    else
        queue_segments<kMaxPer, NT>(bk, cbase, list_stride, lcount, lbase, lists, bucket_count);
    if (queue) {
        const uint32_t qsum = block_sum_u32<NT>(queued, lds32);
        if (threadIdx.x == 0 && qsum)
            atomicAdd(reinterpret_cast<unsigned long long*>(&counters[3]), (unsigned long long)qsum);
    }
    if (staged) {
        // place at the code offsets in LDS ...
        for (uint32_t base = lo; base < hi; base += NT * kSortBatch) {
            uint32_t c[kSortBatch];
            uint64_t pr[kSortBatch];
#pragma unroll
            for (int j = 0; j < kSortBatch; ++j) {
                const uint32_t e = base + (uint32_t)(j * NT) + threadIdx.x;
                c[j] = kNone;
                pr[j] = 0;
                if (e < hi) {
                    c[j] = tmp_code[e];
                    pr[j] = tmp_pair[e];
                }
            }
#pragma unroll
            for (int j = 0; j < kSortBatch; ++j) {
                if (c[j] == kNone) continue;
                const uint32_t q = atomicAdd(&cur[c[j]], 1u);
                stage[q] = pr[j];
                scode[q] = (uint16_t)c[j];
            }
        }
        __syncthreads();
        // ... and write the group out in order, short sub-segments by rank
        for (uint32_t q = threadIdx.x; q < n; q += NT) {
            const uint32_t c = scode[q];
            const uint64_t v = stage[q];
            uint32_t out = q;
            const uint32_t len = hist[c];
            if (len >= 2 && len <= local_max) {
                // the code's slots are [cur - len, cur) once placed
                const uint32_t b = cur[c] - len;
                uint32_t rank = 0;
                for (uint32_t k = 0; k < len; ++k) {
                    const uint64_t x = stage[b + k];
                    rank += (x < v || (x == v && b + k < q)) ? 1u : 0u;
                }
                out = b + rank;
            }
            pairs[lo + out] = v;
        }
    } else {
        for (uint32_t base = lo; base < hi; base += NT * kSortBatch) {
            uint32_t c[kSortBatch];
            uint64_t pr[kSortBatch];
#pragma unroll
            for (int j = 0; j < kSortBatch; ++j) {
                const uint32_t e = base + (uint32_t)(j * NT) + threadIdx.x;
                c[j] = kNone;
                pr[j] = 0;
                if (e < hi) {
                    c[j] = tmp_code[e];
                    pr[j] = tmp_pair[e];
                }
            }
#pragma unroll
            for (int j = 0; j < kSortBatch; ++j) {
                if (c[j] == kNone) continue;
                const uint32_t p = lo + atomicAdd(&cur[c[j]], 1u);
                pairs[p] = pr[j];
                // records exist only with SB == 1, where a code is a segment
                if (rs.masks && hist[c[j]] == 1u) rs.put((uint32_t)(sbase + c[j]), p, pr[j]);
            }
        }
    }
    if (tile_hist) {
        __syncthreads();
        if (threadIdx.x < kTileBuckets && thist[threadIdx.x]) atomicAdd(&tile_hist[threadIdx.x], thist[threadIdx.x]);
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
    const int64_t blocks = n > 0 ? (n + kEmitPerBlock - 1) / kEmitPerBlock : 1;
    hipLaunchKernelGGL(emit_scan_kernel, dim3((unsigned)blocks), dim3(kEmitThreads), 0, s,
                       reinterpret_cast<const uint4*>(info), n, tiles_x, tiles_y, emit_off, vis_ids, ticket, status_x,
                       status_y, counters, capacity);
    return hipGetLastError();
}

hipError_t launch_bin_offsets(uint32_t* count, int64_t nseg, const uint32_t* nseg_dev, uint32_t* bin_off,
                              uint32_t* ticket, uint64_t* status, uint32_t* lists, uint32_t* bucket_count,
                              int64_t* counters, bool queue_all, uint8_t* repaired, hipStream_t s) {
    hipLaunchKernelGGL(bin_offsets_kernel, dim3((unsigned)scan_blocks(nseg)), dim3(kThreads), 0, s, count, nseg,
                       nseg_dev, bin_off, ticket, status, lists, bucket_count, counters, queue_all, repaired);
    return hipGetLastError();
}

hipError_t launch_repair_select(const uint32_t* bin_off, int64_t T, int K, float budget, uint32_t* ticket,
                                uint64_t* status, uint32_t* ctl, uint32_t* lists, uint32_t* bucket_count,
                                int64_t* counters, uint8_t* repaired, hipStream_t s) {
    const int64_t nseg = T * K;
    if (nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(select_prefix_kernel, dim3((unsigned)scan_blocks(nseg)), dim3(kThreads), 0, s, bin_off, nseg,
                       K, budget, ticket, status, ctl, lists, bucket_count, counters, repaired);
    hipLaunchKernelGGL(select_tail_kernel, dim3(1), dim3(kTailThreads), 0, s, bin_off, nseg, K, budget, ctl, lists,
                       bucket_count, counters, repaired);
    return hipGetLastError();
}

hipError_t launch_group_scan(const uint32_t* gcount, GroupMap gm, uint32_t* group_off, uint32_t* order,
                             hipStream_t s) {
    hipLaunchKernelGGL(group_scan_kernel, dim3(1), dim3(kTailThreads), 0, s, gcount, gm, group_off, order);
    return hipGetLastError();
}

hipError_t launch_group_sort(const uint64_t* tmp_pair, const uint16_t* tmp_code, const uint32_t* group_off,
                             const uint32_t* order, GroupMap gm, int64_t nseg, int64_t capacity, uint64_t* pairs, uint32_t* bin_off,
                             uint32_t* lists, int64_t list_stride, uint32_t* bucket_count,
                             int64_t* counters, bool queue_all, uint8_t* repaired, RecordSink rs,
                             uint32_t* tile_hist, hipStream_t s) {
    hipLaunchKernelGGL(group_sort_kernel, dim3((unsigned)gm.G), dim3(kSortThreads), 0, s, tmp_pair, tmp_code, group_off, order, gm,
                       nseg, capacity, pairs, bin_off, lists, list_stride, bucket_count, counters, queue_all, repaired,
                       rs, tile_hist);
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
