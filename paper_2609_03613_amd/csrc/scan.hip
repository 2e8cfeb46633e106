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
constexpr int kRounds = 8;
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
        for (int x = 0; x < kCopies; ++x) t += count[(int64_t)x * nseg + s];
    return t;
}

// Appends the segments with bk >= 0 (one per thread and round) to the
// list of their repair bucket: aggregated per wavefront and per workgroup,
// one global atomic per bucket and workgroup. lcount / lbase: LDS [kBuckets],
// lcount zeroed before the first round.
template <int R>
__device__ __forceinline__ void queue_segments(const int (&bk)[R], int64_t base, int64_t list_stride,
                                               uint32_t* lcount, uint32_t* lbase, uint32_t* __restrict__ lists,
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
        const int64_t sg = base + r * kThreads + threadIdx.x;
        lists[(int64_t)bk[r] * list_stride + lbase[bk[r]] + slot[r]] = (uint32_t)sg;
    }
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
    if (threadIdx.x == 0) tk = atomicAdd(ticket, 1u);
    if (threadIdx.x < kBuckets) lcount[threadIdx.x] = 0;
    __syncthreads();
    const int64_t b = tk;
    const int64_t nseg = nseg_dev ? (int64_t)*nseg_dev : nseg_max;
    const int64_t nb = blocks_for(nseg);
    if (b >= nb) return;
    const int64_t base = b * kPerBlock;
    const bool queue = queue_all && counters[2] == 0;
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
    uint32_t queued = 0;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t sg = base + r * kThreads + threadIdx.x;
        uint32_t tot;
        uint32_t run = carry + block_excl_u32(v[r], lds32, &tot);
        carry += tot;
        bk[r] = -1;
        if (sg < nseg) {
            bin_off[sg] = run;
#pragma unroll
            for (int x = 0; x < kCopies; ++x) {
                uint32_t* c = count + (int64_t)x * nseg + sg;
                const uint32_t cv = *c;
                *c = run;
                run += cv;
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
    if (threadIdx.x == 0) pre = publish_and_look_back(status, b, agg);
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
