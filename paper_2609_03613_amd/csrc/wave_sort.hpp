// Wavefront sorting networks over 64-bit keys (unique keys; the maximum key
// pads): used by the repair sorts of the (tile, bin) segments.
#pragma once

#include "common.hpp"

namespace tgs {

// The value of lane l ^ m (m a power of two below 64, a constant after
// unrolling). Distances 1, 2, 4 and 8 stay inside a row of 16 lanes and use
// DPP moves (ALU, no LDS traffic): quad permutations for 1 and 2, a row
// rotation by 8 for 8, and for 4 a rotation by 4 or 12 chosen by lane bit 2.
// Larger distances use the LDS crossbar (ds_bpermute).
__device__ __forceinline__ uint32_t xor_lane_u32(uint32_t v, int m) {
    const int x = (int)v;
    switch (m) {
        case 1:
            return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
        case 2:
            return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
        case 4: {
            const int r4 = __builtin_amdgcn_mov_dpp(x, 0x124, 0xF, 0xF, true);   // row_ror:4
            const int r12 = __builtin_amdgcn_mov_dpp(x, 0x12C, 0xF, 0xF, true);  // row_ror:12
            return (uint32_t)((lane() & 4) ? r4 : r12);
        }
        case 8:
            return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, true);  // row_ror:8
        default:
            return shfl_xor_u32(v, m);
    }
}

__device__ __forceinline__ uint64_t xor_lane_u64(uint64_t v, int m) {
    const uint32_t lo = xor_lane_u32((uint32_t)v, m), hi = xor_lane_u32((uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// Bitonic network over groups of G lanes, one key per lane (the partner at
// distance j < G is lane l ^ j, inside the group).
template <int G>
__device__ __forceinline__ uint64_t group_bitonic(uint64_t v, int li) {
#pragma unroll
    for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            // the lower lane of an ascending pair keeps the smaller key, the
            // upper one the larger (descending: the reverse): keep the own
            // key exactly when (own < other) says the same
            const uint64_t o = xor_lane_u64(v, j);
            const bool keep_min = ((li & k) == 0) == ((li & j) == 0);
            v = ((v < o) == keep_min) ? v : o;
        }
    }
    return v;
}

// Segments of 65..512 keys: one wavefront, E = 2, 4 or 8 consecutive keys
// per lane in registers (key i = lane * E + k in register k, padded with
// the maximum key): bitonic network whose comparators at distance j < E
// stay inside a lane and at j >= E exchange register k with lane l ^ (j / E).
// REC: write the records of the sorted positions (rs.put).
template <int E, bool REC>
__device__ __forceinline__ void sort_wave_reg(uint64_t* __restrict__ seg, uint32_t s, uint32_t begin, uint32_t len,
                                              const RecordSink& rs) {
    const int l = lane();
    uint64_t v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t i = (uint32_t)(l * E + k);
        v[k] = i < len ? seg[i] : ~0ull;
    }
#pragma unroll
    for (int kk = 2; kk <= E * kWave; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j < E) {
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    if (k & j) continue;
                    const bool up = ((l * E + k) & kk) == 0;
                    const uint64_t a = v[k], b = v[k | j];
                    const bool sw = (a > b) == up;
                    v[k] = sw ? b : a;
                    v[k | j] = sw ? a : b;
                }
            } else {
                const int m = j / E;
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const uint64_t o = xor_lane_u64(v[k], m);
                    const bool keep_min = (((l * E + k) & kk) == 0) == ((l & m) == 0);
                    v[k] = ((v[k] < o) == keep_min) ? v[k] : o;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t i = (uint32_t)(l * E + k);
        if (i < len) {
            seg[i] = v[k];
            if (REC) rs.put(s, begin + i, v[k]);
        }
    }
}

// LDS slot of key i in the workgroup networks below: one pad slot after
// every E keys, so that the E-key runs of consecutive threads start in
// different banks.
template <int E>
__device__ __forceinline__ uint32_t block_slot(uint32_t i) {
    return i + i / E;
}

// Segments of 513..8192 keys: one workgroup of NT threads, E consecutive
// keys per thread in registers (key i = t E + k in register k of thread t,
// padded with the maximum key; P = NT E keys): the bitonic network with the
// comparators at distance j < E inside a thread, E <= j < 64 E between the
// lanes of a wavefront (lane l ^ j / E), and j >= 64 E between wavefronts
// through LDS (lds: block_slot<E>(P) slots). Only the last log2(NT / 64)
// merge levels cross wavefronts, so the network takes 2 barriers per
// cross-wavefront step instead of one per step.
template <int E, int NT>
__device__ __forceinline__ void sort_block_reg(uint64_t (&v)[E], uint64_t* lds) {
    const int t = (int)threadIdx.x, l = lane();
    constexpr int P = NT * E;
#pragma unroll
    for (int kk = 2; kk <= P; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j < E) {
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    if (k & j) continue;
                    const bool up = (((uint32_t)(t * E + k)) & (uint32_t)kk) == 0;
                    const uint64_t a = v[k], b = v[k | j];
                    const bool sw = (a > b) == up;
                    v[k] = sw ? b : a;
                    v[k | j] = sw ? a : b;
                }
            } else if (j < kWave * E) {
                const int m = j / E;
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const uint64_t o = xor_lane_u64(v[k], m);
                    const bool keep_min = ((((uint32_t)(t * E + k)) & (uint32_t)kk) == 0) == ((l & m) == 0);
                    v[k] = ((v[k] < o) == keep_min) ? v[k] : o;
                }
            } else {
#pragma unroll
                for (int k = 0; k < E; ++k) lds[block_slot<E>((uint32_t)(t * E + k))] = v[k];
                __syncthreads();
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const uint32_t i = (uint32_t)(t * E + k);
                    const uint64_t o = lds[block_slot<E>(i ^ (uint32_t)j)];
                    const bool keep_min = ((i & (uint32_t)kk) == 0) == ((i & (uint32_t)j) == 0);
                    v[k] = ((v[k] < o) == keep_min) ? v[k] : o;
                }
                __syncthreads();
            }
        }
    }
}

}  // namespace tgs
