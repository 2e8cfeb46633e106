// Wavefront sorting networks over 64-bit keys (unique keys; the maximum key
// pads): used by the repair sorts of the (tile, bin) segments.
#pragma once

#include "common.hpp"

namespace tgs {

// Bitonic network over groups of G lanes, one key per lane (the partner at
// distance j < G is lane l ^ j, inside the group).
template <int G>
__device__ __forceinline__ uint64_t group_bitonic(uint64_t v, int li) {
#pragma unroll
    for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint64_t o = shfl_xor_u64(v, j);
            const bool up = (li & k) == 0, lower = (li & j) == 0;
            const uint64_t mn = v < o ? v : o, mx = v < o ? o : v;
            v = (lower == up) ? mn : mx;
        }
    }
    return v;
}

// Segments of 65..512 keys: one wavefront, E = 2, 4 or 8 keys per lane in
// registers (key i = k * 64 + lane in register k, padded with the maximum
// key): bitonic network whose comparators at distance j < 64 exchange keys
// across lanes and at j >= 64 between registers of the same lane.
template <int E>
__device__ __forceinline__ void sort_wave_reg(uint64_t* __restrict__ seg, uint32_t s, uint32_t begin, uint32_t len,
                                              const RecordSink& rs) {
    const int l = lane();
    uint64_t v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t i = (uint32_t)(k * kWave + l);
        v[k] = i < len ? seg[i] : ~0ull;
    }
#pragma unroll
    for (int kk = 2; kk <= E * kWave; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j >= kWave) {
                const int jr = j / kWave;
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    if (k & jr) continue;
                    const bool up = ((k * kWave) & kk) == 0;
                    const uint64_t a = v[k], b = v[k | jr];
                    const bool sw = (a > b) == up;
                    v[k] = sw ? b : a;
                    v[k | jr] = sw ? a : b;
                }
            } else {
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const uint64_t o = shfl_xor_u64(v[k], j);
                    const bool up = ((k * kWave + l) & kk) == 0, lower = (l & j) == 0;
                    const uint64_t mn = v[k] < o ? v[k] : o, mx = v[k] < o ? o : v[k];
                    v[k] = (lower == up) ? mn : mx;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t i = (uint32_t)(k * kWave + l);
        if (i < len) {
            seg[i] = v[k];
            rs.put(s, begin + i, v[k]);
        }
    }
}

}  // namespace tgs
