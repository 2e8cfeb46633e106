// Learned bin-count proposal: per-tile features of a frame's stream, a
// 16-64-64-8 ReLU network that picks each tile's bin count K_t = 2^(k+1),
// and its training step (expected-regret loss, backward, momentum SGD).
// The paper fixes K = 64 per tile (section "Implementation details") and
// studies K per frame (Table "Effect of depth-bin count"); exact repair
// keeps the image independent of K, so the network only moves time.
//
// Parameter vector (fp32, 5768 values, row-major): W1 [16][64], b1 [64],
// W2 [64][64], b2 [64], W3 [64][8], b3 [8].
//
// Kernels (lane = tile unless stated; weights staged in LDS):
//   features   one wavefront per tile reads its K_t bin lengths
//   forward    a1, a2, relu(a1), relu(a2) [T][64] (training) and logits
//              [T][8]; inference writes K_t (and optionally the logits)
//   softmax    p, dL/dz = p (r - p.r) / T and the loss
//   backward   dL/da2, dL/da1 [T][64]
//   wgrad      the weight gradients as sums over tiles: one lane per
//              weight and tile chunk, one float atomic per (weight, chunk)
//   sgd        v = mu v + g, w -= lr v, g = 0
#include <math.h>

#include "common.hpp"

namespace tgs {

namespace {

constexpr int kIn = 16, kH = 64, kOut = 8;
constexpr int kW1 = 0, kB1 = kW1 + kIn * kH, kW2 = kB1 + kH, kB2 = kW2 + kH * kH, kW3 = kB2 + kH,
              kB3 = kW3 + kH * kOut, kNumParams = kB3 + kOut;
static_assert(kNumParams == 5768, "parameter layout");

__device__ __forceinline__ void stage_weights(const float* __restrict__ w, float* s) {
    for (int i = threadIdx.x; i < kNumParams; i += blockDim.x) s[i] = w[i];
    __syncthreads();
}

// ---- features ----------------------------------------------------------------

// One wavefront per tile: lanes take the tile's bins 64 at a time
// (coalesced reads of the offsets), then wave reductions.
__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m, kWave);
    return v;
}
__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v = fmaxf(v, __shfl_xor(v, m, kWave));
    return v;
}

__global__ void __launch_bounds__(256) features_kernel(const uint32_t* __restrict__ offsets, SegMap sm, int64_t T,
                                                       const int64_t* __restrict__ counters,
                                                       float* __restrict__ feat) {
    const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (t >= T) return;
    const int l = lane();
    const uint32_t s0 = sm.first(t), s1 = sm.first(t + 1);
    const int K = (int)(s1 - s0);
    float hist[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float n = 0.f, mx = 0.f, nz = 0.f, rep = 0.f, sq = 0.f;
    for (int b = l; b < K; b += kWave) {
        const float len = (float)(offsets[s0 + b + 1] - offsets[s0 + b]);
        n += len;
        mx = fmaxf(mx, len);
        nz += len > 0.f ? 1.f : 0.f;
        rep += len >= 2.f ? len : 0.f;
        sq += len * len;
        if (K >= 8) {
            const int j = (8 * b) / K;
#pragma unroll
            for (int c = 0; c < 8; ++c) hist[c] += c == j ? len : 0.f;
        } else {
            const int c8 = 8 / K;
#pragma unroll
            for (int c = 0; c < 8; ++c) hist[c] += (c >= b * c8 && c < (b + 1) * c8) ? len / (float)c8 : 0.f;
        }
    }
    n = wave_sum_f(n);
    mx = wave_max_f(mx);
    nz = wave_sum_f(nz);
    rep = wave_sum_f(rep);
    sq = wave_sum_f(sq);
#pragma unroll
    for (int c = 0; c < 8; ++c) hist[c] = wave_sum_f(hist[c]);
    if (l != 0) return;
    const float d = fmaxf(n, 1.f);
    const float M = (float)counters[0];
    const float dens = log2f(1.f + M / (float)T);
    float* f = feat + t * 16;
    f[0] = log2f(1.f + n);
#pragma unroll
    for (int j = 0; j < 8; ++j) f[1 + j] = hist[j] / d;
    f[9] = log2f(1.f + mx);
    f[10] = nz / (float)K;
    f[11] = log2f((float)K) / 8.f;
    f[12] = rep / d;
    f[13] = log2f(1.f + sq / d);
    f[14] = dens;
    f[15] = f[0] - dens;
}

// ---- forward ----------------------------------------------------------------

// Forward of one tile's features x: a1, a2 (pre-activations) and logits z.
__device__ __forceinline__ void mlp_forward(const float* s, const float* x, float* a1, float* a2, float* z) {
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float acc = s[kB1 + j];
#pragma unroll
        for (int i = 0; i < kIn; ++i) acc = fmaf(x[i], s[kW1 + i * kH + j], acc);
        a1[j] = acc;
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float acc = s[kB2 + j];
#pragma unroll
        for (int i = 0; i < kH; ++i) acc = fmaf(fmaxf(a1[i], 0.f), s[kW2 + i * kH + j], acc);
        a2[j] = acc;
    }
#pragma unroll
    for (int k = 0; k < kOut; ++k) {
        float acc = s[kB3 + k];
#pragma unroll
        for (int i = 0; i < kH; ++i) acc = fmaf(fmaxf(a2[i], 0.f), s[kW3 + i * kOut + k], acc);
        z[k] = acc;
    }
}

// Inference: K_t = 2^(argmax z + 1) (the first maximum wins); a non-finite
// weight or logit gives the fallback count.
__global__ void __launch_bounds__(64) propose_kernel(const float* __restrict__ w, const float* __restrict__ feat,
                                                      int64_t T, int32_t* __restrict__ bins,
                                                      float* __restrict__ logits, int fallback) {
    __shared__ float s[kNumParams];
    int bad = 0;
    for (int i = threadIdx.x; i < kNumParams; i += blockDim.x) {
        s[i] = w[i];
        bad |= isfinite(s[i]) ? 0 : 1;
    }
    const bool invalid = __syncthreads_or(bad) != 0;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    if (invalid) {
        bins[t] = fallback;
        return;
    }
    float x[kIn], a1[kH], a2[kH], z[kOut];
#pragma unroll
    for (int i = 0; i < kIn; ++i) x[i] = feat[t * kIn + i];
    mlp_forward(s, x, a1, a2, z);
    int best = 0;
    float bestv = z[0];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < kOut; ++k) {
        ok = ok && isfinite(z[k]);
        if (z[k] > bestv) {
            bestv = z[k];
            best = k;
        }
    }
    if (logits)
#pragma unroll
        for (int k = 0; k < kOut; ++k) logits[t * kOut + k] = z[k];
    bins[t] = ok ? (1 << (best + 1)) : fallback;
}

// Training forward: stores a1, a2, relu(a1), relu(a2) and z.
__global__ void __launch_bounds__(256) train_forward_kernel(const float* __restrict__ w, const float* __restrict__ feat,
                                                            int64_t T, float* __restrict__ A1, float* __restrict__ A2,
                                                            float* __restrict__ H1, float* __restrict__ H2,
                                                            float* __restrict__ Z) {
    __shared__ float s[kNumParams];
    stage_weights(w, s);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    float x[kIn], a1[kH], a2[kH], z[kOut];
#pragma unroll
    for (int i = 0; i < kIn; ++i) x[i] = feat[t * kIn + i];
    mlp_forward(s, x, a1, a2, z);
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        A1[t * kH + j] = a1[j];
        A2[t * kH + j] = a2[j];
        H1[t * kH + j] = fmaxf(a1[j], 0.f);
        H2[t * kH + j] = fmaxf(a2[j], 0.f);
    }
#pragma unroll
    for (int k = 0; k < kOut; ++k) Z[t * kOut + k] = z[k];
}

// p = softmax(z), dL/dz = p (r - p.r) / T (in place over Z), loss += p.r / T.
__global__ void __launch_bounds__(256) softmax_kernel(float* __restrict__ Z, const float* __restrict__ regret, int64_t T,
                                                      float* __restrict__ loss) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float contrib = 0.f;
    if (t < T) {
        float z[kOut], r[kOut], mx = -INFINITY, sum = 0.f, pr = 0.f;
#pragma unroll
        for (int k = 0; k < kOut; ++k) {
            z[k] = Z[t * kOut + k];
            r[k] = regret[t * kOut + k];
            mx = fmaxf(mx, z[k]);
        }
#pragma unroll
        for (int k = 0; k < kOut; ++k) {
            z[k] = expf(z[k] - mx);
            sum += z[k];
        }
#pragma unroll
        for (int k = 0; k < kOut; ++k) {
            z[k] /= sum;
            pr = fmaf(z[k], r[k], pr);
        }
        const float inv = 1.f / (float)T;
#pragma unroll
        for (int k = 0; k < kOut; ++k) Z[t * kOut + k] = z[k] * (r[k] - pr) * inv;
        contrib = pr * inv;
    }
    // wave sum, one atomic per wavefront
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) contrib += __shfl_xor(contrib, m, kWave);
    if (loss && lane() == 0) atomicAdd(loss, contrib);
}

// dL/da2 = (dz W3^T) [a2 > 0], dL/da1 = (dL/da2 W2^T) [a1 > 0], in place over
// A2 and A1 (the pre-activation signs are read before they are replaced).
__global__ void __launch_bounds__(256) train_backward_kernel(const float* __restrict__ w, const float* __restrict__ DZ,
                                                             int64_t T, float* __restrict__ A1, float* __restrict__ A2) {
    __shared__ float s[kNumParams];
    stage_weights(w, s);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    float dz[kOut], da2[kH];
#pragma unroll
    for (int k = 0; k < kOut; ++k) dz[k] = DZ[t * kOut + k];
#pragma unroll
    for (int i = 0; i < kH; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < kOut; ++k) acc = fmaf(dz[k], s[kW3 + i * kOut + k], acc);
        da2[i] = A2[t * kH + i] > 0.f ? acc : 0.f;
        A2[t * kH + i] = da2[i];
    }
#pragma unroll
    for (int i = 0; i < kH; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < kH; ++j) acc = fmaf(da2[j], s[kW2 + i * kH + j], acc);
        const float a1 = A1[t * kH + i];
        A1[t * kH + i] = a1 > 0.f ? acc : 0.f;
    }
}

// Weight gradients as sums over tiles. Thread (p, chunk) adds, over the
// tiles of its chunk, the product that parameter p collects:
//   W1[i][j]: x_i da1_j   b1[j]: da1_j   W2[i][j]: relu(a1_i) da2_j
//   b2[j]: da2_j   W3[i][k]: relu(a2_i) dz_k   b3[k]: dz_k
constexpr int kChunk = 512;

__global__ void __launch_bounds__(256) wgrad_kernel(const float* __restrict__ feat,
                                                    const float* __restrict__ DA1, const float* __restrict__ DA2,
                                                    const float* __restrict__ DZ, const float* __restrict__ H1,
                                                    const float* __restrict__ H2, int64_t T, float* __restrict__ g) {
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= kNumParams) return;
    const int64_t t0 = (int64_t)blockIdx.y * kChunk, t1 = min(T, t0 + kChunk);
    float acc = 0.f;
    if (p < kB1) {
        const int i = p / kH, j = p % kH;
        for (int64_t t = t0; t < t1; ++t) acc = fmaf(feat[t * kIn + i], DA1[t * kH + j], acc);
    } else if (p < kW2) {
        const int j = p - kB1;
        for (int64_t t = t0; t < t1; ++t) acc += DA1[t * kH + j];
    } else if (p < kB2) {
        const int i = (p - kW2) / kH, j = (p - kW2) % kH;
        for (int64_t t = t0; t < t1; ++t) acc = fmaf(H1[t * kH + i], DA2[t * kH + j], acc);
    } else if (p < kW3) {
        const int j = p - kB2;
        for (int64_t t = t0; t < t1; ++t) acc += DA2[t * kH + j];
    } else if (p < kB3) {
        const int i = (p - kW3) / kOut, k = (p - kW3) % kOut;
        for (int64_t t = t0; t < t1; ++t) acc = fmaf(H2[t * kH + i], DZ[t * kOut + k], acc);
    } else {
        const int k = p - kB3;
        for (int64_t t = t0; t < t1; ++t) acc += DZ[t * kOut + k];
    }
    if (t1 > t0) atomicAdd(&g[p], acc);
}

__global__ void sgd_kernel(float* __restrict__ w, float* __restrict__ v, float* __restrict__ g, float lr, float mu) {
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= kNumParams) return;
    const float nv = fmaf(mu, v[p], g[p]);
    v[p] = nv;
    w[p] = fmaf(-lr, nv, w[p]);
    g[p] = 0.f;
}

__global__ void zero_kernel(float* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

unsigned grid_of(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int mlp_num_params() { return kNumParams; }

hipError_t launch_tile_features(const uint32_t* offsets, SegMap sm, int64_t T, const int64_t* counters, float* feat,
                                hipStream_t s) {
    if (T == 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel, dim3(grid_of(T * kWave, 256)), dim3(256), 0, s, offsets, sm, T, counters,
                       feat);
    return hipGetLastError();
}

hipError_t launch_propose(const float* w, const float* feat, int64_t T, int32_t* bins, float* logits, int fallback,
                          hipStream_t s) {
    if (T == 0) return hipSuccess;
    hipLaunchKernelGGL(propose_kernel, dim3(grid_of(T, kWave)), dim3(kWave), 0, s, w, feat, T, bins, logits, fallback);
    return hipGetLastError();
}

size_t mlp_train_workspace_floats(int64_t T) { return (size_t)kNumParams + 4 * (size_t)T * kH + (size_t)T * kOut; }

hipError_t launch_mlp_train_step(float* w, float* v, const float* feat, const float* regret, int64_t T, float lr,
                                 float mu, float* ws, float* loss, hipStream_t s) {
    float* g = ws;
    float* A1 = g + kNumParams;
    float* A2 = A1 + T * kH;
    float* H1 = A2 + T * kH;
    float* H2 = H1 + T * kH;
    float* Z = H2 + T * kH;
    hipLaunchKernelGGL(zero_kernel, dim3(grid_of(kNumParams, 256)), dim3(256), 0, s, g, (int64_t)kNumParams);
    if (loss) hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, loss, (int64_t)1);
    if (T > 0) {
        const unsigned gt = grid_of(T, 256);
        hipLaunchKernelGGL(train_forward_kernel, dim3(gt), dim3(256), 0, s, w, feat, T, A1, A2, H1, H2, Z);
        hipLaunchKernelGGL(softmax_kernel, dim3(gt), dim3(256), 0, s, Z, regret, T, loss);
        hipLaunchKernelGGL(train_backward_kernel, dim3(gt), dim3(256), 0, s, w, Z, T, A1, A2);
        hipLaunchKernelGGL(wgrad_kernel, dim3(grid_of(kNumParams, 256), grid_of(T, kChunk)), dim3(256), 0, s, feat,
                           A1, A2, Z, H1, H2, T, g);
    }
    hipLaunchKernelGGL(sgd_kernel, dim3(grid_of(kNumParams, 256)), dim3(256), 0, s, w, v, g, lr, mu);
    return hipGetLastError();
}

}  // namespace tgs
