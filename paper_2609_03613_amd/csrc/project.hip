// Projection of 3D Gaussians to screen-space splats (EWA splatting with the
// 3DGS conventions, which the paper keeps unchanged): camera transform,
// covariance R S^2 R^T, perspective Jacobian with the 3DGS frustum guard (1.3 x the half FOV),
// 0.3 px^2 dilation, conic, sigmoid opacity, real spherical-harmonic colour
// up to degree 3, and the opacity-aware tile rect.
//
// One lane per Gaussian. The arithmetic is binary64 (the projection reads
// 56-236 B per Gaussian and is bound by HBM, so the FP64 units cost nothing
// measurable) and is rounded once to the fp32 outputs; this keeps the
// projected records within one binary32 rounding of exact values.
#include <math.h>

#include "common.hpp"

namespace tgs {

Cam make_cam(const tgs_camera& c, int tile, int footprint) {
    Cam k;
    k.footprint = footprint;
    for (int i = 0; i < 9; ++i) k.R[i] = c.R[i];
    for (int i = 0; i < 3; ++i) k.t[i] = c.t[i];
    k.fx = c.fx; k.fy = c.fy; k.cx = c.cx; k.cy = c.cy;
    k.znear = c.znear; k.zfar = c.zfar;
    k.width = c.width; k.height = c.height;
    k.tile = tile;
    k.tiles_x = div_up(c.width, tile);
    k.tiles_y = div_up(c.height, tile);
    for (int i = 0; i < 3; ++i) k.campos[i] = -(c.R[i] * c.t[0] + c.R[3 + i] * c.t[1] + c.R[6 + i] * c.t[2]);
    // frustum guard: x/z is clamped to the image edge plus 0.3 tan(half
    // FOV), tan(half FOV) = W / (2 fx), i.e. +-1.3 W / (2 fx) when the
    // principal point is centred (and likewise for y)
    const double tanx = 0.5 * c.width / c.fx, tany = 0.5 * c.height / c.fy;
    k.lim_xp = (c.width - c.cx) / c.fx + 0.3 * tanx;
    k.lim_xn = c.cx / c.fx + 0.3 * tanx;
    k.lim_yp = (c.height - c.cy) / c.fy + 0.3 * tany;
    k.lim_yn = c.cy / c.fy + 0.3 * tany;
    return k;
}

// Real SH basis up to degree 3 at the unit direction (x, y, z), expanded as
// polynomials (Condon-Shortley phase), written to Y[l*l + l + m].
__device__ __forceinline__ void sh_basis(double x, double y, double z, int degree, double* Y) {
    Y[0] = 0.28209479177387814;
    if (degree < 1) return;
    const double c1 = 0.4886025119029199;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (degree < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 1.0925484305920792 * x * y;
    Y[5] = -1.0925484305920792 * y * z;
    Y[6] = 0.31539156525252005 * (2.0 * zz - xx - yy);
    Y[7] = -1.0925484305920792 * x * z;
    Y[8] = 0.5462742152960396 * (xx - yy);
    if (degree < 3) return;
    Y[9] = -0.5900435899266435 * y * (3.0 * xx - yy);
    Y[10] = 2.890611442640554 * x * y * z;
    Y[11] = -0.4570457994644658 * y * (4.0 * zz - xx - yy);
    Y[12] = 0.3731763325901154 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -0.4570457994644658 * x * (4.0 * zz - xx - yy);
    Y[14] = 1.445305721320277 * z * (xx - yy);
    Y[15] = -0.5900435899266435 * x * (xx - 3.0 * yy);
}

constexpr int kProjThreads = 128;
constexpr int kMaxShFloats = 16 * 3;
constexpr int kShSink = kProjThreads * kMaxShFloats / 4;  // LDS slot for the stores past the block's data

// Stages cnt floats at src (the SH block of the workgroup's Gaussians) into
// sh_lds [kShSink + 1] with coalesced 16-byte loads, all in flight at once;
// pre() issues the lane's other loads while they are. The loads use a
// clamped index and the stores go to the sink slot past cnt, so no load is
// made conditional (which would let the compiler move it next to its use).
// The caller synchronises before reading sh_lds.
template <class Pre>
__device__ __forceinline__ void stage_sh_block(float4* sh_lds, const float* __restrict__ src, int64_t cnt, Pre&& pre) {
    float* f = reinterpret_cast<float*>(sh_lds);
    if ((reinterpret_cast<uintptr_t>(src) & 15) == 0 && cnt >= 4) {
        constexpr int kVecPerThread = kMaxShFloats / 4;
        const float4* s4 = reinterpret_cast<const float4*>(src);
        const int cnt4 = (int)(cnt / 4);
        float4 v[kVecPerThread];
#pragma unroll
        for (int j = 0; j < kVecPerThread; ++j) {
            const int i = j * kProjThreads + (int)threadIdx.x;
            v[j] = s4[i < cnt4 ? i : cnt4 - 1];
        }
        pre();
#pragma unroll
        for (int j = 0; j < kVecPerThread; ++j) {
            const int i = j * kProjThreads + (int)threadIdx.x;
            sh_lds[i < cnt4 ? i : kShSink] = v[j];
        }
        for (int64_t i = (int64_t)cnt4 * 4 + threadIdx.x; i < cnt; i += kProjThreads) f[i] = src[i];
    } else {
        pre();
        for (int64_t i = threadIdx.x; i < cnt; i += kProjThreads) f[i] = src[i];
    }
}

// Every lane reads its Gaussian's parameters once and writes the splat and
// info lines of up to kProjViews cameras (views.nv of them).
//
// SH3: each lane loads its Gaussian's 48 coefficients itself (twelve
// 16-byte loads, no LDS), all issued before the first wait, which keeps the
// kernel at the copy rate of its bytes without the 24 KB LDS block of the
// staged form. Other degrees (3, 12 or 27 floats per Gaussian, not 16-byte
// multiples) use the staged form.
template <bool DIRECT>
__global__ void __launch_bounds__(kProjThreads) project_kernel(const float* __restrict__ means,
                                                      const float* __restrict__ log_scales,
                                                      const float* __restrict__ quats,
                                                      const float* __restrict__ logits,
                                                      const float* __restrict__ sh, int64_t n, int degree,
                                                      ProjViews views) {
#pragma clang fp contract(off)
    // Staged form: the SH coefficients of the workgroup's Gaussians are one
    // contiguous block, staged through LDS with coalesced 16-byte loads.
    constexpr int kShVecs = kMaxShFloats / 4;
    __shared__ float4 sh_lds[DIRECT ? 1 : kShSink + 1];
    const int nsh = (degree + 1) * (degree + 1);
    const int64_t g0 = (int64_t)blockIdx.x * kProjThreads;
    const int64_t g = g0 + threadIdx.x;
    // the Gaussian's own inputs, requested while the SH block is in flight
    float in_m[3] = {0.f, 0.f, 0.f}, in_q[4] = {0.f, 0.f, 0.f, 0.f}, in_s[3] = {0.f, 0.f, 0.f}, in_l = 0.f;
    float4 shv[DIRECT ? kShVecs : 1];
    if constexpr (DIRECT) {
        if (g < n) {
            const float4* s4 = reinterpret_cast<const float4*>(sh + g * kMaxShFloats);
#pragma unroll
            for (int j = 0; j < kShVecs; ++j) shv[j] = s4[j];
        }
    }
    auto own_inputs = [&]() {
        if (g >= n) return;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            in_m[k] = means[3 * g + k];
            in_s[k] = log_scales[3 * g + k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) in_q[k] = quats[4 * g + k];
        in_l = logits[g];
    };
    if constexpr (DIRECT) {
        own_inputs();
    } else {
        stage_sh_block(sh_lds, sh + g0 * nsh * 3, min((int64_t)kProjThreads, n - g0) * nsh * 3, own_inputs);
        __syncthreads();
    }
    if (g >= n) return;
    // one camera: its splat and info line of this Gaussian
    auto one = [&](const Cam& cam, float4* __restrict__ splats, uint4* __restrict__ info) {
        float4* out = splats + kSplatVec * g;
        const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
        uint4 inf = make_uint4(0u, 0u, 0u, 0u);

        const double mx3 = in_m[0], my3 = in_m[1], mz3 = in_m[2];
        const double* R = cam.R;
        // camera-space point; the z expression is the ordering key's definition
        const double px = R[0] * mx3 + R[1] * my3 + R[2] * mz3 + cam.t[0];
        const double py = R[3] * mx3 + R[4] * my3 + R[5] * mz3 + cam.t[1];
        const double z = R[6] * mx3 + R[7] * my3 + R[8] * mz3 + cam.t[2];

        bool ok = (z > cam.znear) && (z < cam.zfar);
        double qw = in_q[0], qx = in_q[1], qy = in_q[2], qz = in_q[3];
        const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        ok = ok && (qn > 0.0) && isfinite(qn);
        double c00 = 0, c01 = 0, c11 = 0, det = 0, mxs = 0, mys = 0, o = 0, smax = 0;
        if (ok) {
            qw /= qn; qx /= qn; qy /= qn; qz /= qn;
            const double Rq[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy),
                                  2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
                                  2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};
            double s2[3];
    #pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double s = exp((double)in_s[k]);
                s2[k] = s * s;
                smax = fmax(smax, s);
            }
            // M = R_cam Rq: camera covariance = M diag(s^2) M^T
            double M[9];
    #pragma unroll
            for (int i = 0; i < 3; ++i)
    #pragma unroll
                for (int j = 0; j < 3; ++j) M[3 * i + j] = R[3 * i] * Rq[j] + R[3 * i + 1] * Rq[3 + j] + R[3 * i + 2] * Rq[6 + j];
            const double txz = px / z, tyz = py / z;
            const double tx = z * fmin(cam.lim_xp, fmax(-cam.lim_xn, txz));
            const double ty = z * fmin(cam.lim_yp, fmax(-cam.lim_yn, tyz));
            // rows of J M, J = [[fx/z, 0, -fx tx/z^2], [0, fy/z, -fy ty/z^2]]
            const double j00 = cam.fx / z, j02 = -cam.fx * tx / (z * z);
            const double j11 = cam.fy / z, j12 = -cam.fy * ty / (z * z);
            double A[3], B[3];
    #pragma unroll
            for (int k = 0; k < 3; ++k) {
                A[k] = j00 * M[k] + j02 * M[6 + k];
                B[k] = j11 * M[3 + k] + j12 * M[6 + k];
            }
            c00 = A[0] * A[0] * s2[0] + A[1] * A[1] * s2[1] + A[2] * A[2] * s2[2] + 0.3;
            c01 = A[0] * B[0] * s2[0] + A[1] * B[1] * s2[1] + A[2] * B[2] * s2[2];
            c11 = B[0] * B[0] * s2[0] + B[1] * B[1] * s2[1] + B[2] * B[2] * s2[2] + 0.3;
            det = c00 * c11 - c01 * c01;
            ok = (det > 0.0) && isfinite(det);
            mxs = cam.fx * px / z + cam.cx;
            mys = cam.fy * py / z + cam.cy;
            o = 1.0 / (1.0 + exp(-(double)in_l));
            const bool opaque_enough = cam.footprint == TGS_FOOTPRINT_THREE_SIGMA || o >= 1.0 / 255.0;
            ok = ok && opaque_enough && isfinite(mxs) && isfinite(mys);
        }
        int x0 = 0, y0 = 0, x1 = 0, y1 = 0;
        if (ok) {
            double ex, ey;
            if (cam.footprint == TGS_FOOTPRINT_THREE_SIGMA) {
                // the baseline's square: half side ceil(3 sqrt(lambda_max))
                const double mid = 0.5 * (c00 + c11);
                const double lam = mid + sqrt(fmax(0.1, mid * mid - det));
                ex = ey = ceil(3.0 * sqrt(lam));
            } else {
                // opacity-aware footprint: alpha >= 1/255 requires q <= 2 ln(255 o),
                // whose ellipse has half-extents sqrt(tau c00), sqrt(tau c11)
                const double tau = 2.0 * log(255.0 * o);
                ex = sqrt(tau * c00) * (1.0 + 1e-4) + 1e-3;
                ey = sqrt(tau * c11) * (1.0 + 1e-4) + 1e-3;
            }
            const double ts = (double)cam.tile;
            double fx0 = floor((mxs - ex) / ts), fx1 = floor((mxs + ex) / ts) + 1.0;
            double fy0 = floor((mys - ey) / ts), fy1 = floor((mys + ey) / ts) + 1.0;
            fx0 = fmin(fmax(fx0, 0.0), (double)cam.tiles_x);
            fx1 = fmin(fmax(fx1, 0.0), (double)cam.tiles_x);
            fy0 = fmin(fmax(fy0, 0.0), (double)cam.tiles_y);
            fy1 = fmin(fmax(fy1, 0.0), (double)cam.tiles_y);
            x0 = (int)fx0; x1 = (int)fx1; y0 = (int)fy0; y1 = (int)fy1;
            ok = (x1 > x0) && (y1 > y0);
        }
        if (!ok) {
            out[0] = zero4; out[1] = zero4; out[2] = zero4; out[3] = zero4;
            info[g] = inf;
            return;
        }
        // colour: 0.5 + sum sh_lm Y_lm(dir), dir from the camera centre, >= 0
        double dx = mx3 - cam.campos[0], dy = my3 - cam.campos[1], dz = mz3 - cam.campos[2];
        const double dn = sqrt(dx * dx + dy * dy + dz * dz);
        dx /= dn; dy /= dn; dz /= dn;
        double Y[16];
        sh_basis(dx, dy, dz, degree, Y);
        double col[3] = {0.0, 0.0, 0.0};
        if constexpr (DIRECT) {
            const float* shg = reinterpret_cast<const float*>(shv);
    #pragma unroll
            for (int k = 0; k < kMaxShFloats / 3; ++k) {
                col[0] += (double)shg[3 * k] * Y[k];
                col[1] += (double)shg[3 * k + 1] * Y[k];
                col[2] += (double)shg[3 * k + 2] * Y[k];
            }
        } else {
            const float* shg = reinterpret_cast<const float*>(sh_lds) + threadIdx.x * nsh * 3;
            for (int k = 0; k < nsh; ++k) {
                col[0] += (double)shg[3 * k] * Y[k];
                col[1] += (double)shg[3 * k + 1] * Y[k];
                col[2] += (double)shg[3 * k + 2] * Y[k];
            }
        }
        const float hx = (float)mxs, hy = (float)mys;
        out[0] = make_float4(hx, hy, (float)(mxs - (double)hx), (float)(mys - (double)hy));
        out[1] = make_float4((float)(c11 / det), (float)(-c01 / det), (float)(c00 / det), (float)o);
        out[2] = make_float4((float)fmax(0.0, 0.5 + col[0]), (float)fmax(0.0, 0.5 + col[1]),
                             (float)fmax(0.0, 0.5 + col[2]), (float)smax);
        out[3] = zero4;
        const float zf = (float)z;
        inf.x = __float_as_uint(zf);
        inf.y = (uint32_t)x0 | ((uint32_t)y0 << 16);
        inf.z = (uint32_t)x1 | ((uint32_t)y1 << 16);
        inf.w = (uint32_t)((x1 - x0) * (y1 - y0));
        info[g] = inf;
    };
#pragma unroll 1
    for (int v = 0; v < views.nv; ++v) one(views.cam[v], views.splats[v], views.info[v]);
}

// sum_k gY[k] grad Y_k at the unit direction (x, y, z): the derivatives of
// the polynomials of sh_basis.
__device__ __forceinline__ void sh_basis_vjp(double x, double y, double z, int degree, const double* gY,
                                             double* out) {
    out[0] = out[1] = out[2] = 0.0;
    if (degree < 1) return;
    const double c1 = 0.4886025119029199;
    out[1] += -c1 * gY[1];
    out[2] += c1 * gY[2];
    out[0] += -c1 * gY[3];
    if (degree < 2) return;
    const double k4 = 1.0925484305920792, k6 = 0.31539156525252005, k8 = 0.5462742152960396;
    const double xx = x * x, yy = y * y, zz = z * z;
    out[0] += gY[4] * k4 * y;
    out[1] += gY[4] * k4 * x;
    out[1] += -gY[5] * k4 * z;
    out[2] += -gY[5] * k4 * y;
    out[0] += -gY[6] * 2.0 * k6 * x;
    out[1] += -gY[6] * 2.0 * k6 * y;
    out[2] += gY[6] * 4.0 * k6 * z;
    out[0] += -gY[7] * k4 * z;
    out[2] += -gY[7] * k4 * x;
    out[0] += gY[8] * 2.0 * k8 * x;
    out[1] += -gY[8] * 2.0 * k8 * y;
    if (degree < 3) return;
    const double k9 = 0.5900435899266435, k10 = 2.890611442640554, k11 = 0.4570457994644658,
                 k12 = 0.3731763325901154, k14 = 1.445305721320277;
    // Y9 = -k9 y (3 xx - yy)
    out[0] += -gY[9] * k9 * 6.0 * x * y;
    out[1] += -gY[9] * k9 * (3.0 * xx - 3.0 * yy);
    // Y10 = k10 x y z
    out[0] += gY[10] * k10 * y * z;
    out[1] += gY[10] * k10 * x * z;
    out[2] += gY[10] * k10 * x * y;
    // Y11 = -k11 y (4 zz - xx - yy)
    out[0] += gY[11] * k11 * 2.0 * x * y;
    out[1] += -gY[11] * k11 * (4.0 * zz - xx - 3.0 * yy);
    out[2] += -gY[11] * k11 * 8.0 * y * z;
    // Y12 = k12 z (2 zz - 3 xx - 3 yy)
    out[0] += -gY[12] * k12 * 6.0 * x * z;
    out[1] += -gY[12] * k12 * 6.0 * y * z;
    out[2] += gY[12] * k12 * (6.0 * zz - 3.0 * xx - 3.0 * yy);
    // Y13 = -k11 x (4 zz - xx - yy)
    out[0] += -gY[13] * k11 * (4.0 * zz - 3.0 * xx - yy);
    out[1] += gY[13] * k11 * 2.0 * x * y;
    out[2] += -gY[13] * k11 * 8.0 * x * z;
    // Y14 = k14 z (xx - yy)
    out[0] += gY[14] * k14 * 2.0 * x * z;
    out[1] += -gY[14] * k14 * 2.0 * y * z;
    out[2] += gY[14] * k14 * (xx - yy);
    // Y15 = -k9 x (xx - 3 yy)
    out[0] += -gY[15] * k9 * (3.0 * xx - 3.0 * yy);
    out[1] += gY[15] * k9 * 6.0 * x * y;
}

// Backward of project_kernel in two launches, one lane per Gaussian,
// binary64: the forward quantities are recomputed with the forward's
// operations (so the same Gaussians are visible and the same guards and
// clamps are active) and the gradient line d = dL/d(mean_x, mean_y, conic
// a, b, c, opacity, r, g, b) is taken back through
//   sh_bwd:   the clamped SH colour (coefficients, and the mean through the
//             view direction); writes d_sh and the SH part of d_means;
//   geom_bwd: the conic inverse, the screen covariance J M diag(s^2) M^T
//             J^T + 0.3 I (M = R_cam R_q), the guarded perspective Jacobian,
//             the screen mean, the quaternion normalisation, exp of the
//             log-scales and the sigmoid; adds to d_means.
// Splitting keeps each kernel's binary64 register footprint small enough
// for several wavefronts per SIMD. Gaussians whose gradient line is zero
// (invisible or never composited) are skipped and get zero gradients.
// DIRECT (SH3, 16-byte aligned coefficients and gradients): each lane loads
// and stores its own 48 floats with 16-byte accesses, no LDS, as in the
// forward.
template <bool DIRECT>
__global__ void __launch_bounds__(kProjThreads) sh_bwd_kernel(const float* __restrict__ means,
                                                             const float* __restrict__ sh, int64_t n, int degree,
                                                             Cam cam, const float4* __restrict__ dsp,
                                                             float* __restrict__ d_means, float* __restrict__ d_sh) {
#pragma clang fp contract(off)
    constexpr int kShVecs = kMaxShFloats / 4;
    __shared__ float4 sh_lds[DIRECT ? 1 : kShSink + 1];
    const int nsh = DIRECT ? kMaxShFloats / 3 : (degree + 1) * (degree + 1);
    const int nf = nsh * 3;
    const int64_t g0 = (int64_t)blockIdx.x * kProjThreads;
    const int64_t cnt = min((int64_t)kProjThreads, n - g0) * nf;  // floats
    const int64_t g = g0 + threadIdx.x;
    float4 d1 = make_float4(0.f, 0.f, 0.f, 0.f), d2 = d1;
    float in_m[3] = {0.f, 0.f, 0.f};
    float4 shv[DIRECT ? kShVecs : 1];
    if constexpr (DIRECT) {
        if (g < n) {
            const float4* s4 = reinterpret_cast<const float4*>(sh + g * kMaxShFloats);
#pragma unroll
            for (int j = 0; j < kShVecs; ++j) shv[j] = s4[j];
        }
    }
    auto own_inputs = [&]() {
        if (g >= n) return;
        d1 = dsp[kGradWords / 4 * g + 1];
        d2 = dsp[kGradWords / 4 * g + 2];
#pragma unroll
        for (int k = 0; k < 3; ++k) in_m[k] = means[3 * g + k];
    };
    float* f = reinterpret_cast<float*>(sh_lds);
    if constexpr (DIRECT) {
        own_inputs();
    } else {
        stage_sh_block(sh_lds, sh + g0 * nf, cnt, own_inputs);
        __syncthreads();
    }
    if (g < n) {
        // coefficients in, gradients out (in place)
        float* shg = DIRECT ? reinterpret_cast<float*>(shv) : f + threadIdx.x * nf;
        const double dcol[3] = {d1.z, d1.w, d2.x};
        double gm[3] = {0.0, 0.0, 0.0};
        if (dcol[0] != 0.0 || dcol[1] != 0.0 || dcol[2] != 0.0) {
            const double mx3 = in_m[0], my3 = in_m[1], mz3 = in_m[2];
            double ux = mx3 - cam.campos[0], uy = my3 - cam.campos[1], uz = mz3 - cam.campos[2];
            const double dn = sqrt(ux * ux + uy * uy + uz * uz);
            ux /= dn; uy /= dn; uz /= dn;
            double Y[16];
            sh_basis(ux, uy, uz, degree, Y);
            double col[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < nsh; ++k) {
                col[0] += (double)shg[3 * k] * Y[k];
                col[1] += (double)shg[3 * k + 1] * Y[k];
                col[2] += (double)shg[3 * k + 2] * Y[k];
            }
            const bool on[3] = {0.5 + col[0] > 0.0, 0.5 + col[1] > 0.0, 0.5 + col[2] > 0.0};
            double gY[16];
            for (int k = 0; k < nsh; ++k) {
                double acc = 0.0;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    if (!on[ch]) continue;
                    acc += dcol[ch] * (double)shg[3 * k + ch];
                }
                gY[k] = acc;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) shg[3 * k + ch] = on[ch] ? (float)(dcol[ch] * Y[k]) : 0.f;
            }
            double gu[3];
            sh_basis_vjp(ux, uy, uz, degree, gY, gu);
            const double gdot = gu[0] * ux + gu[1] * uy + gu[2] * uz;
            gm[0] = (gu[0] - gdot * ux) / dn;
            gm[1] = (gu[1] - gdot * uy) / dn;
            gm[2] = (gu[2] - gdot * uz) / dn;
        } else {
            for (int k = 0; k < nf; ++k) shg[k] = 0.f;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) d_means[3 * g + k] = (float)gm[k];
        if constexpr (DIRECT) {
            float4* d4 = reinterpret_cast<float4*>(d_sh + g * kMaxShFloats);
#pragma unroll
            for (int j = 0; j < kShVecs; ++j) d4[j] = shv[j];
        }
    }
    if constexpr (!DIRECT) {
        __syncthreads();
        float* dst = d_sh + g0 * nf;
        if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
            float4* d4 = reinterpret_cast<float4*>(dst);
            for (int64_t i = threadIdx.x; i < cnt / 4; i += kProjThreads) d4[i] = sh_lds[i];
            for (int64_t i = (cnt / 4) * 4 + threadIdx.x; i < cnt; i += kProjThreads) dst[i] = f[i];
        } else {
            for (int64_t i = threadIdx.x; i < cnt; i += kProjThreads) dst[i] = f[i];
        }
    }
}

__global__ void __launch_bounds__(256) geom_bwd_kernel(const float* __restrict__ means,
                                                      const float* __restrict__ log_scales,
                                                      const float* __restrict__ quats,
                                                      const float* __restrict__ logits, int64_t n, Cam cam,
                                                      const float4* __restrict__ dsp, float* __restrict__ d_means,
                                                      float* __restrict__ d_ls, float* __restrict__ d_quats,
                                                      float* __restrict__ d_logits) {
#pragma clang fp contract(off)
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    double gm[3] = {0.0, 0.0, 0.0}, gls[3] = {0.0, 0.0, 0.0}, gq4[4] = {0.0, 0.0, 0.0, 0.0}, glogit = 0.0;
    const float4 d0 = dsp[kGradWords / 4 * g], d1 = dsp[kGradWords / 4 * g + 1];
    const bool any = d0.x != 0.f || d0.y != 0.f || d0.z != 0.f || d0.w != 0.f || d1.x != 0.f || d1.y != 0.f;
    const double mx3 = means[3 * g], my3 = means[3 * g + 1], mz3 = means[3 * g + 2];
    const double* R = cam.R;
    const double px = R[0] * mx3 + R[1] * my3 + R[2] * mz3 + cam.t[0];
    const double py = R[3] * mx3 + R[4] * my3 + R[5] * mz3 + cam.t[1];
    const double z = R[6] * mx3 + R[7] * my3 + R[8] * mz3 + cam.t[2];
    bool ok = any && (z > cam.znear) && (z < cam.zfar);
    double qv[4] = {quats[4 * g], quats[4 * g + 1], quats[4 * g + 2], quats[4 * g + 3]};
    const double qn = sqrt(qv[0] * qv[0] + qv[1] * qv[1] + qv[2] * qv[2] + qv[3] * qv[3]);
    ok = ok && (qn > 0.0) && isfinite(qn);
    if (ok) {
        const double qw = qv[0] / qn, qx = qv[1] / qn, qy = qv[2] / qn, qz = qv[3] / qn;
        const double Rq[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz),
                              2.0 * (qx * qz + qw * qy),       2.0 * (qx * qy + qw * qz),
                              1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
                              2.0 * (qx * qz - qw * qy),       2.0 * (qy * qz + qw * qx),
                              1.0 - 2.0 * (qx * qx + qy * qy)};
        double s2[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double sc = exp((double)log_scales[3 * g + k]);
            s2[k] = sc * sc;
        }
        double M[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                M[3 * i + j] = R[3 * i] * Rq[j] + R[3 * i + 1] * Rq[3 + j] + R[3 * i + 2] * Rq[6 + j];
        const double txz = px / z, tyz = py / z;
        const double cxz = fmin(cam.lim_xp, fmax(-cam.lim_xn, txz));
        const double cyz = fmin(cam.lim_yp, fmax(-cam.lim_yn, tyz));
        const bool gx = cxz != txz, gy = cyz != tyz;  // frustum guard active
        const double tx = z * cxz, ty = z * cyz;
        const double j00 = cam.fx / z, j02 = -cam.fx * tx / (z * z);
        const double j11 = cam.fy / z, j12 = -cam.fy * ty / (z * z);
        double A[3], B[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            A[k] = j00 * M[k] + j02 * M[6 + k];
            B[k] = j11 * M[3 + k] + j12 * M[6 + k];
        }
        const double c00 = A[0] * A[0] * s2[0] + A[1] * A[1] * s2[1] + A[2] * A[2] * s2[2] + 0.3;
        const double c01 = A[0] * B[0] * s2[0] + A[1] * B[1] * s2[1] + A[2] * B[2] * s2[2];
        const double c11 = B[0] * B[0] * s2[0] + B[1] * B[1] * s2[1] + B[2] * B[2] * s2[2] + 0.3;
        const double det = c00 * c11 - c01 * c01;
        ok = (det > 0.0) && isfinite(det);
        const double mxs = cam.fx * px / z + cam.cx;
        const double mys = cam.fy * py / z + cam.cy;
        const double o = 1.0 / (1.0 + exp(-(double)logits[g]));
        ok = ok && (o >= 1.0 / 255.0) && isfinite(mxs) && isfinite(mys);
        if (ok) {
            const double dmx = d0.x, dmy = d0.y, dA = d0.z, dB = d0.w, dC = d1.x, dop = d1.y;
            // opacity = sigmoid(logit)
            glogit = dop * o * (1.0 - o);
            // conic = [c11, -c01, c00] / det
            const double dd = det * det;
            const double ga = dA * (-c11 * c11 / dd) + dB * (c01 * c11 / dd) + dC * (-c01 * c01 / dd);
            const double gb = dA * (2.0 * c01 * c11 / dd) + dB * (-1.0 / det - 2.0 * c01 * c01 / dd) +
                              dC * (2.0 * c00 * c01 / dd);
            const double gc = dA * (-c01 * c01 / dd) + dB * (c00 * c01 / dd) + dC * (-c00 * c00 / dd);
            // covariance entries from the rows A, B of J M and s^2
            double gA[3], gB[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                gA[k] = 2.0 * ga * A[k] * s2[k] + gb * B[k] * s2[k];
                gB[k] = 2.0 * gc * B[k] * s2[k] + gb * A[k] * s2[k];
                gls[k] = 2.0 * s2[k] * (ga * A[k] * A[k] + gb * A[k] * B[k] + gc * B[k] * B[k]);
            }
            double g00 = 0.0, g02 = 0.0, g11 = 0.0, g12 = 0.0, gM[9];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                g00 += gA[k] * M[k];
                g02 += gA[k] * M[6 + k];
                g11 += gB[k] * M[3 + k];
                g12 += gB[k] * M[6 + k];
                gM[k] = gA[k] * j00;
                gM[3 + k] = gB[k] * j11;
                gM[6 + k] = gA[k] * j02 + gB[k] * j12;
            }
            // M = R_cam R_q  =>  dL/dR_q = R_cam^T dL/dM
            double gR[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) gR[3 * i + j] = R[i] * gM[j] + R[3 + i] * gM[3 + j] + R[6 + i] * gM[6 + j];
            // R_q entries as functions of the unit quaternion
            const double gw = 2.0 * (-qz * gR[1] + qy * gR[2] + qz * gR[3] - qx * gR[5] - qy * gR[6] + qx * gR[7]);
            const double gxq = 2.0 * (qy * gR[1] + qz * gR[2] + qy * gR[3] - 2.0 * qx * gR[4] - qw * gR[5] +
                                      qz * gR[6] + qw * gR[7] - 2.0 * qx * gR[8]);
            const double gyq = 2.0 * (-2.0 * qy * gR[0] + qx * gR[1] + qw * gR[2] + qx * gR[3] + qz * gR[5] -
                                      qw * gR[6] + qz * gR[7] - 2.0 * qy * gR[8]);
            const double gzq = 2.0 * (-2.0 * qz * gR[0] - qw * gR[1] + qx * gR[2] + qw * gR[3] - 2.0 * qz * gR[4] +
                                      qy * gR[5] + qx * gR[6] + qy * gR[7]);
            // q_hat = q / |q|
            const double qh[4] = {qw, qx, qy, qz};
            const double gh[4] = {gw, gxq, gyq, gzq};
            const double hd = gw * qw + gxq * qx + gyq * qy + gzq * qz;
#pragma unroll
            for (int k = 0; k < 4; ++k) gq4[k] = (gh[k] - hd * qh[k]) / qn;
            // J entries and the screen mean as functions of the camera-space point
            double gp0 = dmx * cam.fx / z, gp1 = dmy * cam.fy / z;
            double gz = -dmx * cam.fx * px / (z * z) - dmy * cam.fy * py / (z * z);
            gz += -g00 * cam.fx / (z * z) - g11 * cam.fy / (z * z);
            if (gx) {
                gz += g02 * cam.fx * cxz / (z * z);
            } else {
                gp0 += -g02 * cam.fx / (z * z);
                gz += g02 * 2.0 * cam.fx * px / (z * z * z);
            }
            if (gy) {
                gz += g12 * cam.fy * cyz / (z * z);
            } else {
                gp1 += -g12 * cam.fy / (z * z);
                gz += g12 * 2.0 * cam.fy * py / (z * z * z);
            }
            // p_cam = R_cam mean + t
#pragma unroll
            for (int c = 0; c < 3; ++c) gm[c] = R[c] * gp0 + R[3 + c] * gp1 + R[6 + c] * gz;
        }
    }
    // the SH part of d_means was written by sh_bwd_kernel (same lane layout)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d_means[3 * g + k] = (float)((double)d_means[3 * g + k] + gm[k]);
        d_ls[3 * g + k] = (float)gls[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) d_quats[4 * g + k] = (float)gq4[k];
    d_logits[g] = (float)glogit;
}

hipError_t launch_project_views(const tgs_gaussians& g, const ProjViews& views, hipStream_t s) {
    if (g.n == 0 || views.nv == 0) return hipSuccess;
    const int block = kProjThreads;
    const int64_t grid = (g.n + block - 1) / block;
    const bool direct = g.sh_degree == 3 && (reinterpret_cast<uintptr_t>(g.sh_dev) & 15) == 0;
    if (direct)
        hipLaunchKernelGGL(project_kernel<true>, dim3((unsigned)grid), dim3(block), 0, s, g.means_dev,
                           g.log_scales_dev, g.quats_dev, g.logits_dev, g.sh_dev, g.n, g.sh_degree, views);
    else
        hipLaunchKernelGGL(project_kernel<false>, dim3((unsigned)grid), dim3(block), 0, s, g.means_dev,
                           g.log_scales_dev, g.quats_dev, g.logits_dev, g.sh_dev, g.n, g.sh_degree, views);
    return hipGetLastError();
}

hipError_t launch_project(const tgs_gaussians& g, const Cam& cam, float* splats, uint32_t* info, hipStream_t s) {
    ProjViews v{};
    v.nv = 1;
    v.cam[0] = cam;
    v.splats[0] = reinterpret_cast<float4*>(splats);
    v.info[0] = reinterpret_cast<uint4*>(info);
    return launch_project_views(g, v, s);
}

hipError_t launch_project_backward(const tgs_gaussians& g, const Cam& cam, const float* d_splats,
                                   const tgs_gaussian_grads& out, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    const int64_t grid = (g.n + kProjThreads - 1) / kProjThreads;
    const auto* dsp = reinterpret_cast<const float4*>(d_splats);
    const bool direct = g.sh_degree == 3 && (reinterpret_cast<uintptr_t>(g.sh_dev) & 15) == 0 &&
                        (reinterpret_cast<uintptr_t>(out.sh_dev) & 15) == 0;
    if (direct)
        hipLaunchKernelGGL(sh_bwd_kernel<true>, dim3((unsigned)grid), dim3(kProjThreads), 0, s, g.means_dev,
                           g.sh_dev, g.n, g.sh_degree, cam, dsp, out.means_dev, out.sh_dev);
    else
        hipLaunchKernelGGL(sh_bwd_kernel<false>, dim3((unsigned)grid), dim3(kProjThreads), 0, s, g.means_dev,
                           g.sh_dev, g.n, g.sh_degree, cam, dsp, out.means_dev, out.sh_dev);
    hipLaunchKernelGGL(geom_bwd_kernel, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, s, g.means_dev,
                       g.log_scales_dev, g.quats_dev, g.logits_dev, g.n, cam, dsp, out.means_dev, out.log_scales_dev,
                       out.quats_dev, out.logits_dev);
    return hipGetLastError();
}

}  // namespace tgs
