// Projection of 3D Gaussians to screen-space splats (EWA splatting with the
// 3DGS conventions, which the paper keeps unchanged): camera transform,
// covariance R S^2 R^T, perspective Jacobian with the 30 % frustum guard,
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

Cam make_cam(const tgs_camera& c) {
    Cam k;
    for (int i = 0; i < 9; ++i) k.R[i] = c.R[i];
    for (int i = 0; i < 3; ++i) k.t[i] = c.t[i];
    k.fx = c.fx; k.fy = c.fy; k.cx = c.cx; k.cy = c.cy;
    k.znear = c.znear; k.zfar = c.zfar;
    k.width = c.width; k.height = c.height;
    k.tiles_x = div_up(c.width, kTile);
    k.tiles_y = div_up(c.height, kTile);
    for (int i = 0; i < 3; ++i) k.campos[i] = -(c.R[i] * c.t[0] + c.R[3 + i] * c.t[1] + c.R[6 + i] * c.t[2]);
    k.lim_xp = (c.width - c.cx) / c.fx + 0.3 * c.width / c.fx;
    k.lim_xn = c.cx / c.fx + 0.3 * c.width / c.fx;
    k.lim_yp = (c.height - c.cy) / c.fy + 0.3 * c.height / c.fy;
    k.lim_yn = c.cy / c.fy + 0.3 * c.height / c.fy;
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

__global__ void __launch_bounds__(kProjThreads) project_kernel(const float* __restrict__ means,
                                                      const float* __restrict__ log_scales,
                                                      const float* __restrict__ quats,
                                                      const float* __restrict__ logits,
                                                      const float* __restrict__ sh, int64_t n, int degree,
                                                      Cam cam, float4* __restrict__ splats,
                                                      uint4* __restrict__ info) {
#pragma clang fp contract(off)
    // The SH coefficients of the workgroup's Gaussians are one contiguous
    // block; stage it through LDS with coalesced 16-byte loads.
    __shared__ float4 sh_lds[kProjThreads * kMaxShFloats / 4];
    const int nsh = (degree + 1) * (degree + 1);
    const int64_t g0 = (int64_t)blockIdx.x * kProjThreads;
    {
        const int64_t cnt = min((int64_t)kProjThreads, n - g0) * nsh * 3;  // floats
        const float* src = sh + g0 * nsh * 3;
        if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
            const float4* s4 = reinterpret_cast<const float4*>(src);
            for (int64_t i = threadIdx.x; i < cnt / 4; i += kProjThreads) sh_lds[i] = s4[i];
            float* f = reinterpret_cast<float*>(sh_lds);
            for (int64_t i = (cnt / 4) * 4 + threadIdx.x; i < cnt; i += kProjThreads) f[i] = src[i];
        } else {
            float* f = reinterpret_cast<float*>(sh_lds);
            for (int64_t i = threadIdx.x; i < cnt; i += kProjThreads) f[i] = src[i];
        }
    }
    __syncthreads();
    const int64_t g = g0 + threadIdx.x;
    if (g >= n) return;
    float4* out = splats + kSplatVec * g;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    uint4 inf = make_uint4(0u, 0u, 0u, 0u);

    const double mx3 = means[3 * g], my3 = means[3 * g + 1], mz3 = means[3 * g + 2];
    const double* R = cam.R;
    // camera-space point; the z expression is the ordering key's definition
    const double px = R[0] * mx3 + R[1] * my3 + R[2] * mz3 + cam.t[0];
    const double py = R[3] * mx3 + R[4] * my3 + R[5] * mz3 + cam.t[1];
    const double z = R[6] * mx3 + R[7] * my3 + R[8] * mz3 + cam.t[2];

    bool ok = (z > cam.znear) && (z < cam.zfar);
    double qw = quats[4 * g], qx = quats[4 * g + 1], qy = quats[4 * g + 2], qz = quats[4 * g + 3];
    const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    ok = ok && (qn > 0.0) && isfinite(qn);
    double c00 = 0, c01 = 0, c11 = 0, det = 0, mxs = 0, mys = 0, o = 0;
    if (ok) {
        qw /= qn; qx /= qn; qy /= qn; qz /= qn;
        const double Rq[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy),
                              2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
                              2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};
        double s2[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double s = exp((double)log_scales[3 * g + k]);
            s2[k] = s * s;
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
        o = 1.0 / (1.0 + exp(-(double)logits[g]));
        ok = ok && (o >= 1.0 / 255.0) && isfinite(mxs) && isfinite(mys);
    }
    int x0 = 0, y0 = 0, x1 = 0, y1 = 0;
    if (ok) {
        // opacity-aware footprint: alpha >= 1/255 requires q <= 2 ln(255 o),
        // whose ellipse has half-extents sqrt(tau c00), sqrt(tau c11)
        const double tau = 2.0 * log(255.0 * o);
        const double ex = sqrt(tau * c00) * (1.0 + 1e-4) + 1e-3;
        const double ey = sqrt(tau * c11) * (1.0 + 1e-4) + 1e-3;
        double fx0 = floor((mxs - ex) / kTile), fx1 = floor((mxs + ex) / kTile) + 1.0;
        double fy0 = floor((mys - ey) / kTile), fy1 = floor((mys + ey) / kTile) + 1.0;
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
    const float* shg = reinterpret_cast<const float*>(sh_lds) + threadIdx.x * nsh * 3;
    for (int k = 0; k < nsh; ++k) {
        col[0] += (double)shg[3 * k] * Y[k];
        col[1] += (double)shg[3 * k + 1] * Y[k];
        col[2] += (double)shg[3 * k + 2] * Y[k];
    }
    const float hx = (float)mxs, hy = (float)mys;
    out[0] = make_float4(hx, hy, (float)(mxs - (double)hx), (float)(mys - (double)hy));
    out[1] = make_float4((float)(c11 / det), (float)(-c01 / det), (float)(c00 / det), (float)o);
    out[2] = make_float4((float)fmax(0.0, 0.5 + col[0]), (float)fmax(0.0, 0.5 + col[1]),
                         (float)fmax(0.0, 0.5 + col[2]), 0.f);
    out[3] = zero4;
    const float zf = (float)z;
    inf.x = __float_as_uint(zf);
    inf.y = (uint32_t)x0 | ((uint32_t)y0 << 16);
    inf.z = (uint32_t)x1 | ((uint32_t)y1 << 16);
    inf.w = (uint32_t)((x1 - x0) * (y1 - y0));
    info[g] = inf;
}

hipError_t launch_project(const tgs_gaussians& g, const Cam& cam, float* splats, uint32_t* info, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    const int block = kProjThreads;
    const int64_t grid = (g.n + block - 1) / block;
    hipLaunchKernelGGL(project_kernel, dim3((unsigned)grid), dim3(block), 0, s, g.means_dev, g.log_scales_dev,
                       g.quats_dev, g.logits_dev, g.sh_dev, g.n, g.sh_degree, cam,
                       reinterpret_cast<float4*>(splats), reinterpret_cast<uint4*>(info));
    return hipGetLastError();
}

}  // namespace tgs
