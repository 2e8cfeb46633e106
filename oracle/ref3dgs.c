/*
 * ref3dgs.c -- plain, slow FP64 CPU reference for the 3D Gaussian splatting
 * forward image, its integer schedule (tile keys, depth bins, offsets) and its
 * adjoint.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link or call this
 * file; only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg use it. It shares no code, header, table or constant generator with the
 * GPU library.
 *
 * What it follows:
 *  - The image model is the unchanged 3DGS one (paper: Introduction and the
 *    Related-work paragraph on 3DGS/EWA splatting; the method section states
 *    that projection, splat evaluation and compositing are kept as in the
 *    baseline). The equations are the standard EWA-splatting / 3DGS ones:
 *    Sigma = R S^2 R^T, Sigma' = J W Sigma W^T J^T + 0.3 I, conic = Sigma'^-1,
 *    alpha = min(0.99, o exp(-q/2)), skip alpha < 1/255, stop before the
 *    Gaussian that would take T below 1e-4, C += T alpha c.
 *  - The baseline ordering is "first by tile, then by depth" (section
 *    "Baseline 3DGS rasterization"); ties are broken by Gaussian id.
 *  - Depth range: supplement, Algorithm "Robust depth-range estimation".
 *  - Tile-local bins, count / exclusive scan / scatter: supplement,
 *    Algorithm "Tile-local bin construction" and the log-depth-bin equation.
 *  - Repair selection rules and budget: Table "Exact-repair selection rules"
 *    and supplement Algorithm "Selective repair selection and local exact
 *    sorting".
 *
 * Everything is computed in double precision except where a floating-point
 * value decides an integer the GPU path also decides (the depth used as the
 * ordering key, the depth range and the bin index): there the computation is
 * done in the precision the GPU path uses (IEEE binary32, no contraction),
 * and ambiguous cases are reported through flag bits instead of guessed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EXPORT __attribute__((visibility("default")))

/* Fixed thresholds of the 3DGS image model. */
static const double ALPHA_MIN = 1.0 / 255.0;
static const double ALPHA_MAX = 0.99;
static const double T_MIN = 1e-4;
static const double DILATION = 0.3;  /* px^2 added to the screen covariance */
static const double GUARD = 0.3;     /* frustum guard: 0.3 tan(half FOV) beyond the image edge */

/* Per-Gaussian flag bits written by orc_project. */
enum {
    ORC_VISIBLE = 1,
    ORC_AMBIG_RECT = 2,   /* a footprint edge sits on a tile boundary */
    ORC_AMBIG_DEPTH = 4,  /* reserved */
    ORC_AMBIG_VIS = 8     /* a visibility test is within rounding of its edge */
};

/* Per-pixel flag bits written by orc_render. */
enum {
    PIX_AMBIG_ALPHA = 1,  /* some alpha within rounding of 1/255 */
    PIX_AMBIG_STOP = 2,   /* the stopping test within rounding of 1e-4 */
    PIX_AMBIG_GAUSS = 4,  /* a Gaussian with an ambiguity flag is involved */
    PIX_POWER_POS = 8     /* -q/2 > 0 was seen (cannot happen in exact math) */
};

ORC_EXPORT int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics from associated Legendre functions.             */
/* ------------------------------------------------------------------------ */

static double factorial(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

/* Associated Legendre P_l^m(x), m >= 0, with the Condon-Shortley phase. */
static double legendre(int l, int m, double x) {
    double pmm = 1.0;
    double s = sqrt(fmax(0.0, 1.0 - x * x));
    for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * s;
    if (l == m) return pmm;
    double pm1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pm1;
    double pl = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pl = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pm1;
        pm1 = pl;
    }
    return pl;
}

/* Y_lm(dir) for l <= degree into out[l*l + l + m]; dir need not be unit. */
ORC_EXPORT void orc_sh_basis(const double* dir, int degree, double* out) {
    double n = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double x = dir[0] / n, y = dir[1] / n, z = dir[2] / n;
    double phi = atan2(y, x);
    for (int l = 0; l <= degree; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double norm = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
            double p = legendre(l, am, z);
            double v;
            if (m > 0)
                v = sqrt(2.0) * norm * p * cos(am * phi);
            else if (m < 0)
                v = sqrt(2.0) * norm * p * sin(am * phi);
            else
                v = norm * p;
            out[l * l + l + m] = v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Projection of one Gaussian (EWA splatting, 3DGS conventions).            */
/* camera: double[20] = R[9] (row-major world->camera), t[3], fx, fy, cx,   */
/* cy, width, height, znear, zfar.                                          */
/* ------------------------------------------------------------------------ */

static int near_integer(double v, double tol) {
    return fabs(v - floor(v + 0.5)) < tol;
}

/*
 * Footprint (tile rect) rules of orc_project:
 *  OPACITY_AWARE: the tiles meeting the bounding box of the ellipse where
 *    o exp(-q/2) >= 1/255, i.e. q <= 2 ln(255 o) (a superset of the alpha
 *    support, so the image does not depend on tiles); Gaussians with
 *    o < 1/255 are invisible.
 *  THREE_SIGMA: the rule of the baseline rasterizer the paper compares
 *    against: the tiles meeting the square of half side r = ceil(3
 *    sqrt(lambda_max)) pixels around the mean, lambda_max = mid + sqrt(max(
 *    0.1, mid^2 - det)) the larger eigenvalue of the screen covariance (mid
 *    its mean diagonal); the alpha support is cut at those tiles, so the
 *    image depends on the tile size; no opacity cut.
 */
enum { FOOT_OPACITY_AWARE = 0, FOOT_THREE_SIGMA = 1 };

ORC_EXPORT int orc_project(int64_t n, const float* means, const float* log_scales,
                           const float* quats, const float* logits, const float* sh,
                           int sh_degree, const double* cam, int tile_size, int footprint,
                           double* mean2d, double* cov2d, double* conic, double* depth,
                           double* opacity, double* rgb, int32_t* rect, float* depth_key,
                           uint8_t* flags) {
    if (n < 0 || sh_degree < 0 || sh_degree > 3 || tile_size <= 0) return 1;
    if (footprint != FOOT_OPACITY_AWARE && footprint != FOOT_THREE_SIGMA) return 1;
    const double* R = cam;
    const double* t = cam + 9;
    const double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    const int W = (int)cam[16], H = (int)cam[17];
    const double znear = cam[18], zfar = cam[19];
    const int tiles_x = (W + tile_size - 1) / tile_size;
    const int tiles_y = (H + tile_size - 1) / tile_size;
    const int nsh = (sh_degree + 1) * (sh_degree + 1);
    /* camera centre c = -R^T t */
    double campos[3];
    for (int i = 0; i < 3; ++i) campos[i] = -(R[0 * 3 + i] * t[0] + R[1 * 3 + i] * t[1] + R[2 * 3 + i] * t[2]);

#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        uint8_t fl = 0;
        mean2d[2 * g] = mean2d[2 * g + 1] = 0.0;
        for (int k = 0; k < 3; ++k) { cov2d[3 * g + k] = 0.0; conic[3 * g + k] = 0.0; rgb[3 * g + k] = 0.0; }
        depth[g] = 0.0;
        opacity[g] = 0.0;
        depth_key[g] = 0.0f;
        rect[4 * g] = rect[4 * g + 1] = rect[4 * g + 2] = rect[4 * g + 3] = 0;

        double mu[3] = {means[3 * g], means[3 * g + 1], means[3 * g + 2]};
        double pc[3];
        for (int i = 0; i < 3; ++i) pc[i] = R[3 * i] * mu[0] + R[3 * i + 1] * mu[1] + R[3 * i + 2] * mu[2] + t[i];
        double z = pc[2];
        if (!(z > znear && z < zfar)) {
            if (fabs(z - znear) <= 1e-12 * fabs(znear) + 1e-300) fl |= ORC_AMBIG_VIS;
            flags[g] = fl;
            continue;
        }
        if (fabs(z - znear) <= 1e-12 * znear) fl |= ORC_AMBIG_VIS;
        /* The ordering key is the binary32 rounding of this binary64 depth,
           evaluated as ((R20 x + R21 y) + R22 z) + t2 without contraction, so
           any implementation that performs the same IEEE operations in the
           same order obtains the same key bits. */
        depth[g] = z;
        depth_key[g] = (float)z;

        /* rotation from the normalised quaternion (w, x, y, z) */
        double qw = quats[4 * g], qx = quats[4 * g + 1], qy = quats[4 * g + 2], qz = quats[4 * g + 3];
        double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        if (!(qn > 0.0) || !isfinite(qn)) { flags[g] = fl; continue; }
        qw /= qn; qx /= qn; qy /= qn; qz /= qn;
        double Rq[9] = {
            1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy),
            2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
            2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};
        double s2[3];
        for (int k = 0; k < 3; ++k) { double s = exp((double)log_scales[3 * g + k]); s2[k] = s * s; }
        /* world covariance Sigma = Rq diag(s^2) Rq^T */
        double Sw[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += Rq[3 * i + k] * s2[k] * Rq[3 * j + k];
                Sw[3 * i + j] = acc;
            }
        /* camera covariance R Sigma R^T */
        double RS[9], Sc[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += R[3 * i + k] * Sw[3 * k + j];
                RS[3 * i + j] = acc;
            }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += RS[3 * i + k] * R[3 * j + k];
                Sc[3 * i + j] = acc;
            }
        /* Jacobian of the perspective map at the (guarded) centre */
        /* x/z is clamped to the image edge plus 0.3 tan(half FOV), tan(half
           FOV) = W / (2 fx): +-1.3 W / (2 fx) for a centred principal point */
        double tanx = 0.5 * W / fx, tany = 0.5 * H / fy;
        double lim_xp = (W - cx) / fx + GUARD * tanx, lim_xn = cx / fx + GUARD * tanx;
        double lim_yp = (H - cy) / fy + GUARD * tany, lim_yn = cy / fy + GUARD * tany;
        double txz = pc[0] / z, tyz = pc[1] / z;
        double tx = z * fmin(lim_xp, fmax(-lim_xn, txz));
        double ty = z * fmin(lim_yp, fmax(-lim_yn, tyz));
        double J[6] = {fx / z, 0.0, -fx * tx / (z * z), 0.0, fy / z, -fy * ty / (z * z)};
        double JS[6];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += J[3 * i + k] * Sc[3 * k + j];
                JS[3 * i + j] = acc;
            }
        double C2[4];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += JS[3 * i + k] * J[3 * j + k];
                C2[2 * i + j] = acc;
            }
        double c00 = C2[0] + DILATION, c01 = 0.5 * (C2[1] + C2[2]), c11 = C2[3] + DILATION;
        cov2d[3 * g] = c00; cov2d[3 * g + 1] = c01; cov2d[3 * g + 2] = c11;
        double det = c00 * c11 - c01 * c01;
        if (!(det > 0.0) || !isfinite(det)) { flags[g] = fl; continue; }
        conic[3 * g] = c11 / det;
        conic[3 * g + 1] = -c01 / det;
        conic[3 * g + 2] = c00 / det;
        double mx = fx * pc[0] / z + cx, my = fy * pc[1] / z + cy;
        mean2d[2 * g] = mx;
        mean2d[2 * g + 1] = my;

        double o = 1.0 / (1.0 + exp(-(double)logits[g]));
        opacity[g] = o;

        /* colour: 0.5 + sum_lm sh_lm Y_lm(dir), clamped below at 0 */
        double dir[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
        double Y[16];
        orc_sh_basis(dir, sh_degree, Y);
        for (int ch = 0; ch < 3; ++ch) {
            double acc = 0.0;
            for (int k = 0; k < nsh; ++k) acc += (double)sh[((int64_t)g * nsh + k) * 3 + ch] * Y[k];
            rgb[3 * g + ch] = fmax(0.0, 0.5 + acc);
        }

        double ex, ey;
        if (footprint == FOOT_OPACITY_AWARE) {
            /* alpha >= 1/255 needs q <= 2 ln(255 o) */
            if (fabs(o * 255.0 - 1.0) < 1e-12) fl |= ORC_AMBIG_VIS;
            if (!(o >= ALPHA_MIN)) { flags[g] = fl; continue; }
            double tau = 2.0 * log(255.0 * o);
            double hx = sqrt(tau * c00), hy = sqrt(tau * c11);
            ex = hx * (1.0 + 1e-4) + 1e-3;
            ey = hy * (1.0 + 1e-4) + 1e-3;
        } else {
            double mid = 0.5 * (c00 + c11);
            double lam = mid + sqrt(fmax(0.1, mid * mid - det));
            double r3 = 3.0 * sqrt(lam);
            if (near_integer(r3, 1e-9)) fl |= ORC_AMBIG_RECT;
            ex = ey = ceil(r3);
        }
        double fx0 = (mx - ex) / tile_size, fx1 = (mx + ex) / tile_size;
        double fy0 = (my - ey) / tile_size, fy1 = (my + ey) / tile_size;
        if (near_integer(fx0, 1e-9) || near_integer(fx1, 1e-9) || near_integer(fy0, 1e-9) || near_integer(fy1, 1e-9))
            fl |= ORC_AMBIG_RECT;
        double x0 = floor(fx0), x1 = floor(fx1) + 1.0, y0 = floor(fy0), y1 = floor(fy1) + 1.0;
        x0 = fmin(fmax(x0, 0.0), tiles_x); x1 = fmin(fmax(x1, 0.0), tiles_x);
        y0 = fmin(fmax(y0, 0.0), tiles_y); y1 = fmin(fmax(y1, 0.0), tiles_y);
        if (!(x1 > x0 && y1 > y0)) { flags[g] = fl; continue; }
        rect[4 * g] = (int32_t)x0; rect[4 * g + 1] = (int32_t)y0;
        rect[4 * g + 2] = (int32_t)x1; rect[4 * g + 3] = (int32_t)y1;
        fl |= ORC_VISIBLE;
        flags[g] = fl;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Compositing: the per-pixel definition.                                   */
/* ------------------------------------------------------------------------ */

typedef struct { float key; uint32_t gid; } ord_t;

static int ord_cmp(const void* a, const void* b) {
    const ord_t* x = (const ord_t*)a;
    const ord_t* y = (const ord_t*)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->gid > y->gid) - (x->gid < y->gid);
}

/* Traverse one pixel over an ordered candidate list (front to back). */
static void composite_pixel(const ord_t* list, int64_t len, int64_t pos_base, double px, double py,
                            const double* mean2d, const double* conic, const double* opacity,
                            const double* rgb, const uint8_t* gflags, const double* bg,
                            double* out_rgb, double* out_alpha, int64_t* out_last_gid,
                            int64_t* out_last_pos, int32_t* out_ncontrib, int32_t* out_nvisit,
                            int32_t* out_nsupport, uint8_t* out_flags) {
    double T = 1.0, C[3] = {0.0, 0.0, 0.0};
    int64_t last_gid = -1, last_pos = -1;
    int32_t ncontrib = 0, nvisit = 0, nsupport = 0;
    uint8_t pf = 0;
    for (int64_t i = 0; i < len; ++i) {
        uint32_t g = list[i].gid;
        nvisit++;
        double dx = mean2d[2 * g] - px, dy = mean2d[2 * g + 1] - py;
        double a = conic[3 * g], b = conic[3 * g + 1], c = conic[3 * g + 2];
        double q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy;
        double power = -0.5 * q;
        if (power > 0.0) { pf |= PIX_POWER_POS; continue; }
        double araw = opacity[g] * exp(power);
        /* rounding bound of a binary32 evaluation of q, in q units */
        double qerr = 2e-6 * (fabs(a) * dx * dx + 2.0 * fabs(b * dx * dy) + fabs(c) * dy * dy) + 2e-6;
        double margin = log(araw * 255.0);
        if (fabs(margin) < 0.5 * qerr + 2e-5) {
            pf |= PIX_AMBIG_ALPHA;
            if (gflags && (gflags[g] & (ORC_AMBIG_RECT | ORC_AMBIG_DEPTH | ORC_AMBIG_VIS))) pf |= PIX_AMBIG_GAUSS;
        }
        if (araw < ALPHA_MIN) continue;
        if (gflags && (gflags[g] & (ORC_AMBIG_RECT | ORC_AMBIG_DEPTH | ORC_AMBIG_VIS))) pf |= PIX_AMBIG_GAUSS;
        double alpha = fmin(ALPHA_MAX, araw);
        nsupport++;
        double test = T * (1.0 - alpha);
        if (fabs(test / T_MIN - 1.0) < 2e-4) pf |= PIX_AMBIG_STOP;
        if (test < T_MIN) break;
        for (int ch = 0; ch < 3; ++ch) C[ch] += T * alpha * rgb[3 * g + ch];
        T = test;
        last_gid = g;
        last_pos = pos_base + i;
        ncontrib++;
    }
    for (int ch = 0; ch < 3; ++ch) out_rgb[ch] = C[ch] + T * bg[ch];
    *out_alpha = 1.0 - T;
    *out_last_gid = last_gid;
    *out_last_pos = last_pos;
    *out_ncontrib = ncontrib;
    *out_nvisit = nvisit;
    *out_nsupport = nsupport;
    *out_flags = pf;
}

/*
 * Input check of the tiled entry points: every non-empty rect of a Gaussian
 * that counts (gflags NULL, or ORC_VISIBLE set) lies inside the tiles_x x
 * tiles_y grid, and every listed pixel inside the image. A rect in another
 * tile size's units would otherwise index past the tile lists.
 */
static int rects_in_grid(int64_t n, const int32_t* rect, const uint8_t* gflags, int tiles_x, int tiles_y) {
    for (int64_t g = 0; g < n; ++g) {
        if (gflags && !(gflags[g] & ORC_VISIBLE)) continue;
        const int32_t* r = rect + 4 * g;
        if (r[2] <= r[0] || r[3] <= r[1]) continue;
        if (r[0] < 0 || r[1] < 0 || r[2] > tiles_x || r[3] > tiles_y) return 0;
    }
    return 1;
}

static int pixels_in_image(int64_t npix, const int32_t* pix, int width, int height) {
    for (int64_t p = 0; pix && p < npix; ++p)
        if (pix[2 * p] < 0 || pix[2 * p] >= width || pix[2 * p + 1] < 0 || pix[2 * p + 1] >= height) return 0;
    return 1;
}

/*
 * Render the pixels listed in pix ([npix][2] as x, y; NULL = every pixel,
 * row-major). With rect != NULL ("tiled"), each pixel walks the ordered list
 * of its tile (Gaussians whose half-open tile rect contains the tile), and
 * last_pos is the position in the concatenation of the tile lists in
 * row-major tile order. With rect == NULL ("brute"), each pixel considers
 * every Gaussian with ORC_VISIBLE set; nvisit and last_pos are -1 there.
 * Every Gaussian is assumed valid when gflags is NULL.
 */
ORC_EXPORT int orc_render(int64_t n, const double* mean2d, const double* conic, const double* opacity,
                          const double* rgb, const float* depth_key, const int32_t* rect,
                          const uint8_t* gflags, int width, int height, int tile_size,
                          const double* bg, int64_t npix, const int32_t* pix, double* out_rgb,
                          double* out_alpha, int64_t* out_last_gid, int64_t* out_last_pos,
                          int32_t* out_ncontrib, int32_t* out_nvisit, int32_t* out_nsupport,
                          uint8_t* out_flags) {
    if (n < 0 || width <= 0 || height <= 0 || tile_size <= 0) return 1;
    const int64_t P = pix ? npix : (int64_t)width * height;
    const int tiles_x = (width + tile_size - 1) / tile_size;
    const int tiles_y = (height + tile_size - 1) / tile_size;
    const int64_t T = (int64_t)tiles_x * tiles_y;
    if (!pixels_in_image(npix, pix, width, height)) return 1;

    if (rect) {
        if (!rects_in_grid(n, rect, gflags, tiles_x, tiles_y)) return 1;
        /* tile lists in CSR form */
        int64_t* off = (int64_t*)calloc((size_t)T + 1, sizeof(int64_t));
        if (!off) return 2;
        for (int64_t g = 0; g < n; ++g) {
            if (gflags && !(gflags[g] & ORC_VISIBLE)) continue;
            for (int y = rect[4 * g + 1]; y < rect[4 * g + 3]; ++y)
                for (int x = rect[4 * g]; x < rect[4 * g + 2]; ++x) off[(int64_t)y * tiles_x + x + 1]++;
        }
        for (int64_t t = 0; t < T; ++t) off[t + 1] += off[t];
        int64_t M = off[T];
        ord_t* lists = (ord_t*)malloc((size_t)(M > 0 ? M : 1) * sizeof(ord_t));
        int64_t* cur = (int64_t*)malloc((size_t)(T > 0 ? T : 1) * sizeof(int64_t));
        if (!lists || !cur) { free(off); free(lists); free(cur); return 2; }
        memcpy(cur, off, (size_t)T * sizeof(int64_t));
        for (int64_t g = 0; g < n; ++g) {
            if (gflags && !(gflags[g] & ORC_VISIBLE)) continue;
            for (int y = rect[4 * g + 1]; y < rect[4 * g + 3]; ++y)
                for (int x = rect[4 * g]; x < rect[4 * g + 2]; ++x) {
                    int64_t t = (int64_t)y * tiles_x + x;
                    lists[cur[t]].key = depth_key[g];
                    lists[cur[t]].gid = (uint32_t)g;
                    cur[t]++;
                }
        }
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t t = 0; t < T; ++t)
            qsort(lists + off[t], (size_t)(off[t + 1] - off[t]), sizeof(ord_t), ord_cmp);
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t p = 0; p < P; ++p) {
            int x = pix ? pix[2 * p] : (int)(p % width);
            int y = pix ? pix[2 * p + 1] : (int)(p / width);
            int64_t t = (int64_t)(y / tile_size) * tiles_x + x / tile_size;
            composite_pixel(lists + off[t], off[t + 1] - off[t], off[t], x + 0.5, y + 0.5, mean2d, conic,
                            opacity, rgb, gflags, bg, out_rgb + 3 * p, out_alpha + p, out_last_gid + p,
                            out_last_pos + p, out_ncontrib + p, out_nvisit + p, out_nsupport + p,
                            out_flags + p);
        }
        free(off);
        free(lists);
        free(cur);
        return 0;
    }

    /* brute force: every visible Gaussian, sorted per pixel */
    int err = 0;
#pragma omp parallel
    {
        ord_t* list = (ord_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(ord_t));
        if (!list) {
#pragma omp atomic write
            err = 2;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < P; ++p) {
            if (!list) continue;
            int x = pix ? pix[2 * p] : (int)(p % width);
            int y = pix ? pix[2 * p + 1] : (int)(p / width);
            double px = x + 0.5, py = y + 0.5;
            int64_t len = 0;
            for (int64_t g = 0; g < n; ++g) {
                if (gflags && !(gflags[g] & ORC_VISIBLE)) continue;
                double dx = mean2d[2 * g] - px, dy = mean2d[2 * g + 1] - py;
                double q = conic[3 * g] * dx * dx + 2.0 * conic[3 * g + 1] * dx * dy + conic[3 * g + 2] * dy * dy;
                /* keep a slightly larger set than the alpha support so that the
                   near-threshold flags are raised exactly as in tiled mode */
                if (opacity[g] * exp(-0.5 * q) < ALPHA_MIN * 0.999) continue;
                list[len].key = depth_key[g];
                list[len].gid = (uint32_t)g;
                len++;
            }
            qsort(list, (size_t)len, sizeof(ord_t), ord_cmp);
            composite_pixel(list, len, 0, px, py, mean2d, conic, opacity, rgb, gflags, bg,
                            out_rgb + 3 * p, out_alpha + p, out_last_gid + p, out_last_pos + p,
                            out_ncontrib + p, out_nvisit + p, out_nsupport + p, out_flags + p);
            out_nvisit[p] = -1;
            out_last_pos[p] = -1;
        }
        free(list);
    }
    return err;
}

/*
 * Render over a given per-tile traversal order instead of the depth order:
 * tile t's pixels walk ids[tile_offsets[t] .. tile_offsets[t+1]) front to
 * back in the order listed (the binned order of a schedule whose bins are
 * not monotone in the depth, section "Repair for correctness"). Same outputs
 * as orc_render in tiled mode; last_pos is the position in ids.
 */
ORC_EXPORT int orc_render_stream(int64_t n, const double* mean2d, const double* conic, const double* opacity,
                                 const double* rgb, const uint8_t* gflags, int width, int height, int tile_size,
                                 const double* bg, const uint32_t* tile_offsets, const uint32_t* ids, int64_t npix,
                                 const int32_t* pix, double* out_rgb, double* out_alpha, int64_t* out_last_gid,
                                 int64_t* out_last_pos, int32_t* out_ncontrib, int32_t* out_nvisit,
                                 int32_t* out_nsupport, uint8_t* out_flags) {
    if (n < 0 || width <= 0 || height <= 0 || tile_size <= 0) return 1;
    const int64_t P = pix ? npix : (int64_t)width * height;
    const int tiles_x = (width + tile_size - 1) / tile_size;
    const int tiles_y = (height + tile_size - 1) / tile_size;
    const int64_t T = (int64_t)tiles_x * tiles_y;
    const int64_t M = tile_offsets[T];
    if (!pixels_in_image(npix, pix, width, height)) return 1;
    ord_t* lists = (ord_t*)malloc((size_t)(M > 0 ? M : 1) * sizeof(ord_t));
    if (!lists) return 2;
    for (int64_t i = 0; i < M; ++i) {
        if (ids[i] >= (uint64_t)n) { free(lists); return 1; }
        lists[i].key = 0.0f;
        lists[i].gid = ids[i];
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < P; ++p) {
        int x = pix ? pix[2 * p] : (int)(p % width);
        int y = pix ? pix[2 * p + 1] : (int)(p / width);
        int64_t t = (int64_t)(y / tile_size) * tiles_x + x / tile_size;
        composite_pixel(lists + tile_offsets[t], (int64_t)tile_offsets[t + 1] - tile_offsets[t], tile_offsets[t],
                        x + 0.5, y + 0.5, mean2d, conic, opacity, rgb, gflags, bg, out_rgb + 3 * p,
                        out_alpha + p, out_last_gid + p, out_last_pos + p, out_ncontrib + p, out_nvisit + p,
                        out_nsupport + p, out_flags + p);
    }
    free(lists);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Integer schedule: keys, global order, depth range, bins, offsets.        */
/* ------------------------------------------------------------------------ */

static uint32_t f32_bits(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* Number of (Gaussian, tile) entries: the sum of the rect areas. */
ORC_EXPORT int64_t orc_count_entries(int64_t n, const int32_t* rect) {
    int64_t M = 0;
    for (int64_t g = 0; g < n; ++g) {
        int64_t w = rect[4 * g + 2] - rect[4 * g], h = rect[4 * g + 3] - rect[4 * g + 1];
        if (w > 0 && h > 0) M += w * h;
    }
    return M;
}

typedef struct { uint64_t key; uint32_t gid; } kv_t;

static int kv_cmp(const void* a, const void* b) {
    const kv_t* x = (const kv_t*)a;
    const kv_t* y = (const kv_t*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->gid > y->gid) - (x->gid < y->gid);
}

static int u32_cmp(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return (x > y) - (x < y);
}

static int u64_cmp(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

/*
 * Robust depth range (supplement, Algorithm "Robust depth-range estimation"),
 * without the near-depth shift: sample the depths of the visible Gaussians
 * (non-empty rect), take the exact order statistics at the p_lo / p_hi
 * percentiles, pad by pad * span and clamp to [znear, zfar].
 * Readings: with V visible Gaussians and S samples, all are taken when
 * V <= S, otherwise the visible Gaussians at ranks floor(i V / S) of the
 * ascending id list; the order statistics are the 0-based ranks
 * floor(p_lo/100 (n-1)) and ceil(p_hi/100 (n-1)); the arithmetic after the
 * selection is binary32 without contraction.
 */
ORC_EXPORT int orc_depth_range(int64_t n, const float* depth, const int32_t* rect, int S, double p_lo,
                               double p_hi, float pad, float znear, float zfar, float* zrange) {
    int64_t V = 0;
    for (int64_t g = 0; g < n; ++g)
        if (rect[4 * g + 2] > rect[4 * g] && rect[4 * g + 3] > rect[4 * g + 1]) V++;
    if (V == 0) { zrange[0] = znear; zrange[1] = zfar; return 0; }
    int64_t* vis = (int64_t*)malloc((size_t)V * sizeof(int64_t));
    if (!vis) return 2;
    int64_t k = 0;
    for (int64_t g = 0; g < n; ++g)
        if (rect[4 * g + 2] > rect[4 * g] && rect[4 * g + 3] > rect[4 * g + 1]) vis[k++] = g;
    int64_t ns = V <= S ? V : S;
    uint32_t* sample = (uint32_t*)malloc((size_t)ns * sizeof(uint32_t));
    if (!sample) { free(vis); return 2; }
    for (int64_t i = 0; i < ns; ++i) {
        int64_t r = V <= S ? i : (i * V) / S;
        sample[i] = f32_bits(depth[vis[r]]);
    }
    qsort(sample, (size_t)ns, sizeof(uint32_t), u32_cmp);
    int64_t klo = (int64_t)floor(p_lo / 100.0 * (double)(ns - 1));
    int64_t khi = (int64_t)ceil(p_hi / 100.0 * (double)(ns - 1));
    if (klo < 0) klo = 0;
    if (khi > ns - 1) khi = ns - 1;
    float zlo, zhi;
    memcpy(&zlo, &sample[klo], 4);
    memcpy(&zhi, &sample[khi], 4);
    volatile float diff = zhi - zlo;
    float span = diff > 1e-6f ? diff : 1e-6f;
    volatile float padv = pad * span;
    volatile float lo = zlo - padv;
    volatile float hi = zhi + padv;
    zrange[0] = lo > znear ? lo : znear;
    zrange[1] = hi < zfar ? hi : zfar;
    free(sample);
    free(vis);
    return 0;
}

/*
 * Log-depth bin of a binary32 depth: the paper's clamped log-space map
 * floor(K u), u = (log z - log zmin) / (log zmax - log zmin), realised with
 * the IEEE-754 bit pattern as the logarithm (a monotone piecewise-linear
 * log2), evaluated exactly in integers.
 */
static int bin_of(float z, float zmin, float zmax, int K) {
    int64_t L = f32_bits(z), Lmin = f32_bits(zmin), Lmax = f32_bits(zmax);
    if (Lmax <= Lmin || L <= Lmin) return 0;
    if (L >= Lmax) return K - 1;
    int64_t b = ((int64_t)K * (L - Lmin)) / (Lmax - Lmin);
    return b > K - 1 ? K - 1 : (int)b;
}

ORC_EXPORT int orc_bin_of(float z, float zmin, float zmax, int K) { return bin_of(z, zmin, zmax, K); }

/*
 * The whole integer schedule for binary32 depths and tile rects.
 * keys/vals: the global list, sorted by (tile << 32 | depth bits, id).
 * tile_offsets[T+1]: each tile's range in it.
 * zrange[2]: the depth range.
 * Bins: tile t has K_t = per_tile_bins[t] bins (per_tile_bins NULL: K in
 * every tile); its segments are numbered from seg_base[t] = K_0 + ... +
 * K_{t-1}, so segment seg_base[t] + b is bin b of tile t (tile-major,
 * bin-minor; with a uniform K this is t K + b). bin_offsets[sum K_t + 1]:
 * exclusive scan of the segment counts (supplement, Algorithm "Tile-local
 * bin construction"); seg_base[T+1].
 * stream[M]: the tile-bin-major stream with every (tile, bin) segment sorted
 * by (depth bits << 32 | id), the exact-repair order.
 * Any output pointer may be NULL.
 */
static int schedule_impl(int64_t n, const float* depth, const float* bin_depth, const int32_t* rect, int tiles_x,
                         int tiles_y, int K,
                         const int32_t* per_tile_bins, int S, double p_lo, double p_hi, float pad, float znear,
                         float zfar, uint64_t* keys, uint32_t* vals, uint32_t* tile_offsets, float* zrange,
                         uint32_t* seg_base_out, uint32_t* bin_offsets, uint64_t* stream) {
    const int64_t T = (int64_t)tiles_x * tiles_y;
    if (tiles_x <= 0 || tiles_y <= 0 || !rects_in_grid(n, rect, NULL, tiles_x, tiles_y)) return 1;
    const int64_t M = orc_count_entries(n, rect);
    kv_t* e = (kv_t*)malloc((size_t)(M > 0 ? M : 1) * sizeof(kv_t));
    int64_t* sb = (int64_t*)malloc(((size_t)T + 1) * sizeof(int64_t));
    if (!e || !sb) { free(e); free(sb); return 2; }
    sb[0] = 0;
    for (int64_t t = 0; t < T; ++t) sb[t + 1] = sb[t] + (per_tile_bins ? per_tile_bins[t] : K);
    if (seg_base_out)
        for (int64_t t = 0; t <= T; ++t) seg_base_out[t] = (uint32_t)sb[t];
    int64_t m = 0;
    for (int64_t g = 0; g < n; ++g)
        for (int y = rect[4 * g + 1]; y < rect[4 * g + 3]; ++y)
            for (int x = rect[4 * g]; x < rect[4 * g + 2]; ++x) {
                uint64_t t = (uint64_t)y * tiles_x + x;
                e[m].key = (t << 32) | f32_bits(depth[g]);
                e[m].gid = (uint32_t)g;
                m++;
            }
    qsort(e, (size_t)M, sizeof(kv_t), kv_cmp);
    if (keys)
        for (int64_t i = 0; i < M; ++i) keys[i] = e[i].key;
    if (vals)
        for (int64_t i = 0; i < M; ++i) vals[i] = e[i].gid;
    if (tile_offsets) {
        int64_t i = 0;
        for (int64_t t = 0; t <= T; ++t) {
            while (i < M && (int64_t)(e[i].key >> 32) < t) i++;
            tile_offsets[t] = (uint32_t)i;
        }
    }
    float zr[2];
    const float* bd = bin_depth ? bin_depth : depth;
    int rc = orc_depth_range(n, bd, rect, S, p_lo, p_hi, pad, znear, zfar, zr);
    if (rc) { free(e); free(sb); return rc; }
    if (zrange) { zrange[0] = zr[0]; zrange[1] = zr[1]; }
    if (bin_offsets || stream) {
        const int64_t NS = sb[T];
        uint32_t* cnt = (uint32_t*)calloc((size_t)NS + 1, sizeof(uint32_t));
        uint32_t* off = (uint32_t*)malloc(((size_t)NS + 1) * sizeof(uint32_t));
        uint32_t* cur = (uint32_t*)malloc(((size_t)NS + 1) * sizeof(uint32_t));
        uint64_t* st = (uint64_t*)malloc((size_t)(M > 0 ? M : 1) * sizeof(uint64_t));
        if (!cnt || !off || !cur || !st) { free(cnt); free(off); free(cur); free(st); free(e); free(sb); return 2; }
        /* count in emission order (the order is irrelevant for counts) */
        for (int64_t g = 0; g < n; ++g)
            for (int y = rect[4 * g + 1]; y < rect[4 * g + 3]; ++y)
                for (int x = rect[4 * g]; x < rect[4 * g + 2]; ++x) {
                    const int64_t t = (int64_t)y * tiles_x + x;
                    cnt[sb[t] + bin_of(bd[g], zr[0], zr[1], (int)(sb[t + 1] - sb[t]))]++;
                }
        off[0] = 0;
        for (int64_t s2 = 0; s2 < NS; ++s2) off[s2 + 1] = off[s2] + cnt[s2];
        memcpy(cur, off, ((size_t)NS + 1) * sizeof(uint32_t));
        for (int64_t g = 0; g < n; ++g)
            for (int y = rect[4 * g + 1]; y < rect[4 * g + 3]; ++y)
                for (int x = rect[4 * g]; x < rect[4 * g + 2]; ++x) {
                    const int64_t t = (int64_t)y * tiles_x + x;
                    const int64_t s2 = sb[t] + bin_of(bd[g], zr[0], zr[1], (int)(sb[t + 1] - sb[t]));
                    st[cur[s2]++] = ((uint64_t)f32_bits(depth[g]) << 32) | (uint64_t)g;
                }
        for (int64_t s2 = 0; s2 < NS; ++s2)
            qsort(st + off[s2], (size_t)(off[s2 + 1] - off[s2]), sizeof(uint64_t), u64_cmp);
        if (bin_offsets) memcpy(bin_offsets, off, ((size_t)NS + 1) * sizeof(uint32_t));
        if (stream) memcpy(stream, st, (size_t)M * sizeof(uint64_t));
        free(cnt); free(off); free(cur); free(st);
    }
    free(e);
    free(sb);
    return 0;
}

/*
 * Near-depth binning key (supplement, Algorithm "Robust depth-range
 * estimation", near-depth mode; the tile-local bin map takes the same key):
 * z_key = z - min(alpha s_max, gamma z), with s_max the Gaussian's largest
 * axis scale (world units). Binary32 arithmetic without contraction, the
 * minimum taken as (a < b ? a : b). Readings: s_max is the largest of the
 * three activated scales exp(log_scale); the clamp "using the near/far planes
 * and epsilon" is to [max(znear, 1e-4), zfar]; with gamma < 1 every key of a
 * visible Gaussian is positive, so the discard of keys <= 0 never applies.
 */
static float near_key(float z, float smax, float alpha, float gamma, float znear, float zfar) {
    volatile float a = alpha * smax;
    volatile float b = gamma * z;
    float d = a < b ? a : b;
    volatile float k = z - d;
    float lo = znear > 1e-4f ? znear : 1e-4f;
    float v = k;
    if (v < lo) v = lo;
    if (v > zfar) v = zfar;
    return v;
}

ORC_EXPORT void orc_near_keys(int64_t n, const float* depth, const float* smax, float alpha, float gamma,
                              float znear, float zfar, float* out) {
    for (int64_t g = 0; g < n; ++g) out[g] = near_key(depth[g], smax[g], alpha, gamma, znear, zfar);
}

/*
 * The binned schedule when bins are formed on another per-Gaussian key
 * (bin_depth, e.g. the near-depth key) than the depth the baseline sorts by:
 * the depth range is sampled from bin_depth and each entry's bin is that of
 * its bin_depth, while the stream entries stay (depth bits << 32 | id) and
 * each segment is sorted by them. bin_offsets[T*K+1], stream[M].
 */
ORC_EXPORT int orc_schedule_keyed(int64_t n, const float* depth, const float* bin_depth, const int32_t* rect,
                                  int tiles_x, int tiles_y, int K, int S, double p_lo, double p_hi, float pad,
                                  float znear, float zfar, float* zrange, uint32_t* bin_offsets, uint64_t* stream) {
    return schedule_impl(n, depth, bin_depth, rect, tiles_x, tiles_y, K, NULL, S, p_lo, p_hi, pad, znear, zfar,
                         NULL, NULL, NULL, zrange, NULL, bin_offsets, stream);
}

/*
 * Selective repair selection (Table "Exact-repair selection rules" and the
 * supplement's Algorithm "Selective repair selection and local exact
 * sorting"): segments q = t K + b are visited in that order; a segment of
 * length l >= 2 in a tile of l_tile entries is kept when any of
 *   (i) l >= 320, (ii) l > 512, (iii) l / l_tile >= 45 %,
 *   (iv) 129 <= l <= 256 and l / l_tile >= 10 %, (v) b < 2 and l >= 16
 * holds, and a kept segment is selected when used + l <= B, B =
 * floor(budget_frac M), after which used grows by l (first fit). Reading:
 * the shares are compared in integers, 100 l >= 45 l_tile and 100 l >= 10
 * l_tile. selected[T*K] gets 1 / 0; returns the selected entries (used).
 */
ORC_EXPORT int64_t orc_repair_select(int64_t T, int K, const uint32_t* bin_offsets, double budget_frac,
                                     uint8_t* selected) {
    const int64_t M = bin_offsets[T * K];
    const int64_t B = (int64_t)floor(budget_frac * (double)M);
    int64_t used = 0;
    for (int64_t t = 0; t < T; ++t) {
        const int64_t tile_len = (int64_t)bin_offsets[t * K + K] - bin_offsets[t * K];
        for (int b = 0; b < K; ++b) {
            const int64_t q = t * K + b;
            const int64_t len = (int64_t)bin_offsets[q + 1] - bin_offsets[q];
            selected[q] = 0;
            if (len <= 1) continue;
            int keep = 0;
            if (len >= 320) keep = 1;                                    /* (i) */
            if (len > 512) keep = 1;                                     /* (ii) */
            if (100 * len >= 45 * tile_len) keep = 1;                    /* (iii) */
            if (len >= 129 && len <= 256 && 100 * len >= 10 * tile_len) keep = 1; /* (iv) */
            if (b < 2 && len >= 16) keep = 1;                            /* (v) */
            if (keep && used + len <= B) {
                selected[q] = 1;
                used += len;
            }
        }
    }
    return used;
}

/* The schedule with K bins in every tile (bin_offsets[T*K+1]). */
ORC_EXPORT int orc_schedule(int64_t n, const float* depth, const int32_t* rect, int tiles_x, int tiles_y,
                            int K, int S, double p_lo, double p_hi, float pad, float znear, float zfar,
                            uint64_t* keys, uint32_t* vals, uint32_t* tile_offsets, float* zrange,
                            uint32_t* bin_offsets, uint64_t* stream) {
    return schedule_impl(n, depth, NULL, rect, tiles_x, tiles_y, K, NULL, S, p_lo, p_hi, pad, znear, zfar, keys, vals,
                         tile_offsets, zrange, NULL, bin_offsets, stream);
}

/* The schedule with per_tile_bins[t] bins in tile t (each >= 1). */
ORC_EXPORT int orc_schedule_tiles(int64_t n, const float* depth, const int32_t* rect, int tiles_x, int tiles_y,
                                  const int32_t* per_tile_bins, int S, double p_lo, double p_hi, float pad,
                                  float znear, float zfar, float* zrange, uint32_t* seg_base,
                                  uint32_t* bin_offsets, uint64_t* stream) {
    const int64_t T = (int64_t)tiles_x * tiles_y;
    for (int64_t t = 0; t < T; ++t)
        if (per_tile_bins[t] < 1) return 1;
    return schedule_impl(n, depth, NULL, rect, tiles_x, tiles_y, 0, per_tile_bins, S, p_lo, p_hi, pad, znear, zfar, NULL,
                         NULL, NULL, zrange, seg_base, bin_offsets, stream);
}

/* ------------------------------------------------------------------------ */
/* Adjoint: the gradient of a scalar loss of the image with respect to the  */
/* Gaussian parameters. The paper leaves the backward pass to future work   */
/* (Conclusion / Limitations); this is the derivative of the forward model  */
/* above, written out by the chain rule in binary64 and taken in reverse    */
/* order (compositing first, then the projection). Inputs are binary64 so   */
/* that central finite differences of the same forward model can check it.  */
/* Zero-gradient paths, as in the forward definition: the 0.99 alpha cap,   */
/* colour channels clamped at 0, the frustum guard of the Jacobian, and     */
/* Gaussians that are skipped, culled or after the stopping point.          */
/* ------------------------------------------------------------------------ */

/* The forward quantities of one Gaussian that its adjoint needs. */
typedef struct {
    int vis;
    double mu[3], pc[3], z;
    double qn, qh[4];      /* |q| and q / |q| as (w, x, y, z) */
    double s2[3], M[9];    /* exp(log_scale)^2, R_cam R_q */
    int clx, cly;          /* frustum guard active on x / y */
    double limx, limy;     /* signed guard value when active */
    double j00, j02, j11, j12;
    double A[3], B[3];     /* rows of J M */
    double c00, c01, c11, det;
    double conic[3], mean[2], o;
    double dir[3], Y[16];
    double rgb[3], rgb_raw[3];
    int rect[4];
    float key;
} adj_g;

static void adj_project_one(const double* means, const double* log_scales, const double* quats,
                            const double* logits, const double* sh, int nsh, int degree, const double* cam,
                            int tile_size, int64_t g, adj_g* P) {
    const double* R = cam;
    const double* t = cam + 9;
    const double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    const int W = (int)cam[16], H = (int)cam[17];
    memset(P, 0, sizeof(*P));
    for (int i = 0; i < 3; ++i) P->mu[i] = means[3 * g + i];
    for (int i = 0; i < 3; ++i)
        P->pc[i] = R[3 * i] * P->mu[0] + R[3 * i + 1] * P->mu[1] + R[3 * i + 2] * P->mu[2] + t[i];
    const double z = P->z = P->pc[2];
    if (!(z > cam[18] && z < cam[19])) return;
    const double* q = quats + 4 * g;
    P->qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(P->qn > 0.0) || !isfinite(P->qn)) return;
    for (int i = 0; i < 4; ++i) P->qh[i] = q[i] / P->qn;
    const double w = P->qh[0], x = P->qh[1], y = P->qh[2], zq = P->qh[3];
    const double Rq[9] = {1 - 2 * (y * y + zq * zq), 2 * (x * y - w * zq), 2 * (x * zq + w * y),
                          2 * (x * y + w * zq), 1 - 2 * (x * x + zq * zq), 2 * (y * zq - w * x),
                          2 * (x * zq - w * y), 2 * (y * zq + w * x), 1 - 2 * (x * x + y * y)};
    for (int k = 0; k < 3; ++k) {
        double s = exp(log_scales[3 * g + k]);
        P->s2[k] = s * s;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            P->M[3 * i + j] = R[3 * i] * Rq[j] + R[3 * i + 1] * Rq[3 + j] + R[3 * i + 2] * Rq[6 + j];
    const double tanx = 0.5 * W / fx, tany = 0.5 * H / fy;
    const double lxp = (W - cx) / fx + GUARD * tanx, lxn = cx / fx + GUARD * tanx;
    const double lyp = (H - cy) / fy + GUARD * tany, lyn = cy / fy + GUARD * tany;
    double tx = P->pc[0], ty = P->pc[1];
    if (P->pc[0] / z > lxp) { P->clx = 1; P->limx = lxp; tx = z * lxp; }
    else if (P->pc[0] / z < -lxn) { P->clx = 1; P->limx = -lxn; tx = -z * lxn; }
    if (P->pc[1] / z > lyp) { P->cly = 1; P->limy = lyp; ty = z * lyp; }
    else if (P->pc[1] / z < -lyn) { P->cly = 1; P->limy = -lyn; ty = -z * lyn; }
    P->j00 = fx / z; P->j02 = -fx * tx / (z * z);
    P->j11 = fy / z; P->j12 = -fy * ty / (z * z);
    for (int k = 0; k < 3; ++k) {
        P->A[k] = P->j00 * P->M[k] + P->j02 * P->M[6 + k];
        P->B[k] = P->j11 * P->M[3 + k] + P->j12 * P->M[6 + k];
    }
    P->c00 = DILATION; P->c01 = 0.0; P->c11 = DILATION;
    for (int k = 0; k < 3; ++k) {
        P->c00 += P->A[k] * P->A[k] * P->s2[k];
        P->c01 += P->A[k] * P->B[k] * P->s2[k];
        P->c11 += P->B[k] * P->B[k] * P->s2[k];
    }
    P->det = P->c00 * P->c11 - P->c01 * P->c01;
    if (!(P->det > 0.0) || !isfinite(P->det)) return;
    P->conic[0] = P->c11 / P->det;
    P->conic[1] = -P->c01 / P->det;
    P->conic[2] = P->c00 / P->det;
    P->mean[0] = fx * P->pc[0] / z + cx;
    P->mean[1] = fy * P->pc[1] / z + cy;
    P->o = 1.0 / (1.0 + exp(-logits[g]));
    if (!(P->o >= ALPHA_MIN)) return;
    for (int i = 0; i < 3; ++i) P->dir[i] = P->mu[i] + (R[i] * t[0] + R[3 + i] * t[1] + R[6 + i] * t[2]);
    orc_sh_basis(P->dir, degree, P->Y);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int k = 0; k < nsh; ++k) acc += sh[((int64_t)g * nsh + k) * 3 + ch] * P->Y[k];
        P->rgb_raw[ch] = 0.5 + acc;
        P->rgb[ch] = fmax(0.0, P->rgb_raw[ch]);
    }
    const double tau = 2.0 * log(255.0 * P->o);
    const double ex = sqrt(tau * P->c00) * (1.0 + 1e-4) + 1e-3, ey = sqrt(tau * P->c11) * (1.0 + 1e-4) + 1e-3;
    const int tiles_x = (W + tile_size - 1) / tile_size, tiles_y = (H + tile_size - 1) / tile_size;
    double x0 = floor((P->mean[0] - ex) / tile_size), x1 = floor((P->mean[0] + ex) / tile_size) + 1.0;
    double y0 = floor((P->mean[1] - ey) / tile_size), y1 = floor((P->mean[1] + ey) / tile_size) + 1.0;
    x0 = fmin(fmax(x0, 0.0), tiles_x); x1 = fmin(fmax(x1, 0.0), tiles_x);
    y0 = fmin(fmax(y0, 0.0), tiles_y); y1 = fmin(fmax(y1, 0.0), tiles_y);
    if (!(x1 > x0 && y1 > y0)) return;
    P->rect[0] = (int)x0; P->rect[1] = (int)y0; P->rect[2] = (int)x1; P->rect[3] = (int)y1;
    P->key = (float)z;
    P->vis = 1;
}

/* One composited entry of a pixel: Gaussian, its alpha, the transmittance
   in front of it, exp(-q/2), and whether the 0.99 cap was active. */
typedef struct { uint32_t g; double alpha, T, G, dx, dy; int capped; } adj_c;

/* Compositing adjoint of one pixel: given dL/d(rgb) (gc) and dL/d(alpha)
   (ga) of the pixel, accumulate dL/d(mean2d, conic, opacity, rgb) of every
   composited Gaussian into gm[9 g + 0..8]. The colour behind entry k,
   S_k = sum_{i > k} T_i alpha_i c_i + T_final bg, gives
   dC/d alpha_k = T_k c_k - S_k / (1 - alpha_k) and
   d(1 - T_final)/d alpha_k = T_final / (1 - alpha_k). */
static void adj_pixel_reverse(const adj_g* P, const adj_c* cl, int nc, double Tf, const double* bg,
                              const double* gc, double ga, double* gm) {
    double S[3] = {Tf * bg[0], Tf * bg[1], Tf * bg[2]};
    for (int k = nc - 1; k >= 0; --k) {
        const uint32_t g = cl[k].g;
        const double a = cl[k].alpha, Tk = cl[k].T;
        double dLda = ga * Tf / (1.0 - a);
        for (int ch = 0; ch < 3; ++ch) {
            gm[9 * g + 6 + ch] += gc[ch] * Tk * a;
            dLda += gc[ch] * (Tk * P[g].rgb[ch] - S[ch] / (1.0 - a));
        }
        for (int ch = 0; ch < 3; ++ch) S[ch] += Tk * a * P[g].rgb[ch];
        if (cl[k].capped) continue;
        /* alpha = o G, G = exp(-q/2), q = a dx^2 + 2 b dx dy + c dy^2 */
        const double dLdq = dLda * (-0.5 * a);
        const double dx = cl[k].dx, dy = cl[k].dy;
        gm[9 * g + 5] += dLda * cl[k].G;
        gm[9 * g + 2] += dLdq * dx * dx;
        gm[9 * g + 3] += dLdq * 2.0 * dx * dy;
        gm[9 * g + 4] += dLdq * dy * dy;
        gm[9 * g + 0] += dLdq * 2.0 * (P[g].conic[0] * dx + P[g].conic[1] * dy);
        gm[9 * g + 1] += dLdq * 2.0 * (P[g].conic[1] * dx + P[g].conic[2] * dy);
    }
}

/* Projection adjoint of one Gaussian: from d = dL/d(mean2d x, y, conic a, b,
   c, opacity, r, g, b) to the parameter gradients. The direction derivative
   of the SH basis is a central difference of orc_sh_basis with step
   1e-6 |dir| (truncation and rounding error below 1e-9 relative). */
static void adj_project_reverse(const adj_g* p, const double* d, const double* sh, int nsh, int degree,
                                const double* cam, double* d_means, double* d_log_scales, double* d_quats,
                                double* d_logit, double* d_sh) {
    const double* R = cam;
    const double fx = cam[12], fy = cam[13];
    *d_logit = d[5] * p->o * (1.0 - p->o);
    double gY[16] = {0};
    for (int ch = 0; ch < 3; ++ch) {
        if (!(p->rgb_raw[ch] > 0.0)) continue;
        for (int k = 0; k < nsh; ++k) {
            d_sh[3 * k + ch] = d[6 + ch] * p->Y[k];
            gY[k] += d[6 + ch] * sh[3 * k + ch];
        }
    }
    double gmu[3] = {0, 0, 0};
    const double dn = sqrt(p->dir[0] * p->dir[0] + p->dir[1] * p->dir[1] + p->dir[2] * p->dir[2]);
    const double h = 1e-6 * dn;
    for (int c = 0; c < 3; ++c) {
        double vp[3] = {p->dir[0], p->dir[1], p->dir[2]}, vm[3] = {p->dir[0], p->dir[1], p->dir[2]};
        vp[c] += h;
        vm[c] -= h;
        double Yp[16], Ym[16];
        orc_sh_basis(vp, degree, Yp);
        orc_sh_basis(vm, degree, Ym);
        for (int k = 0; k < nsh; ++k) gmu[c] += gY[k] * (Yp[k] - Ym[k]) / (vp[c] - vm[c]);
    }
    /* conic = [c11, -c01, c00] / det */
    const double a = p->c00, b = p->c01, c = p->c11, det = p->det, d2 = det * det;
    const double gA = d[2], gB = d[3], gC = d[4];
    const double ga = gA * (-c * c / d2) + gB * (b * c / d2) + gC * (-b * b / d2);
    const double gb = gA * (2.0 * b * c / d2) + gB * (-1.0 / det - 2.0 * b * b / d2) + gC * (2.0 * a * b / d2);
    const double gc = gA * (-b * b / d2) + gB * (a * b / d2) + gC * (-a * a / d2);
    /* c00 = sum A_k^2 s2_k + 0.3, c01 = sum A_k B_k s2_k, c11 = sum B_k^2 s2_k + 0.3 */
    double gAr[3], gBr[3];
    for (int k = 0; k < 3; ++k) {
        gAr[k] = 2.0 * ga * p->A[k] * p->s2[k] + gb * p->B[k] * p->s2[k];
        gBr[k] = 2.0 * gc * p->B[k] * p->s2[k] + gb * p->A[k] * p->s2[k];
        const double gs2 = ga * p->A[k] * p->A[k] + gb * p->A[k] * p->B[k] + gc * p->B[k] * p->B[k];
        d_log_scales[k] = gs2 * 2.0 * p->s2[k];
    }
    /* A = j00 M_0 + j02 M_2, B = j11 M_1 + j12 M_2 */
    double gj00 = 0, gj02 = 0, gj11 = 0, gj12 = 0, gM[9];
    for (int k = 0; k < 3; ++k) {
        gj00 += gAr[k] * p->M[k];
        gj02 += gAr[k] * p->M[6 + k];
        gj11 += gBr[k] * p->M[3 + k];
        gj12 += gBr[k] * p->M[6 + k];
        gM[k] = gAr[k] * p->j00;
        gM[3 + k] = gBr[k] * p->j11;
        gM[6 + k] = gAr[k] * p->j02 + gBr[k] * p->j12;
    }
    /* M = R_cam R_q */
    double gRq[9];
    for (int l = 0; l < 3; ++l)
        for (int j = 0; j < 3; ++j) gRq[3 * l + j] = R[l] * gM[j] + R[3 + l] * gM[3 + j] + R[6 + l] * gM[6 + j];
    const double w = p->qh[0], x = p->qh[1], y = p->qh[2], zq = p->qh[3];
    const double dRw[9] = {0, -2 * zq, 2 * y, 2 * zq, 0, -2 * x, -2 * y, 2 * x, 0};
    const double dRx[9] = {0, 2 * y, 2 * zq, 2 * y, -4 * x, -2 * w, 2 * zq, 2 * w, -4 * x};
    const double dRy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * zq, -2 * w, 2 * zq, -4 * y};
    const double dRz[9] = {-4 * zq, -2 * w, 2 * x, 2 * w, -4 * zq, 2 * y, 2 * x, 2 * y, 0};
    double gq[4] = {0, 0, 0, 0};
    for (int k = 0; k < 9; ++k) {
        gq[0] += gRq[k] * dRw[k];
        gq[1] += gRq[k] * dRx[k];
        gq[2] += gRq[k] * dRy[k];
        gq[3] += gRq[k] * dRz[k];
    }
    /* q_hat = q / |q| */
    const double qd = gq[0] * p->qh[0] + gq[1] * p->qh[1] + gq[2] * p->qh[2] + gq[3] * p->qh[3];
    for (int k = 0; k < 4; ++k) d_quats[k] = (gq[k] - qd * p->qh[k]) / p->qn;
    /* the Jacobian entries and the screen mean, as functions of the
       camera-space point */
    const double z = p->z, X = p->pc[0], Yc = p->pc[1];
    double gp[3] = {0, 0, 0};
    gp[2] += gj00 * (-fx / (z * z)) + gj11 * (-fy / (z * z));
    if (p->clx) gp[2] += gj02 * (fx * p->limx / (z * z));
    else { gp[0] += gj02 * (-fx / (z * z)); gp[2] += gj02 * (2.0 * fx * X / (z * z * z)); }
    if (p->cly) gp[2] += gj12 * (fy * p->limy / (z * z));
    else { gp[1] += gj12 * (-fy / (z * z)); gp[2] += gj12 * (2.0 * fy * Yc / (z * z * z)); }
    gp[0] += d[0] * fx / z;
    gp[1] += d[1] * fy / z;
    gp[2] += -d[0] * fx * X / (z * z) - d[1] * fy * Yc / (z * z);
    for (int c2 = 0; c2 < 3; ++c2) d_means[c2] = gmu[c2] + R[c2] * gp[0] + R[3 + c2] * gp[1] + R[6 + c2] * gp[2];
}

/*
 * Tiled compositing of the projected Gaussians P[0..n) (those with vis set),
 * the per-pixel definition of orc_render: the image into out_rgb [H][W][3]
 * and out_alpha [H][W]; with d_img != NULL also dL/d(projected) into d_proj
 * [n][9] (mean2d x, y, conic a, b, c, opacity, r, g, b).
 */
static int adj_composite(const adj_g* P, int64_t n, int W, int H, int tile_size, const double* bg,
                         double* out_rgb, double* out_alpha, const double* d_img, const double* d_alpha,
                         double* d_proj) {
    const int tiles_x = (W + tile_size - 1) / tile_size, tiles_y = (H + tile_size - 1) / tile_size;
    const int64_t T = (int64_t)tiles_x * tiles_y;
    const size_t n1 = (size_t)(n > 0 ? n : 1);
    int64_t* off = (int64_t*)calloc((size_t)T + 1, sizeof(int64_t));
    if (!off) return 2;
    /* ordered tile lists, as in orc_render */
    for (int64_t g = 0; g < n; ++g)
        if (P[g].vis)
            for (int y = P[g].rect[1]; y < P[g].rect[3]; ++y)
                for (int x = P[g].rect[0]; x < P[g].rect[2]; ++x) off[(int64_t)y * tiles_x + x + 1]++;
    for (int64_t t = 0; t < T; ++t) off[t + 1] += off[t];
    ord_t* lists = (ord_t*)malloc((size_t)(off[T] > 0 ? off[T] : 1) * sizeof(ord_t));
    int64_t* cur = (int64_t*)malloc((size_t)(T > 0 ? T : 1) * sizeof(int64_t));
    if (!lists || !cur) { free(off); free(lists); free(cur); return 2; }
    memcpy(cur, off, (size_t)T * sizeof(int64_t));
    for (int64_t g = 0; g < n; ++g)
        if (P[g].vis)
            for (int y = P[g].rect[1]; y < P[g].rect[3]; ++y)
                for (int x = P[g].rect[0]; x < P[g].rect[2]; ++x) {
                    const int64_t t = (int64_t)y * tiles_x + x;
                    lists[cur[t]].key = P[g].key;
                    lists[cur[t]].gid = (uint32_t)g;
                    cur[t]++;
                }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < T; ++t) qsort(lists + off[t], (size_t)(off[t + 1] - off[t]), sizeof(ord_t), ord_cmp);
    int64_t maxlen = 1;
    for (int64_t t = 0; t < T; ++t) if (off[t + 1] - off[t] > maxlen) maxlen = off[t + 1] - off[t];

    /* per-thread accumulators of dL/d(projected), reduced in thread order */
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double* acc = d_img ? (double*)calloc((size_t)nth * n1 * 9, sizeof(double)) : NULL;
    if (d_img && !acc) { free(off); free(lists); free(cur); return 2; }
    int err = 0;
#pragma omp parallel num_threads(nth)
    {
        int me = 0;
#ifdef _OPENMP
        me = omp_get_thread_num();
#endif
        adj_c* cl = (adj_c*)malloc((size_t)maxlen * sizeof(adj_c));
        if (!cl) {
#pragma omp atomic write
            err = 2;
        }
#pragma omp for schedule(static)
        for (int py = 0; py < H; ++py) {
            if (!cl) continue;
            for (int px = 0; px < W; ++px) {
                const int64_t t = (int64_t)(py / tile_size) * tiles_x + px / tile_size;
                double Tr = 1.0, C[3] = {0.0, 0.0, 0.0};
                int nc = 0;
                for (int64_t i = off[t]; i < off[t + 1]; ++i) {
                    const uint32_t g = lists[i].gid;
                    const double dx = P[g].mean[0] - (px + 0.5), dy = P[g].mean[1] - (py + 0.5);
                    const double q = P[g].conic[0] * dx * dx + 2.0 * P[g].conic[1] * dx * dy +
                                     P[g].conic[2] * dy * dy;
                    const double power = -0.5 * q;
                    if (power > 0.0) continue;
                    const double G = exp(power), araw = P[g].o * G;
                    if (araw < ALPHA_MIN) continue;
                    const double alpha = fmin(ALPHA_MAX, araw);
                    const double test = Tr * (1.0 - alpha);
                    if (test < T_MIN) break;
                    for (int ch = 0; ch < 3; ++ch) C[ch] += Tr * alpha * P[g].rgb[ch];
                    cl[nc].g = g; cl[nc].alpha = alpha; cl[nc].T = Tr; cl[nc].G = G;
                    cl[nc].dx = dx; cl[nc].dy = dy; cl[nc].capped = araw > ALPHA_MAX;
                    nc++;
                    Tr = test;
                }
                const int64_t pix = (int64_t)py * W + px;
                for (int ch = 0; ch < 3; ++ch) out_rgb[3 * pix + ch] = C[ch] + Tr * bg[ch];
                out_alpha[pix] = 1.0 - Tr;
                if (d_img)
                    adj_pixel_reverse(P, cl, nc, Tr, bg, d_img + 3 * pix, d_alpha ? d_alpha[pix] : 0.0,
                                      acc + (size_t)me * n1 * 9);
            }
        }
        free(cl);
    }
    if (d_img && !err) {
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < n; ++g)
            for (int k = 0; k < 9; ++k) {
                double v = 0.0;
                for (int th = 0; th < nth; ++th) v += acc[((size_t)th * n1 + g) * 9 + k];
                d_proj[9 * g + k] = v;
            }
    }
    free(off); free(lists); free(cur); free(acc);
    return err;
}

/*
 * Forward image of the binary64 parameters (the tiled definition of
 * orc_render over the Gaussians orc_project would make visible) into out_rgb
 * [H][W][3] and out_alpha [H][W]; then, when d_img ([H][W][3], dL/d rgb) is
 * not NULL, the gradients: d_proj [n][9] = dL/d(mean2d x, y, conic a, b, c,
 * opacity, r, g, b) and the parameter gradients in the input layouts
 * (d_sh: [n][(D+1)^2][3]). d_alpha ([H][W], dL/d alpha) may be NULL.
 * Gaussians that are not visible get zero gradients.
 */
ORC_EXPORT int orc_adjoint(int64_t n, const double* means, const double* log_scales, const double* quats,
                           const double* logits, const double* sh, int sh_degree, const double* cam, int tile_size,
                           const double* bg, double* out_rgb, double* out_alpha, const double* d_img,
                           const double* d_alpha, double* d_proj, double* d_means, double* d_log_scales,
                           double* d_quats, double* d_logits, double* d_sh) {
    if (n < 0 || sh_degree < 0 || sh_degree > 3 || tile_size <= 0) return 1;
    const int W = (int)cam[16], H = (int)cam[17];
    const int nsh = (sh_degree + 1) * (sh_degree + 1);
    adj_g* P = (adj_g*)calloc((size_t)(n > 0 ? n : 1), sizeof(adj_g));
    if (!P) return 2;
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g)
        adj_project_one(means, log_scales, quats, logits, sh, nsh, sh_degree, cam, tile_size, g, &P[g]);
    int err = adj_composite(P, n, W, H, tile_size, bg, out_rgb, out_alpha, d_img, d_alpha, d_proj);
    if (d_img && !err) {
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < n; ++g) {
            for (int k = 0; k < 3; ++k) d_means[3 * g + k] = d_log_scales[3 * g + k] = 0.0;
            for (int k = 0; k < 4; ++k) d_quats[4 * g + k] = 0.0;
            d_logits[g] = 0.0;
            for (int k = 0; k < nsh * 3; ++k) d_sh[(int64_t)g * nsh * 3 + k] = 0.0;
            if (P[g].vis)
                adj_project_reverse(&P[g], d_proj + 9 * g, sh + (int64_t)g * nsh * 3, nsh, sh_degree, cam,
                                    d_means + 3 * g, d_log_scales + 3 * g, d_quats + 4 * g, d_logits + g,
                                    d_sh + (int64_t)g * nsh * 3);
        }
    }
    free(P);
    return err;
}

/*
 * The compositing adjoint alone, for projected records in the layout of
 * orc_render (mean2d [n][2], conic [n][3], opacity [n], rgb [n][3],
 * depth_key [n], rect [n][4]; gflags NULL = every Gaussian with a non-empty
 * rect is visible): the image into out_rgb / out_alpha and, when d_img is
 * not NULL, d_proj [n][9] as in orc_adjoint.
 */
ORC_EXPORT int orc_composite_adjoint(int64_t n, const double* mean2d, const double* conic, const double* opacity,
                                     const double* rgb, const float* depth_key, const int32_t* rect,
                                     const uint8_t* gflags, int width, int height, int tile_size, const double* bg,
                                     const double* d_img, const double* d_alpha, double* out_rgb, double* out_alpha,
                                     double* d_proj) {
    if (n < 0 || width <= 0 || height <= 0 || tile_size <= 0) return 1;
    if (!rects_in_grid(n, rect, gflags, (width + tile_size - 1) / tile_size, (height + tile_size - 1) / tile_size))
        return 1;
    adj_g* P = (adj_g*)calloc((size_t)(n > 0 ? n : 1), sizeof(adj_g));
    if (!P) return 2;
    for (int64_t g = 0; g < n; ++g) {
        for (int k = 0; k < 4; ++k) P[g].rect[k] = rect[4 * g + k];
        P[g].vis = (gflags ? (gflags[g] & ORC_VISIBLE) != 0 : 1) && rect[4 * g + 2] > rect[4 * g] &&
                   rect[4 * g + 3] > rect[4 * g + 1];
        P[g].mean[0] = mean2d[2 * g];
        P[g].mean[1] = mean2d[2 * g + 1];
        for (int k = 0; k < 3; ++k) { P[g].conic[k] = conic[3 * g + k]; P[g].rgb[k] = rgb[3 * g + k]; }
        P[g].o = opacity[g];
        P[g].key = depth_key[g];
    }
    int err = adj_composite(P, n, width, height, tile_size, bg, out_rgb, out_alpha, d_img, d_alpha, d_proj);
    free(P);
    return err;
}

/*
 * The projection adjoint alone: given d_proj [n][9] = dL/d(mean2d x, y,
 * conic a, b, c, opacity, r, g, b) of the binary64 projection of the
 * parameters, the parameter gradients in the input layouts (d_sh:
 * [n][(D+1)^2][3]), as the last step of orc_adjoint. Gaussians the
 * projection makes invisible get zero gradients.
 */
ORC_EXPORT int orc_project_adjoint(int64_t n, const double* means, const double* log_scales, const double* quats,
                                   const double* logits, const double* sh, int sh_degree, const double* cam,
                                   int tile_size, const double* d_proj, double* d_means, double* d_log_scales,
                                   double* d_quats, double* d_logits, double* d_sh) {
    if (n < 0 || sh_degree < 0 || sh_degree > 3 || tile_size <= 0) return 1;
    const int nsh = (sh_degree + 1) * (sh_degree + 1);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        adj_g P;
        adj_project_one(means, log_scales, quats, logits, sh, nsh, sh_degree, cam, tile_size, g, &P);
        for (int k = 0; k < 3; ++k) d_means[3 * g + k] = d_log_scales[3 * g + k] = 0.0;
        for (int k = 0; k < 4; ++k) d_quats[4 * g + k] = 0.0;
        d_logits[g] = 0.0;
        for (int k = 0; k < nsh * 3; ++k) d_sh[(int64_t)g * nsh * 3 + k] = 0.0;
        if (P.vis)
            adj_project_reverse(&P, d_proj + 9 * g, sh + (int64_t)g * nsh * 3, nsh, sh_degree, cam, d_means + 3 * g,
                                d_log_scales + 3 * g, d_quats + 4 * g, d_logits + g, d_sh + (int64_t)g * nsh * 3);
    }
    return 0;
}
