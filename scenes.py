"""Seeded synthetic inputs: 3D Gaussian scenes and pinhole cameras.

This module only draws random numbers and builds camera poses. It holds none
of the rasterizer's arithmetic (no projection, colour evaluation, binning or
compositing), so both the FP64 oracle tests and the GPU path can take their
inputs from it without sharing any of the method.

Conventions used throughout the project:
- Gaussians are fp32 structure-of-arrays: ``means`` [N,3], ``log_scales``
  [N,3], ``quats`` [N,4] as (w, x, y, z), ``logits`` [N] (opacity before the
  sigmoid), ``sh`` [N,(D+1)^2,3] real spherical-harmonic coefficients in the
  order l^2+l+m, m = -l..l.
- A camera is a dict with ``R`` [3,3] world-to-camera rotation (rows are the
  camera x right, y down, z forward axes), ``t`` [3] so that p_cam = R p + t,
  focal lengths ``fx``, ``fy``, principal point ``cx``, ``cy``, ``width``,
  ``height``, ``znear``, ``zfar``. Camera values are float64.
- "N(m, s)" always means mean m and standard deviation s.
- Draw order inside each scene: means, log-scales, quaternions, logits, SH.
  Every draw is float64 cast to float32.

The paper evaluates on nine captured scenes (Mip-NeRF 360, Tanks and Temples,
Deep Blending) with trained models; none of those are available here, so these
synthetic scenes of the same kind (many small anisotropic splats on surfaces,
long per-tile ranges at 1080p) stand in for them.
"""
from __future__ import annotations

import math

import numpy as np

ZNEAR = 0.01
ZFAR = 1.0e10


def camera(R, t, fx, fy, cx, cy, width, height, znear=ZNEAR, zfar=ZFAR):
    return {
        "R": np.asarray(R, dtype=np.float64).reshape(3, 3).copy(),
        "t": np.asarray(t, dtype=np.float64).reshape(3).copy(),
        "fx": float(fx), "fy": float(fy), "cx": float(cx), "cy": float(cy),
        "width": int(width), "height": int(height),
        "znear": float(znear), "zfar": float(zfar),
    }


def look_at(position, target, down=(0.0, 1.0, 0.0)):
    """World-to-camera (R, t) for a camera at ``position`` looking at ``target``.

    The camera z axis points at the target, y points along the component of
    ``down`` orthogonal to z, x = y cross z (right-handed, image x right, y down).
    """
    c = np.asarray(position, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - c
    f /= np.linalg.norm(f)
    d = np.asarray(down, dtype=np.float64)
    y = d - np.dot(d, f) * f
    y /= np.linalg.norm(y)
    x = np.cross(y, f)
    R = np.stack([x, y, f])
    t = -R @ c
    return R, t


def _unit_quats(rng, n):
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _pack(means, log_scales, quats, logits, sh, degree):
    return {
        "means": np.ascontiguousarray(means, dtype=np.float32),
        "log_scales": np.ascontiguousarray(log_scales, dtype=np.float32),
        "quats": np.ascontiguousarray(quats, dtype=np.float32),
        "logits": np.ascontiguousarray(logits, dtype=np.float32),
        "sh": np.ascontiguousarray(sh, dtype=np.float32),
        "sh_degree": int(degree),
    }


def uniform_box_scene(n, seed=0, sh_degree=0, lo=(-1.0, -1.0, 2.0), hi=(1.0, 1.0, 6.0),
                      log_scale_mean=-4.0, log_scale_std=0.5, logit_std=1.5, sh_std=0.2):
    """Means uniform in a box; the small forward config and its relatives.

    Degree 0: the DC coefficient is uniform in [-sqrt(pi), sqrt(pi)], which is
    the range whose colours are uniform in [0, 1]. Degree > 0: every
    coefficient is N(0, sh_std).
    """
    rng = np.random.default_rng(seed)
    means = rng.uniform(lo, hi, size=(n, 3))
    log_scales = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    quats = _unit_quats(rng, n)
    logits = rng.normal(0.0, logit_std, size=n)
    k = (sh_degree + 1) ** 2
    if sh_degree == 0:
        r = math.sqrt(math.pi)
        sh = rng.uniform(-r, r, size=(n, 1, 3))
    else:
        sh = rng.normal(0.0, sh_std, size=(n, k, 3))
    return _pack(means, log_scales, quats, logits, sh, sh_degree)


def surface_scene(n, seed=0, sh_degree=3, n_prims=64, box=5.0, jitter=0.01,
                  log_scale_mean=-4.5, log_scale_std=0.7, logit_std=2.0, sh_std=0.2):
    """Gaussians sampled on random spheres and planes inside a cube of side 2*box.

    Each primitive is a sphere (probability 1/2: centre U[-4,4]^3, radius
    U[0.5,2]) or a square plane (centre U[-4,4]^3, normal uniform on the
    sphere, side U[1,4]). Points are uniform on the surface, n/n_prims per
    primitive (the remainder goes to the first primitives), offset along the
    surface normal by N(0, jitter), then clipped to the cube.
    """
    rng = np.random.default_rng(seed)
    counts = np.full(n_prims, n // n_prims, dtype=np.int64)
    counts[: n % n_prims] += 1
    kinds = rng.random(n_prims) < 0.5
    centres = rng.uniform(-4.0, 4.0, size=(n_prims, 3))
    radii = rng.uniform(0.5, 2.0, size=n_prims)
    normals = rng.normal(0.0, 1.0, size=(n_prims, 3))
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    sides = rng.uniform(1.0, 4.0, size=n_prims)
    chunks = []
    for p in range(n_prims):
        m = int(counts[p])
        if m == 0:
            continue
        if kinds[p]:
            d = rng.normal(0.0, 1.0, size=(m, 3))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            off = rng.normal(0.0, jitter, size=(m, 1))
            pts = centres[p] + d * (radii[p] + off)
        else:
            nrm = normals[p]
            a = np.array([1.0, 0.0, 0.0]) if abs(nrm[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
            e1 = np.cross(nrm, a)
            e1 /= np.linalg.norm(e1)
            e2 = np.cross(nrm, e1)
            uv = rng.uniform(-0.5 * sides[p], 0.5 * sides[p], size=(m, 2))
            off = rng.normal(0.0, jitter, size=(m, 1))
            pts = centres[p] + uv[:, :1] * e1 + uv[:, 1:] * e2 + off * nrm
        chunks.append(pts)
    means = np.clip(np.concatenate(chunks, axis=0), -box, box)
    log_scales = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    quats = _unit_quats(rng, n)
    logits = rng.normal(0.0, logit_std, size=n)
    k = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, sh_std, size=(n, k, 3))
    return _pack(means, log_scales, quats, logits, sh, sh_degree)


# ---------------------------------------------------------------------------
# The five workloads (small forward, scene-shaped 1080p, batched cameras,
# training step, learned bins). Each returns (gaussians, camera or cameras).
# ---------------------------------------------------------------------------

def small_forward(seed=0, n=2000):
    """2k Gaussians in camera space, identity pose, 128x128, f=128, D=0."""
    g = uniform_box_scene(n, seed=seed, sh_degree=0)
    cam = camera(np.eye(3), np.zeros(3), 128.0, 128.0, 64.0, 64.0, 128, 128)
    return g, cam


def scene_1080p(seed=0, n=1_000_000, width=1920, height=1080, focal=1100.0):
    """1M Gaussians on 64 surfaces, 1920x1080 at f=1100, camera at z=-15."""
    g = surface_scene(n, seed=seed, sh_degree=3)
    cam = camera(np.eye(3), np.array([0.0, 0.0, 15.0]), focal, focal,
                 width / 2.0, height / 2.0, width, height)
    return g, cam


def ring_cameras(n_cams=16, seed=0, radius=5.0, centre=(0.0, 0.0, 4.0)):
    """Cameras on a ring in the xz-plane looking at ``centre``; W = round(640 s),
    H = round(360 s) with s ~ U[1,4]; fx = fy = W; principal point at the centre."""
    rng = np.random.default_rng(seed + 7919)
    s = rng.uniform(1.0, 4.0, size=n_cams)
    cams = []
    for k in range(n_cams):
        th = 2.0 * math.pi * k / n_cams
        pos = np.array([centre[0] + radius * math.sin(th), centre[1],
                        centre[2] - radius * math.cos(th)])
        R, t = look_at(pos, centre)
        W = int(round(640 * s[k]))
        H = int(round(360 * s[k]))
        cams.append(camera(R, t, W, W, W / 2.0, H / 2.0, W, H))
    return cams


def batched_scene(seed=0, n=3_000_000, n_cams=16):
    g = uniform_box_scene(n, seed=seed, sh_degree=0)
    return g, ring_cameras(n_cams, seed=seed)


def training_scene(seed=0, n=500_000, width=1297, height=840):
    """500k Gaussians of the small-forward structure with D=3, 1297x840."""
    g = uniform_box_scene(n, seed=seed, sh_degree=3)
    cam = camera(np.eye(3), np.zeros(3), float(width), float(width),
                 width / 2.0, height / 2.0, width, height)
    return g, cam


def training_target(width, height, seed=1):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(height, width, 3)).astype(np.float32)


def fd_subcase(n=200, size=64, seed=0):
    """The first 200 Gaussians of the training scene at 64x64, f=64."""
    g = subset(uniform_box_scene(500_000, seed=seed, sh_degree=3), slice(0, n))
    cam = camera(np.eye(3), np.zeros(3), float(size), float(size), size / 2.0,
                 size / 2.0, size, size)
    return g, cam


def learned_eval_scene(seed=0, n=6_000_000):
    """6M Gaussians of the surface structure at 3840x2160, f=2200."""
    g = surface_scene(n, seed=seed, sh_degree=3)
    cam = camera(np.eye(3), np.array([0.0, 0.0, 15.0]), 2200.0, 2200.0,
                 1920.0, 1080.0, 3840, 2160)
    return g, cam


def learned_train_scenes(first_seed=1000, count=50, small_n=2000, surface_n=200_000):
    """Seeds 1000..1049 alternating the small-forward and surface structures."""
    out = []
    for i in range(count):
        s = first_seed + i
        if i % 2 == 0:
            out.append(small_forward(seed=s, n=small_n))
        else:
            out.append(scene_1080p(seed=s, n=surface_n))
    return out


STRESS_KINDS = ("sparse", "dense", "bimodal")


def depth_stress_scene(kind, n=None, seed=0, width=1920, height=1080, focal=1100.0, sh_degree=3):
    """Synthetic depth-distribution stress scenes (identity camera at the
    origin looking down +z; means spread uniformly over the image, 5 % beyond
    its edges; log-scales N(-4.5, 0.5) + ln(z / 10), so that the screen size
    does not depend on the depth; logits N(0, 2); SH coefficients N(0, 0.2)).

    sparse:  n = 100k, depth log-uniform in [2, 200] (few entries per
             tile, spread over the whole bin range);
    dense:   n = 1M, 96 % at depth U[10, 10.05], 2 % log-uniform in [2, 10]
             and 2 % in [10.05, 200] (a thin slab inside a wide depth range:
             one or two bins hold nearly every entry of a tile, long
             segments);
    bimodal: n = 1M, half at depth U[3, 3.2] and half at U[40, 42] (two
             slabs, the bins between them empty).
    Draw order: depths, image positions, log-scales, quaternions, logits, SH.
    """
    defaults = {"sparse": 100_000, "dense": 1_000_000, "bimodal": 1_000_000}
    if kind not in defaults:
        raise ValueError(f"unknown stress kind {kind!r}")
    n = defaults[kind] if n is None else int(n)
    rng = np.random.default_rng(seed)
    if kind == "sparse":
        z = np.exp(rng.uniform(np.log(2.0), np.log(200.0), size=n))
    elif kind == "dense":
        r = rng.random(n)
        z = np.where(r < 0.96, rng.uniform(10.0, 10.05, size=n),
                     np.where(r < 0.98, np.exp(rng.uniform(np.log(2.0), np.log(10.0), size=n)),
                              np.exp(rng.uniform(np.log(10.05), np.log(200.0), size=n))))
    else:
        near = rng.random(n) < 0.5
        z = np.where(near, rng.uniform(3.0, 3.2, size=n), rng.uniform(40.0, 42.0, size=n))
    u = rng.uniform(-0.05 * width, 1.05 * width, size=n)
    v = rng.uniform(-0.05 * height, 1.05 * height, size=n)
    means = np.stack([(u - width / 2.0) * z / focal, (v - height / 2.0) * z / focal, z], axis=1)
    log_scales = rng.normal(-4.5, 0.5, size=(n, 3)) + np.log(z / 10.0)[:, None]
    quats = _unit_quats(rng, n)
    logits = rng.normal(0.0, 2.0, size=n)
    k = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.2, size=(n, k, 3))
    g = _pack(means, log_scales, quats, logits, sh, sh_degree)
    cam = camera(np.eye(3), np.zeros(3), focal, focal, width / 2.0, height / 2.0, width, height)
    return g, cam


def guard_scene(seed=0, n=4000, width=256, height=192, focal=200.0):
    """Large Gaussians around and beyond the edges of the field of view, to
    exercise the frustum guard: x/z and y/z uniform in +-2.2 x the half FOV,
    z U[2, 6] (camera space, identity pose), log-scales N(-1.5, 0.3), logits
    N(1, 1), SH degree 1 with coefficients N(0, 0.2)."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(2.0, 6.0, size=n)
    u = rng.uniform(-2.2, 2.2, size=n) * (0.5 * width / focal)
    v = rng.uniform(-2.2, 2.2, size=n) * (0.5 * height / focal)
    means = np.stack([u * z, v * z, z], 1)
    log_scales = rng.normal(-1.5, 0.3, size=(n, 3))
    quats = _unit_quats(rng, n)
    logits = rng.normal(1.0, 1.0, size=n)
    sh = rng.normal(0.0, 0.2, size=(n, 4, 3))
    g = _pack(means, log_scales, quats, logits, sh, 1)
    cam = camera(np.eye(3), np.zeros(3), focal, focal, width / 2.0, height / 2.0, width, height)
    return g, cam


def morton_sorted(g, bits=10):
    """The same Gaussians stored in the Z-order (Morton order) of their
    means over the scene's bounding box, quantised to 2^bits cells per
    axis: a storage layout in which Gaussians that are near in space, and so
    in the same screen tiles, are near in memory."""
    m = np.asarray(g["means"], np.float64)
    lo, hi = m.min(0), m.max(0)
    q = ((m - lo) / np.maximum(hi - lo, 1e-12) * ((1 << bits) - 1)).astype(np.uint64)
    code = np.zeros(len(m), np.uint64)
    for b in range(bits):
        for a in range(3):
            code |= ((q[:, a] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + a)
    return subset(g, np.argsort(code, kind="stable"))


def subset(g, idx):
    """Gaussians ``idx`` of scene ``g`` (keeps the degree)."""
    out = {k: np.ascontiguousarray(v[idx]) for k, v in g.items() if k != "sh_degree"}
    out["sh_degree"] = g["sh_degree"]
    return out


# ---------------------------------------------------------------------------
# Synthetic projected splats, for exercising the ordering and raster stages
# on their own. Two arrays per splat set:
#   splats [n, 16] fp32: mean_x, mean_y (binary32 parts), mean_x_lo, mean_y_lo
#       (the remainders, so that hi + lo carries the mean to ~1e-11 px),
#       conic_a, conic_b, conic_c, opacity, r, g, b, s_max (the largest
#       world axis scale; zero unless drawn), four zeros.
#   info [n, 4] uint32: depth (binary32 bits), rect word 0 (x0 | y0 << 16),
#       rect word 1 (x1 | y1 << 16), number of tiles; the rect is half-open
#       in tile units.
# ---------------------------------------------------------------------------

def random_splats(n, width, height, tile_size=16, seed=0, depth_lo=1.0, depth_hi=50.0,
                  max_sigma_px=12.0, tie_fraction=0.0, opacity_lo=0.02, hidden_fraction=0.0, smax_range=None):
    """Random projected splats (splats, info), see the layout above.

    Each splat's screen covariance has standard deviations log-uniform in
    [0.6, max_sigma_px] px and correlation U[-0.9, 0.9]; the conic is its
    inverse. The rect covers the mean +- 3.5 standard deviations, a superset
    of where any splat with opacity <= 1 can reach 1/255 (that needs
    q <= 2 ln 255 < 3.5^2). ``tie_fraction`` of the splats copy the depth of
    another one so that the id tie-break is exercised; ``hidden_fraction``
    get an empty rect. ``smax_range`` = (lo, hi): word 11 (the largest world
    axis scale) log-uniform in [lo, hi], drawn after everything else; None
    leaves it zero.
    """
    rng = np.random.default_rng(seed)
    tx = (width + tile_size - 1) // tile_size
    ty = (height + tile_size - 1) // tile_size
    mx = rng.uniform(-8.0, width + 8.0, size=n)
    my = rng.uniform(-8.0, height + 8.0, size=n)
    lo, hi = np.log(0.6), np.log(max_sigma_px)
    sx = np.exp(rng.uniform(lo, hi, size=n))
    sy = np.exp(rng.uniform(lo, hi, size=n))
    rho = rng.uniform(-0.9, 0.9, size=n)
    opac = rng.uniform(opacity_lo, 1.0, size=n)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    depth = np.exp(rng.uniform(np.log(depth_lo), np.log(depth_hi), size=n)).astype(np.float32)
    if tie_fraction > 0 and n > 1:
        k = int(tie_fraction * n)
        src = rng.integers(0, n, size=k)
        dst = rng.integers(0, n, size=k)
        depth[dst] = depth[src]
    hidden = rng.random(n) < hidden_fraction
    cxx, cyy, cxy = sx * sx, sy * sy, rho * sx * sy
    det = cxx * cyy - cxy * cxy
    splats = np.zeros((n, 16), dtype=np.float32)
    mxh, myh = mx.astype(np.float32), my.astype(np.float32)
    splats[:, 0], splats[:, 1] = mxh, myh
    splats[:, 2] = (mx - mxh.astype(np.float64)).astype(np.float32)
    splats[:, 3] = (my - myh.astype(np.float64)).astype(np.float32)
    splats[:, 4], splats[:, 5], splats[:, 6] = cyy / det, -cxy / det, cxx / det
    splats[:, 7] = opac
    splats[:, 8:11] = rgb
    ex, ey = 3.5 * sx, 3.5 * sy
    x0 = np.clip(np.floor((mx - ex) / tile_size), 0, tx).astype(np.int64)
    x1 = np.clip(np.floor((mx + ex) / tile_size) + 1, 0, tx).astype(np.int64)
    y0 = np.clip(np.floor((my - ey) / tile_size), 0, ty).astype(np.int64)
    y1 = np.clip(np.floor((my + ey) / tile_size) + 1, 0, ty).astype(np.int64)
    x1 = np.where(hidden, x0, x1)
    if smax_range is not None:
        splats[:, 11] = np.exp(rng.uniform(np.log(smax_range[0]), np.log(smax_range[1]), size=n))
    return splats, make_info(depth, np.stack([x0, y0, x1, y1], 1))


def make_info(depth, rect):
    """Pack binary32 depths [n] and int rects [n, 4] into the info layout."""
    rect = np.asarray(rect, dtype=np.int64)
    info = np.zeros((len(rect), 4), dtype=np.uint32)
    info[:, 0] = np.ascontiguousarray(depth, dtype=np.float32).view(np.uint32)
    info[:, 1] = (rect[:, 0] | (rect[:, 1] << 16)).astype(np.uint32)
    info[:, 2] = (rect[:, 2] | (rect[:, 3] << 16)).astype(np.uint32)
    w = np.maximum(rect[:, 2] - rect[:, 0], 0)
    h = np.maximum(rect[:, 3] - rect[:, 1], 0)
    info[:, 3] = (w * h).astype(np.uint32)
    return info


def info_rects(info):
    """Decode the rect words of an info array into int64 [n, 4] (x0, y0, x1, y1)."""
    w = np.asarray(info, dtype=np.uint32)
    return np.stack([w[:, 1] & 0xFFFF, w[:, 1] >> 16, w[:, 2] & 0xFFFF, w[:, 2] >> 16],
                    axis=1).astype(np.int64)


def info_depth(info):
    return np.ascontiguousarray(np.asarray(info, dtype=np.uint32)[:, 0]).view(np.float32)
