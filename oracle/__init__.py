"""Python access to the FP64 CPU oracle in ``ref3dgs.c``.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers. The GPU library never imports this
package and this package never imports the GPU library.

``build()`` compiles the C file with gcc (OpenMP, no floating-point
contraction) into ``oracle/libref3dgs.so``; ``lib()`` loads it, building it
first if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ref3dgs.c")
_SO = os.path.join(_HERE, "libref3dgs.so")
_lib = None

# per-Gaussian flags
VISIBLE, AMBIG_RECT, AMBIG_DEPTH, AMBIG_VIS = 1, 2, 4, 8
# per-pixel flags
PIX_AMBIG_ALPHA, PIX_AMBIG_STOP, PIX_AMBIG_GAUSS, PIX_POWER_POS = 1, 2, 4, 8

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4


def build():
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-shared", "-fPIC", "-Wall", "-o", _SO + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64, i32, dbl, flt = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_float
        L.orc_num_threads.restype = i32
        L.orc_sh_basis.argtypes = [P, i32, P]
        L.orc_project.argtypes = [i64, P, P, P, P, P, i32, P, i32, i32, P, P, P, P, P, P, P, P, P]
        L.orc_render.argtypes = [i64, P, P, P, P, P, P, P, i32, i32, i32, P, i64, P,
                                 P, P, P, P, P, P, P, P]
        L.orc_count_entries.argtypes = [i64, P]
        L.orc_count_entries.restype = i64
        L.orc_depth_range.argtypes = [i64, P, P, i32, dbl, dbl, flt, flt, flt, P]
        L.orc_bin_of.argtypes = [flt, flt, flt, i32]
        L.orc_schedule.argtypes = [i64, P, P, i32, i32, i32, i32, dbl, dbl, flt, flt, flt,
                                   P, P, P, P, P, P]
        L.orc_schedule_tiles.argtypes = [i64, P, P, i32, i32, P, i32, dbl, dbl, flt, flt, flt, P, P, P, P]
        L.orc_near_keys.argtypes = [i64, P, P, flt, flt, flt, flt, P]
        L.orc_schedule_keyed.argtypes = [i64, P, P, P, i32, i32, i32, i32, dbl, dbl, flt, flt, flt, P, P, P]
        L.orc_repair_select.argtypes = [i64, i32, P, dbl, P]
        L.orc_repair_select.restype = i64
        L.orc_render_stream.argtypes = [i64, P, P, P, P, P, i32, i32, i32, P, P, P, i64, P,
                                        P, P, P, P, P, P, P, P]
        L.orc_adjoint.argtypes = [i64, P, P, P, P, P, i32, P, i32, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_composite_adjoint.argtypes = [i64, P, P, P, P, P, P, P, i32, i32, i32, P, P, P, P, P, P]
        L.orc_project_adjoint.argtypes = [i64, P, P, P, P, P, i32, P, i32, P, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads():
    return lib().orc_num_threads()


def cam_array(cam):
    """Camera dict (see scenes.py) -> double[20] layout of the C oracle."""
    return np.concatenate([np.asarray(cam["R"], np.float64).reshape(9),
                           np.asarray(cam["t"], np.float64).reshape(3),
                           [cam["fx"], cam["fy"], cam["cx"], cam["cy"],
                            cam["width"], cam["height"], cam["znear"], cam["zfar"]]]).astype(np.float64)


def sh_basis(direction, degree=3):
    out = np.zeros(16, np.float64)
    lib().orc_sh_basis(_p(_c(direction, np.float64)), int(degree), _p(out))
    return out[: (degree + 1) ** 2]


FOOTPRINTS = {"opacity": 0, "three_sigma": 1}


def project(g, cam, tile_size=16, footprint="opacity"):
    """FP64 projection of Gaussians ``g`` (scenes.py layout) through ``cam``;
    ``footprint`` "opacity" (the alpha-support box, the default) or
    "three_sigma" (the baseline's 3-sigma square, cut at tiles)."""
    n = g["means"].shape[0]
    means = _c(g["means"], np.float32)
    ls = _c(g["log_scales"], np.float32)
    qs = _c(g["quats"], np.float32)
    lg = _c(g["logits"], np.float32)
    sh = _c(g["sh"], np.float32)
    out = {
        "mean2d": np.zeros((n, 2)), "cov2d": np.zeros((n, 3)), "conic": np.zeros((n, 3)),
        "depth": np.zeros(n), "opacity": np.zeros(n), "rgb": np.zeros((n, 3)),
        "rect": np.zeros((n, 4), np.int32), "depth_key": np.zeros(n, np.float32),
        "flags": np.zeros(n, np.uint8),
    }
    rc = lib().orc_project(n, _p(means), _p(ls), _p(qs), _p(lg), _p(sh), int(g["sh_degree"]),
                           _p(cam_array(cam)), int(tile_size), FOOTPRINTS[footprint], _p(out["mean2d"]),
                           _p(out["cov2d"]),
                           _p(out["conic"]), _p(out["depth"]), _p(out["opacity"]), _p(out["rgb"]),
                           _p(out["rect"]), _p(out["depth_key"]), _p(out["flags"]))
    assert rc == 0, rc
    # largest activated axis scale, the s_max of the near-depth binning key
    out["smax"] = np.exp(ls.astype(np.float64).max(axis=1)).astype(np.float32)
    return out


def render(proj, width, height, tile_size=16, bg=(0.0, 0.0, 0.0), pix=None, mode="tiled"):
    """Composite projected Gaussians (dict with mean2d, conic, opacity, rgb,
    depth_key, rect, flags) at every pixel or at the [k, 2] (x, y) ``pix``."""
    n = proj["mean2d"].shape[0]
    npix = width * height if pix is None else len(pix)
    pixa = None if pix is None else _c(pix, np.int32)
    out = {
        "rgb": np.zeros((npix, 3)), "alpha": np.zeros(npix), "last_gid": np.zeros(npix, np.int64),
        "last_pos": np.zeros(npix, np.int64), "ncontrib": np.zeros(npix, np.int32),
        "nvisit": np.zeros(npix, np.int32), "nsupport": np.zeros(npix, np.int32),
        "flags": np.zeros(npix, np.uint8),
    }
    rect = _c(proj["rect"], np.int32) if mode == "tiled" else None
    flags = None if proj.get("flags") is None else _c(proj["flags"], np.uint8)
    rc = lib().orc_render(n, _p(_c(proj["mean2d"], np.float64)), _p(_c(proj["conic"], np.float64)),
                          _p(_c(proj["opacity"], np.float64)), _p(_c(proj["rgb"], np.float64)),
                          _p(_c(proj["depth_key"], np.float32)), _p(rect), _p(flags), int(width),
                          int(height), int(tile_size), _p(_c(bg, np.float64)), npix, _p(pixa),
                          _p(out["rgb"]), _p(out["alpha"]), _p(out["last_gid"]), _p(out["last_pos"]),
                          _p(out["ncontrib"]), _p(out["nvisit"]), _p(out["nsupport"]), _p(out["flags"]))
    assert rc == 0, rc
    if pix is None:
        for k in list(out):
            v = out[k]
            out[k] = v.reshape((height, width) + v.shape[1:])
    return out


def render_stream(proj, width, height, tile_offsets, ids, tile_size=16, bg=(0.0, 0.0, 0.0), pix=None):
    """Composite each tile's pixels over the Gaussian ids of its range
    ids[tile_offsets[t]:tile_offsets[t + 1]] in the listed order."""
    n = proj["mean2d"].shape[0]
    npix = width * height if pix is None else len(pix)
    pixa = None if pix is None else _c(pix, np.int32)
    off = _c(tile_offsets, np.uint32)
    tiles = ((width + tile_size - 1) // tile_size) * ((height + tile_size - 1) // tile_size)
    assert off.shape == (tiles + 1,)
    idv = _c(ids, np.uint32)
    assert len(idv) >= int(off[-1])
    out = {
        "rgb": np.zeros((npix, 3)), "alpha": np.zeros(npix), "last_gid": np.zeros(npix, np.int64),
        "last_pos": np.zeros(npix, np.int64), "ncontrib": np.zeros(npix, np.int32),
        "nvisit": np.zeros(npix, np.int32), "nsupport": np.zeros(npix, np.int32),
        "flags": np.zeros(npix, np.uint8),
    }
    flags = None if proj.get("flags") is None else _c(proj["flags"], np.uint8)
    rc = lib().orc_render_stream(n, _p(_c(proj["mean2d"], np.float64)), _p(_c(proj["conic"], np.float64)),
                                 _p(_c(proj["opacity"], np.float64)), _p(_c(proj["rgb"], np.float64)), _p(flags),
                                 int(width), int(height), int(tile_size), _p(_c(bg, np.float64)), _p(off), _p(idv),
                                 npix, _p(pixa), _p(out["rgb"]), _p(out["alpha"]), _p(out["last_gid"]),
                                 _p(out["last_pos"]), _p(out["ncontrib"]), _p(out["nvisit"]), _p(out["nsupport"]),
                                 _p(out["flags"]))
    assert rc == 0, rc
    if pix is None:
        for k in list(out):
            v = out[k]
            out[k] = v.reshape((height, width) + v.shape[1:])
    return out


def splats_to_proj(splats, info):
    """Projected splats in the two-array layout of scenes.random_splats
    (splats [n, 16] fp32, info [n, 4] uint32) as the float64 record dict
    that ``render`` takes. The mean is hi + lo, exactly, in float64."""
    s = np.ascontiguousarray(splats, dtype=np.float32)
    w = np.ascontiguousarray(info, dtype=np.uint32)
    rect = np.stack([w[:, 1] & 0xFFFF, w[:, 1] >> 16, w[:, 2] & 0xFFFF, w[:, 2] >> 16], 1)
    rect = rect.astype(np.int32)
    vis = (rect[:, 2] > rect[:, 0]) & (rect[:, 3] > rect[:, 1])
    return {
        "mean2d": s[:, 0:2].astype(np.float64) + s[:, 2:4].astype(np.float64),
        "conic": s[:, 4:7].astype(np.float64),
        "opacity": s[:, 7].astype(np.float64),
        "rgb": s[:, 8:11].astype(np.float64),
        "depth_key": np.ascontiguousarray(w[:, 0]).view(np.float32).copy(),
        "rect": rect,
        "flags": vis.astype(np.uint8) * VISIBLE,
    }


def count_entries(rect):
    return int(lib().orc_count_entries(len(rect), _p(_c(rect, np.int32))))


def depth_range(depth, rect, S=8192, p_lo=1.0, p_hi=99.0, pad=0.05, znear=0.01, zfar=1e10):
    zr = np.zeros(2, np.float32)
    rc = lib().orc_depth_range(len(depth), _p(_c(depth, np.float32)), _p(_c(rect, np.int32)), int(S),
                               float(p_lo), float(p_hi), float(pad), float(znear), float(zfar), _p(zr))
    assert rc == 0
    return zr


def bin_of(z, zmin, zmax, K):
    return int(lib().orc_bin_of(float(z), float(zmin), float(zmax), int(K)))


def schedule(depth, rect, tiles_x, tiles_y, K=64, S=8192, p_lo=1.0, p_hi=99.0, pad=0.05,
             znear=0.01, zfar=1e10):
    """Integer schedule (keys, vals, tile_offsets, zrange, bin_offsets, stream)."""
    depth = _c(depth, np.float32)
    rect = _c(rect, np.int32)
    n = len(depth)
    M = count_entries(rect)
    T = tiles_x * tiles_y
    out = {
        "keys": np.zeros(M, np.uint64), "vals": np.zeros(M, np.uint32),
        "tile_offsets": np.zeros(T + 1, np.uint32), "zrange": np.zeros(2, np.float32),
        "bin_offsets": np.zeros(T * K + 1, np.uint32), "stream": np.zeros(M, np.uint64),
    }
    rc = lib().orc_schedule(n, _p(depth), _p(rect), int(tiles_x), int(tiles_y), int(K), int(S),
                            float(p_lo), float(p_hi), float(pad), float(znear), float(zfar),
                            _p(out["keys"]), _p(out["vals"]), _p(out["tile_offsets"]),
                            _p(out["zrange"]), _p(out["bin_offsets"]), _p(out["stream"]))
    assert rc == 0, rc
    out["M"] = M
    return out


def near_keys(depth, smax, alpha=1.0, gamma=0.25, znear=0.01, zfar=1e10):
    """Near-depth binning keys (binary32) of the Gaussians."""
    d = _c(depth, np.float32)
    out = np.zeros(len(d), np.float32)
    lib().orc_near_keys(len(d), _p(d), _p(_c(smax, np.float32)), float(alpha), float(gamma), float(znear),
                        float(zfar), _p(out))
    return out


def schedule_keyed(depth, bin_depth, rect, tiles_x, tiles_y, K=64, S=8192, p_lo=1.0, p_hi=99.0, pad=0.05,
                   znear=0.01, zfar=1e10):
    """Binned schedule with the bins (and the depth range) formed on
    ``bin_depth`` and every segment sorted by (depth bits, id): zrange,
    bin_offsets [T K + 1], stream [M]."""
    depth = _c(depth, np.float32)
    bd = _c(bin_depth, np.float32)
    rect = _c(rect, np.int32)
    M = count_entries(rect)
    T = tiles_x * tiles_y
    out = {"zrange": np.zeros(2, np.float32), "bin_offsets": np.zeros(T * K + 1, np.uint32),
           "stream": np.zeros(M, np.uint64)}
    rc = lib().orc_schedule_keyed(len(depth), _p(depth), _p(bd), _p(rect), int(tiles_x), int(tiles_y), int(K),
                                  int(S), float(p_lo), float(p_hi), float(pad), float(znear), float(zfar),
                                  _p(out["zrange"]), _p(out["bin_offsets"]), _p(out["stream"]))
    assert rc == 0, rc
    out["M"] = M
    return out


def repair_select(bin_offsets, T, K, budget_frac=0.25):
    """Selected segments (uint8 [T K]) and the selected entry count of the
    rule-based, budgeted repair selection."""
    off = _c(bin_offsets, np.uint32)
    assert off.shape == (T * K + 1,)
    sel = np.zeros(T * K, np.uint8)
    used = int(lib().orc_repair_select(int(T), int(K), _p(off), float(budget_frac), _p(sel)))
    return sel, used


def schedule_tiles(depth, rect, tiles_x, tiles_y, per_tile_bins, S=8192, p_lo=1.0, p_hi=99.0, pad=0.05,
                   znear=0.01, zfar=1e10):
    """Binned schedule with per_tile_bins[t] bins in tile t: zrange,
    seg_base [T + 1], bin_offsets [sum + 1], stream [M]."""
    depth = _c(depth, np.float32)
    rect = _c(rect, np.int32)
    kt = _c(per_tile_bins, np.int32)
    T = tiles_x * tiles_y
    assert kt.shape == (T,)
    M = count_entries(rect)
    out = {"zrange": np.zeros(2, np.float32), "seg_base": np.zeros(T + 1, np.uint32),
           "bin_offsets": np.zeros(int(kt.astype(np.int64).sum()) + 1, np.uint32), "stream": np.zeros(M, np.uint64)}
    rc = lib().orc_schedule_tiles(len(depth), _p(depth), _p(rect), int(tiles_x), int(tiles_y), _p(kt), int(S),
                                  float(p_lo), float(p_hi), float(pad), float(znear), float(zfar), _p(out["zrange"]),
                                  _p(out["seg_base"]), _p(out["bin_offsets"]), _p(out["stream"]))
    assert rc == 0, rc
    out["M"] = M
    return out


def adjoint(g, cam, tile_size=16, bg=(0.0, 0.0, 0.0), d_img=None, d_alpha=None):
    """Binary64 forward image of the parameters in ``g`` (converted to
    float64) and, when ``d_img`` ([H, W, 3], dL/d rgb) is given, the
    gradients: ``d_proj`` [n, 9] (mean2d x, y, conic a, b, c, opacity, r, g,
    b) and ``means``, ``log_scales``, ``quats``, ``logits``, ``sh`` in the
    input layouts. ``d_alpha`` [H, W] is dL/d alpha (optional)."""
    n = g["means"].shape[0]
    W, H = int(cam["width"]), int(cam["height"])
    deg = int(g["sh_degree"])
    nsh = (deg + 1) ** 2
    ins = [_c(g[k], np.float64) for k in ("means", "log_scales", "quats", "logits", "sh")]
    out = {"rgb": np.zeros((H, W, 3)), "alpha": np.zeros((H, W))}
    grads = None
    if d_img is not None:
        grads = {"d_proj": np.zeros((n, 9)), "means": np.zeros((n, 3)), "log_scales": np.zeros((n, 3)),
                 "quats": np.zeros((n, 4)), "logits": np.zeros(n), "sh": np.zeros((n, nsh, 3))}
    dimg = None if d_img is None else _c(d_img, np.float64)
    dal = None if d_alpha is None else _c(d_alpha, np.float64)
    gp = (lambda k: None) if grads is None else (lambda k: _p(grads[k]))
    rc = lib().orc_adjoint(n, *[_p(a) for a in ins], deg, _p(cam_array(cam)), int(tile_size),
                           _p(_c(bg, np.float64)), _p(out["rgb"]), _p(out["alpha"]), _p(dimg), _p(dal),
                           gp("d_proj"), gp("means"), gp("log_scales"), gp("quats"), gp("logits"), gp("sh"))
    assert rc == 0, rc
    if grads is not None:
        out.update(grads)
    return out


def project_adjoint(g, cam, d_proj, tile_size=16):
    """Parameter gradients (``means``, ``log_scales``, ``quats``, ``logits``,
    ``sh`` in the input layouts) of the binary64 projection of ``g``, given
    ``d_proj`` [n, 9] = dL/d(mean2d x, y, conic a, b, c, opacity, r, g, b)."""
    n = g["means"].shape[0]
    deg = int(g["sh_degree"])
    nsh = (deg + 1) ** 2
    ins = [_c(g[k], np.float64) for k in ("means", "log_scales", "quats", "logits", "sh")]
    dp = _c(d_proj, np.float64)
    assert dp.shape == (n, 9)
    out = {"means": np.zeros((n, 3)), "log_scales": np.zeros((n, 3)), "quats": np.zeros((n, 4)),
           "logits": np.zeros(n), "sh": np.zeros((n, nsh, 3))}
    rc = lib().orc_project_adjoint(n, *[_p(a) for a in ins], deg, _p(cam_array(cam)), int(tile_size), _p(dp),
                                   _p(out["means"]), _p(out["log_scales"]), _p(out["quats"]), _p(out["logits"]),
                                   _p(out["sh"]))
    assert rc == 0, rc
    return out


def mse_upstream(rgb, target):
    """Loss mean((rgb - target)^2) over pixels and channels and its gradient
    with respect to rgb."""
    d = np.asarray(rgb, np.float64) - np.asarray(target, np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def composite_adjoint(proj, width, height, tile_size=16, bg=(0.0, 0.0, 0.0), d_img=None, d_alpha=None):
    """The compositing adjoint alone for projected records (the dict that
    ``render`` takes): image ``rgb`` [H, W, 3], ``alpha`` [H, W] and, when
    ``d_img`` is given, ``d_proj`` [n, 9] (mean2d x, y, conic a, b, c,
    opacity, r, g, b)."""
    n = proj["mean2d"].shape[0]
    out = {"rgb": np.zeros((height, width, 3)), "alpha": np.zeros((height, width))}
    dp = np.zeros((n, 9)) if d_img is not None else None
    flags = None if proj.get("flags") is None else _c(proj["flags"], np.uint8)
    rc = lib().orc_composite_adjoint(
        n, _p(_c(proj["mean2d"], np.float64)), _p(_c(proj["conic"], np.float64)),
        _p(_c(proj["opacity"], np.float64)), _p(_c(proj["rgb"], np.float64)), _p(_c(proj["depth_key"], np.float32)),
        _p(_c(proj["rect"], np.int32)), _p(flags), int(width), int(height), int(tile_size), _p(_c(bg, np.float64)),
        _p(None if d_img is None else _c(d_img, np.float64)), _p(None if d_alpha is None else _c(d_alpha, np.float64)),
        _p(out["rgb"]), _p(out["alpha"]), _p(dp))
    assert rc == 0, rc
    if dp is not None:
        out["d_proj"] = dp
    return out
