"""Shared test helpers (no method arithmetic: decoding and comparisons only)."""
import numpy as np

import scenes


def decode_info(info):
    """GPU info tensor/array [n, 4] -> (depth float32 [n], rect int64 [n, 4])."""
    a = np.ascontiguousarray(np.asarray(info)).view(np.uint32)
    return scenes.info_depth(a), scenes.info_rects(a)


def to_np(t):
    return t.detach().cpu().numpy()


def image_compare(gpu_rgb, gpu_alpha, ref, tol=1e-4):
    """max |delta| over pixels the oracle did not flag; returns (rgb err, alpha err, n flagged)."""
    mask = ref["flags"] == 0
    rgb = np.asarray(gpu_rgb, np.float64)
    a = np.asarray(gpu_alpha, np.float64)
    e_rgb = np.abs(rgb - ref["rgb"])[mask].max() if mask.any() else 0.0
    e_a = np.abs(a - ref["alpha"])[mask].max() if mask.any() else 0.0
    return float(e_rgb), float(e_a), int((~mask).sum())


def proj_to_splats(proj):
    """The oracle's projection dict as GPU splat / info arrays (the mean as a
    binary32 pair hi + lo, the other values rounded once to binary32, word 11
    the largest axis scale; rect zero for invisible Gaussians)."""
    import oracle
    n = len(proj["depth_key"])
    vis = (proj["flags"] & oracle.VISIBLE) > 0
    sp = np.zeros((n, 16), np.float32)
    m = np.asarray(proj["mean2d"], np.float64)
    hi = m.astype(np.float32)
    sp[:, 0:2] = hi
    sp[:, 2:4] = (m - hi.astype(np.float64)).astype(np.float32)
    sp[:, 4:7] = proj["conic"]
    sp[:, 7] = proj["opacity"]
    sp[:, 8:11] = proj["rgb"]
    sp[:, 11] = proj["smax"]
    sp[~vis] = 0.0
    rect = np.where(vis[:, None], proj["rect"], 0)
    return sp, scenes.make_info(np.where(vis, proj["depth_key"], np.float32(0)), rect)
