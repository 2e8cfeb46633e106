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
