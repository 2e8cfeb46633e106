"""Per-camera tile-size / bin-count autotuner.

For one camera and scene size it times the whole per-view frame as the
batched renderer runs it (projection, binning with exact repair, the
persistent multi-view raster on this one view) for every candidate (tile
size in {8, 16, 32}) x (bins K in {16, 32, 64, 128, 256}) x (sub-bins per bin in
{8, 4, 2}) with HIP events on the launch stream and keeps the fastest. The
choice never changes the image beyond rounding (exact repair keeps the
global order, whatever the bins and sub-bins; the tile size only moves the
tile-relative origin of the staged means), so only time is compared.

Results are cached in a JSON file keyed by (GPU architecture, W x H, power-
of-two bucket of the Gaussian count); a cached entry is reused without
timing. The cache is plain data and can be deleted at any time.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

from .api import BatchRenderer, Params, project

TILE_SIZES = (8, 16, 32)
BIN_COUNTS = (16, 32, 64, 128, 256)
CANDIDATES = tuple((ts, k) for ts in TILE_SIZES for k in BIN_COUNTS)
SUB_BINS = (8, 4, 2)  # sub-bins per bin of the exact repair: more split the long segments finer
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "tilegs", "autotune.json")


def cache_key(cam, n):
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    bucket = int(round(math.log2(max(int(n), 1))))
    return f"{arch}|{int(cam['width'])}x{int(cam['height'])}|n2^{bucket}"


def measure(g, cam, tile_size, num_bins, reps=5, warmup=2, sub_bins=0):
    """Median ms of one view's frame (project + bin + the persistent batched
    raster on this view alone) with these options, inputs resident."""
    p = Params(tile_size=tile_size, num_bins=num_bins, sub_bins=sub_bins)
    br = BatchRenderer([cam], [p], device=g["means"].device)
    r = br.views[0]
    s, i = project(g, cam, p)
    b = r.bin(s, i, "binned", sync=True)  # sizes the buffers
    stream = torch.cuda.current_stream()

    def once():
        project(g, cam, p, out=(s, i))
        bb = r.bin(s, i, "binned", sync=False)
        br.rasterize([(s, i)], [bb])

    for _ in range(warmup):
        once()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        once()
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    if int(b.counters[2].item()) != 0:
        return float("inf"), b.num_entries
    return float(np.median(ms)), b.num_entries


def load_cache(path):
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(path, data):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(g, cam, cache_path=DEFAULT_CACHE, candidates=CANDIDATES, reps=5, use_cache=True, sub_bins=SUB_BINS):
    """Returns (Params, record) for this camera and scene; record holds the
    per-candidate times (ms) and whether it came from the cache."""
    key = cache_key(cam, int(g["means"].shape[0]))
    cache = load_cache(cache_path) if cache_path else {}
    hit = cache.get(key) if use_cache else None
    valid = (isinstance(hit, dict) and hit.get("tile_size") in TILE_SIZES
             and isinstance(hit.get("num_bins"), int) and 1 <= hit["num_bins"] <= 1024
             and hit.get("sub_bins", 0) in (0, 1, 2, 4, 8))
    if valid:
        p = Params(tile_size=hit["tile_size"], num_bins=hit["num_bins"], sub_bins=hit.get("sub_bins", 0))
        return p, dict(hit, cached=True)
    table = {}
    runs = [(ts, k, sb) for ts, k in candidates for sb in sub_bins]

    def name(ts, k, sb):
        return f"{ts}x{k}" + ("" if sb in (0, 8) else f"s{sb}")

    for ts, k, sb in runs:
        ms, m = measure(g, cam, ts, k, reps=reps, sub_bins=sb)
        table[name(ts, k, sb)] = {"ms": ms, "entries": m}
    best = min(runs, key=lambda c: table[name(*c)]["ms"])
    rec = {"tile_size": best[0], "num_bins": best[1], "sub_bins": best[2], "ms": table[name(*best)]["ms"],
           "table": table}
    if cache_path:
        cache[key] = rec
        save_cache(cache_path, cache)
    return Params(tile_size=best[0], num_bins=best[1], sub_bins=best[2]), dict(rec, cached=False)
