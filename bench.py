"""Benchmark: the depth-binned forward rasterizer against the globally sorted
comparator on one MI355X, scene-shaped 1080p workload (1M Gaussians on 64
spheres/planes, SH degree 3, 1920x1080 at f = 1100), synthetic data.

One step = one binned frame on resident inputs: projection + SH, entry
emission scan, depth range, bin count / offsets / scatter, exact repair,
packed records, binned raster. The globally sorted frame (projection, key
emission, radix sort, tile ranges, plain raster) is timed the same way beside
it. Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--config 1080p|small]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import scenes  # noqa: E402

# Roofline of the raster (no dense contraction, so plain VALU): the published
# MI355X fp32 vector peak, 157.3 TFLOP/s (256 CUs x 128 fp32 lanes x 2 FLOP x
# 2.4 GHz, the lane count that packed fp32 reaches). The algorithmic work is
# 15 fp32 operations per alpha-supported pixel test: 2 sub (dx, dy), 5 for q,
# 1 exp, 1 mul (opacity), 1 min, 1 sub + 1 mul (T (1 - alpha)), 3 fma
# (colour), counted once each.
PEAK_FP32_FLOPS = 157.3e12
FLOPS_PER_TEST = 15
# the same work against one fp32 operation per lane per cycle on 64 lanes per
# CU (the issue rate of unpacked wave64 VALU instructions): 3.93e13 op/s
PEAK_LANE_OPS_64 = 256 * 64 * 2.4e9
HBM_PEAK = 8.0e12


def profiled_counters():
    """Counter figures of the product raster from the committed summary
    (profiles/raster_1080p.md): HBM bytes per launch (FETCH_SIZE and
    WRITE_SIZE scaled by a 256 MiB copy) and the measured VALU issue, or
    None for both when the raster sources changed since the counters were
    taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "raster_1080p.md")
    if not os.path.exists(path):
        return None, None
    h = hashlib.sha256()
    for f in ("raster.hip", "raster.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2609_03613_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    text = open(path).read()
    m_hash = re.search(r"source_sha256: ([0-9a-f]+)", text)
    if not m_hash or m_hash.group(1) != h.hexdigest():
        return None, None
    m_traffic = re.search(r"traffic_bytes_per_launch: ([0-9.e+]+)", text)
    m_valu = re.search(r"valu_insts_per_launch: ([0-9.e+]+)", text)
    m_dur = re.search(r"valu_kernel_us: ([0-9.e+]+)", text)
    traffic = float(m_traffic.group(1)) if m_traffic else None
    issue = None
    if m_valu and m_dur:
        insts, us = float(m_valu.group(1)), float(m_dur.group(1))
        # wave64 VALU instructions x 64 lanes against 64 lanes per CU per cycle
        issue = {"valu_insts_per_launch": insts, "kernel_us": us,
                 "achieved_lane_ops_per_s": insts * 64 / (us * 1e-6), "peak_lane_ops_per_s": PEAK_LANE_OPS_64,
                 "frac": insts * 64 / (us * 1e-6) / PEAK_LANE_OPS_64,
                 "note": "rocprofv3 SQ_INSTS_VALU of the product raster x 64 lanes per kernel second, against one "
                         "wave64 VALU instruction per CU per cycle (256 CUs x 64 lanes x 2.4 GHz)"}
    return traffic, issue


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="1080p", choices=["1080p", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--mode", default="frame", choices=["frame", "kernels", "train", "batch", "batch-replay",
                                                      "learned", "repair", "scale", "stress", "layout",
                                                      "oracle-single"],
                    help="kernels: only launch the product and comparator raster kernels and a "
                         "256 MiB device copy (for profiler counter runs); train: only the training "
                         "step (forward + backward) on the 500k-Gaussian 1297x840 scene; batch-replay: "
                         "only replays of the captured 16-view frame (32-pixel tiles, K = 128, "
                         "2 sub-bins, binnings on one stream), for a kernel trace of the replay alone")
    ap.add_argument("--no-train", action="store_true", help="skip the training-step measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched multi-camera measurement")
    ap.add_argument("--no-repair", action="store_true", help="skip the repair-variant ablation")
    ap.add_argument("--no-ksweep", action="store_true", help="skip the bins-per-tile sweep")
    ap.add_argument("--no-scale", action="store_true", help="skip the 10M-Gaussian scale-up point")
    ap.add_argument("--no-tune", action="store_true", help="training step: skip the autotuned configuration")
    ap.add_argument("--scale-sizes", default="5,10,15,20,25,30",
                    help="Gaussian counts (millions) of --mode scale, comma separated")
    return ap.parse_args()


def kernels_only(args):
    """Launches, after one binned and one global frame, the product raster
    (binned, wave, packed) and the comparator raster (global, plain) `steps`
    times each, then a 256 MiB elementwise copy used to calibrate the
    profiler's HBM byte counters."""
    import torch
    import paper_2609_03613_amd as tg
    dev = torch.device("cuda:0")
    g, cam, desc = workload(args.config)
    gd = tg.to_device(g, dev)
    rb = tg.Renderer(cam, tg.Params(raster="wave", packed=0), device=dev)
    rg = tg.Renderer(cam, tg.Params(raster="plain", packed=0, tile_order=False), device=dev)
    splats, info = tg.project(gd, cam)
    bb = rb.bin(splats, info, "binned", sync=True)
    bgl = rg.bin(splats, info, "global", sync=True)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        rb.rasterize(splats, info, bb)
    for _ in range(args.steps):
        rg.rasterize(splats, info, bgl)
    # plain copy of 256 MiB through an elementwise kernel: reads 256 MiB,
    # writes 256 MiB
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.add(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "kernels", "entries": bb.num_entries, "steps": args.steps,
                      "copy_bytes": src.numel() * 4}), flush=True)


def train_step(args):
    """Forward + backward on the training scene (500k Gaussians of the
    small-forward structure, SH degree 3, 1297x840), binned order, inputs
    resident: project, bin, raster, the loss gradient of mean((rgb -
    target)^2), raster backward, projection backward. Returns per-stage
    median ms (HIP events on the launch stream) and the whole-step rate,
    with the paper's tile size and bins (16 px, K = 64) and with the ones
    the autotuner picks for this camera."""
    import torch
    import paper_2609_03613_amd as tg
    from paper_2609_03613_amd import autotune
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    g, cam = scenes.training_scene(seed=0)
    gd = tg.to_device(g, dev)
    target = torch.as_tensor(scenes.training_target(cam["width"], cam["height"])).to(dev)
    H, W = cam["height"], cam["width"]
    n = int(g["means"].shape[0])
    names = ["project", "bin+repair", "raster", "loss grad", "raster backward", "project backward"]

    def measure(p):
        r = tg.Renderer(cam, p, device=dev)
        splats, info = tg.project(gd, cam, p)
        b = r.bin(splats, info, "binned", sync=True)
        M = b.num_entries
        out = {"rgb": torch.empty((H, W, 3), dtype=torch.float32, device=dev),
               "alpha": torch.empty((H, W), dtype=torch.float32, device=dev),
               "last": torch.empty((H, W), dtype=torch.int32, device=dev),
               "trans": torch.empty((H, W), dtype=torch.float32, device=dev)}
        d_splats = torch.empty((n, 12), dtype=torch.float32, device=dev)
        d_rgb = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
        scale = 2.0 / (3 * W * H)

        def step(evs=None):
            if evs: evs[0].record(stream)
            s, i = tg.project(gd, cam, p)
            if evs: evs[1].record(stream)
            bb = r.bin(s, i, "binned", sync=False)
            if evs: evs[2].record(stream)
            o = r.rasterize(s, i, bb, out=out)
            if evs: evs[3].record(stream)
            torch.sub(o["rgb"], target, out=d_rgb)
            d_rgb.mul_(scale)
            if evs: evs[4].record(stream)
            r.rasterize_backward(s, i, bb, d_rgb, None, out=d_splats, saved=o)
            if evs: evs[5].record(stream)
            grads = tg.project_backward(gd, cam, d_splats)
            if evs: evs[6].record(stream)
            return grads

        for _ in range(args.warmup):
            step()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            step(evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = np.array([[evs[k][j].elapsed_time(evs[k][j + 1]) for j in range(6)] for k in range(args.steps)])
        med = dict(zip(names, np.median(st, 0).tolist()))
        return M, wall, med

    M, wall, med = measure(tg.Params(raster="wave", packed=0))
    res = {"workload": "training scene: 500k Gaussians, SH3, 1297x840, f=1297, binned order",
            "gaussians": n, "entries": M, "ms_per_step": 1000.0 * wall / args.steps,
            "steps_per_s": args.steps / wall, "stage_ms_median": med,
            "backward_ms": med["raster backward"] + med["project backward"],
            "forward_ms": med["project"] + med["bin+repair"] + med["raster"]}
    if not args.no_tune:
        tp, _ = autotune.tune(gd, cam, cache_path=None, reps=3)
        tM, twall, tmed = measure(tp)
        res["tuned"] = {"tile_size": tp.tile_size, "num_bins": tp.num_bins, "sub_bins": tp.sub_bins or 8,
                        "entries": tM,
                        "ms_per_step": 1000.0 * twall / args.steps, "steps_per_s": args.steps / twall,
                        "stage_ms_median": tmed}
    return res

def batch_replay(args):
    """The 16-view batched frame with fixed per-view parameters (32-pixel
    tiles, K = 128, 2 sub-bins: the autotuner's usual choice on this
    workload) and the binnings on one stream, captured once and replayed:
    warmup replays, then `steps` timed ones. No autotuning, eager or
    per-view legs, so that a kernel trace holds the replays alone."""
    import torch
    import paper_2609_03613_amd as tg
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    g, cams = scenes.batched_scene(seed=0)
    gd = tg.to_device(g, dev)
    br = tg.BatchRenderer(cams, [tg.Params(tile_size=32, num_bins=128, sub_bins=2) for _ in cams], device=dev,
                          lanes=1)
    br.capture(gd)
    for _ in range(args.warmup):
        br.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        br.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    assert not br.overflowed()
    return {"workload": "batched: 3M Gaussians (SH0) on 16 ring cameras, 640x360 .. 2560x1440; "
                        "32-pixel tiles, K = 128, 2 sub-bins, binnings on one stream",
            "views": len(cams), "entries": int(sum(br.entries)), "entries_per_view": [int(e) for e in br.entries],
            "replays": args.steps, "ms_per_replay": e0.elapsed_time(e1) / args.steps}


def batched(args):
    """16 cameras of uneven resolution on a ring around 3M Gaussians (SH0):
    per-view tile size and bins from the autotuner, the whole multi-view
    frame (projection in launches of eight views, 16 binnings on four
    streams, one persistent raster launch) captured in a HIP graph and
    replayed. Beside it: the same frame launched eagerly, eagerly with the
    binnings on one stream, and the per-view default path (16 px tiles,
    K = 64, one raster launch per view)."""
    import torch
    import paper_2609_03613_amd as tg
    from paper_2609_03613_amd import autotune
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    g, cams = scenes.batched_scene(seed=0)
    gd = tg.to_device(g, dev)
    tuned, tune_recs = [], []
    for c in cams:
        p, rec = autotune.tune(gd, c, cache_path=None, reps=3)
        tuned.append(p)
        tune_recs.append({"tile_size": p.tile_size, "num_bins": p.num_bins, "sub_bins": p.sub_bins or 8,
                          "ms": rec["ms"]})
    br = tg.BatchRenderer(cams, tuned, device=dev)
    br.capture(gd)
    torch.cuda.synchronize()
    entries = int(sum(br.entries))
    pixels = int(sum(c["width"] * c["height"] for c in cams))

    def timed(fn, k):
        for _ in range(args.warmup):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    graph_ms = timed(br.replay, args.steps)
    assert not br.overflowed()
    eager_ms = timed(lambda: br.frame(gd), args.steps)
    # the same frame with the per-view binnings one after another on one
    # stream, eager and captured
    lanes = br.lanes
    br.lanes = 1
    one_lane_ms = timed(lambda: br.frame(gd), args.steps)
    br.capture(gd)
    graph_one_lane_ms = timed(br.replay, args.steps)
    br.lanes = lanes
    # per-view default path, one raster launch per view
    views = [tg.Renderer(c, tg.Params(), device=dev) for c in cams]
    prep = []
    for r in views:
        s_, i_ = tg.project(gd, r.cam, r.params)
        r.bin(s_, i_, "binned", sync=True)
        prep.append((s_, i_))

    def per_view():
        for r, (s_, i_) in zip(views, prep):
            tg.project(gd, r.cam, r.params, out=(s_, i_))
            b = r.bin(s_, i_, "binned", sync=False)
            r.rasterize(s_, i_, b)

    default_ms = timed(per_view, args.steps)
    # the tuned tile sizes and bins, still one raster launch per view: the
    # tuning's share of the gain, apart from the single persistent launch
    tviews = [tg.Renderer(c, p, device=dev) for c, p in zip(cams, tuned)]
    tprep = []
    for r in tviews:
        s_, i_ = tg.project(gd, r.cam, r.params)
        r.bin(s_, i_, "binned", sync=True)
        tprep.append((s_, i_))

    def per_view_tuned():
        for r, (s_, i_) in zip(tviews, tprep):
            tg.project(gd, r.cam, r.params, out=(s_, i_))
            b = r.bin(s_, i_, "binned", sync=False)
            r.rasterize(s_, i_, b)

    tuned_ms = timed(per_view_tuned, args.steps)
    return {"workload": "batched: 3M Gaussians (SH0) on 16 ring cameras, 640x360 .. 2560x1440",
            "views": len(cams), "pixels": pixels, "entries": entries,
            "graph_ms_per_batch": graph_ms, "eager_batched_ms_per_batch": eager_ms,
            "binning_lanes": lanes, "eager_one_lane_ms_per_batch": one_lane_ms,
            "graph_one_lane_ms_per_batch": graph_one_lane_ms,
            "per_view_default_ms_per_batch": default_ms, "per_view_tuned_ms_per_batch": tuned_ms,
            "tuning_gain": default_ms / tuned_ms, "persistent_launch_gain": tuned_ms / one_lane_ms,
            "binning_overlap_gain": graph_one_lane_ms / graph_ms,
            "views_per_s": len(cams) / (graph_ms * 1e-3), "pairs_per_s": entries / (graph_ms * 1e-3),
            "speedup_vs_per_view_default": default_ms / graph_ms, "tuned": tune_recs}


def learned_bins(args):
    """Steady-state bin construction + exact repair per frame on the
    6M-Gaussian 3840x2160 scene (SH3): fixed K = 64 against the learned
    per-tile counts (features of the previous frame's stream + network
    proposal + binning, all timed), and whether the images are equal."""
    import torch
    import paper_2609_03613_amd as tg
    from paper_2609_03613_amd import bins
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    g, cam = scenes.learned_eval_scene(seed=0)
    gd = tg.to_device(g, dev)
    del g
    w = bins.load_weights()
    fixed = tg.Renderer(cam, tg.Params(), device=dev)
    s, i = tg.project(gd, cam, fixed.params)
    bf = fixed.bin(s, i, "binned", sync=True)
    lb = bins.LearnedBins(cam, weights=w, device=dev, judge=False)
    for _ in range(3):
        lb.bin(s, i, sync=True)  # frame 1 fixed K, then learned; sizes the buffers

    def timed(fn, k):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    steps = max(args.steps, 10)
    # the per-tile machinery with 64 bins everywhere (its own overhead)
    var = tg.Renderer(cam, tg.Params(num_bins=bins.MAX_BINS), device=dev)
    var.set_per_tile_bins(torch.full((fixed.tiles,), 64, dtype=torch.int32, device=dev))
    var.bin(s, i, "binned", sync=True)
    var64_ms = timed(lambda: var.bin(s, i, "binned", sync=False), steps)
    sweep = {}
    for K in (8, 16, 32, 64, 128, 256):
        rk = tg.Renderer(cam, tg.Params(num_bins=K), device=dev)
        rk.bin(s, i, "binned", sync=True)
        sweep[K] = timed(lambda: rk.bin(s, i, "binned", sync=False), steps)
    fixed_ms = timed(lambda: fixed.bin(s, i, "binned", sync=False), steps)
    learned_ms = timed(lambda: lb.bin(s, i, sync=False), steps)
    fixed_ms2 = timed(lambda: fixed.bin(s, i, "binned", sync=False), steps)
    # the product configuration: the network judged against the fixed K at
    # run time (probes included in the mean)
    lj = bins.LearnedBins(cam, weights=w, device=dev, judge=True, warm=4, probe_every=32)
    for _ in range(8):
        lj.bin(s, i, sync=True)
    judged_ms = timed(lambda: lj.bin(s, i, sync=False), max(steps, 32))
    r, b = lb.bin(s, i, sync=True)
    out_l = r.rasterize(s, i, b)
    out_f = fixed.rasterize(s, i, fixed.bin(s, i, "binned", sync=True))
    torch.cuda.synchronize()
    same = bool(torch.equal(out_l["rgb"], out_f["rgb"]) and torch.equal(out_l["last"], out_f["last"]))
    kt = lb.kt.cpu().numpy()
    ks, counts = np.unique(kt, return_counts=True)
    fixed_ms = min(fixed_ms, fixed_ms2)
    return {"workload": "6M Gaussians on 64 surfaces (SH3), 3840x2160, f=2200", "entries": bf.num_entries,
            "weights": "trained" if w is not None else "missing (fixed K fallback)",
            "fixed64_bin_ms": fixed_ms, "learned_bin_ms": learned_ms, "gain": fixed_ms / learned_ms,
            "judged_bin_ms": judged_ms, "judged_gain": fixed_ms / judged_ms, "judge_choice": lj.choice(),
            "per_tile_machinery_all64_ms": var64_ms, "uniform_k_sweep_ms": sweep,
            "images_equal": same, "per_tile_bins": {int(k): int(c) for k, c in zip(ks, counts)}}


def repair_ablation(args, gd, cam):
    """Repair variants on the same workload: the exact default, every
    segment sorted on near-depth bins, the paper's rule-based selection with
    the 25 % entry budget (near-depth bins, and plain depth bins), and no
    repair. Per variant: bin stage, raster and whole-frame ms (HIP events,
    medians), the repaired share of the entries, and the image error against
    the exact image (max |delta|, PSNR over RGB, pixels off by more than
    1e-4), plus the largest change between two frames of the same variant
    (unsorted segments keep the scatter's order, which varies)."""
    import torch
    import paper_2609_03613_amd as tg
    dev = gd["means"].device
    stream = torch.cuda.current_stream()
    variants = [("exact: all segments, depth bins", tg.Params()),
                ("all segments, near-depth bins", tg.Params(near_shift=True)),
                ("paper: rules + 25% budget, near-depth bins", tg.paper_params()),
                ("rules + 25% budget, depth bins", tg.Params(repair="rules")),
                ("none, near-depth bins", tg.Params(near_shift=True, repair="none"))]
    steps = max(args.steps, 10)

    def timed(fn):
        for _ in range(3):
            fn()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        e[0].record(stream)
        for k in range(steps):
            fn()
            e[k + 1].record(stream)
        torch.cuda.synchronize()
        return float(np.median([e[k].elapsed_time(e[k + 1]) for k in range(steps)]))

    out, ref = {}, None
    for name, prm in variants:
        r = tg.Renderer(cam, prm, device=dev)
        s, i = tg.project(gd, cam)
        b = r.bin(s, i, "binned", sync=True)
        M = b.num_entries
        img = r.rasterize(s, i, b)
        frame_out = {k: torch.empty_like(v) for k, v in img.items()}
        bin_ms = timed(lambda: r.bin(s, i, "binned", sync=False))
        b = r.bin(s, i, "binned", sync=True)
        rep = int(b.counters[3].item())
        segs = int(b.repaired[: r.tiles * prm.num_bins].sum().item())
        img = {k: v.clone() for k, v in r.rasterize(s, i, b).items()}
        raster_ms = timed(lambda: r.rasterize(s, i, b, out=frame_out))

        def frame():
            s2, i2 = tg.project(gd, cam, prm, out=(s, i))
            r.rasterize(s2, i2, r.bin(s2, i2, "binned", sync=False), out=frame_out)
        frame_ms = timed(frame)
        b2 = r.bin(s, i, "binned", sync=True)
        img2 = r.rasterize(s, i, b2)
        torch.cuda.synchronize()
        rgb = img["rgb"].double()
        if ref is None:
            ref = rgb
        d = (rgb - ref).abs()
        mse = float(((rgb - ref) ** 2).mean().item())
        out[name] = {"bin_ms": bin_ms, "raster_ms": raster_ms, "frame_ms": frame_ms,
                     "repaired_entries_frac": rep / max(M, 1), "repaired_segments": segs,
                     "max_abs_delta_vs_exact": float(d.max().item()),
                     "psnr_vs_exact_db": (float("inf") if mse == 0.0 else float(10.0 * np.log10(1.0 / mse))),
                     "pixels_off_1e-4": int((d.amax(dim=2) > 1e-4).sum().item()),
                     "frame_to_frame_max_delta": float((img2["rgb"].double() - rgb).abs().max().item())}
    return out


def k_sweep(args, gd, cam):
    """Bins per tile K in {4, ..., 128} on the same workload (the paper's
    bin-count ablation): bin stage, raster and whole-frame ms, and whether
    the image equals the K = 64 one bit for bit (exact repair makes the
    stream independent of K)."""
    import torch
    import paper_2609_03613_amd as tg
    dev = gd["means"].device
    stream = torch.cuda.current_stream()
    steps = max(args.steps, 10)

    def timed(fn):
        for _ in range(3):
            fn()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        e[0].record(stream)
        for k in range(steps):
            fn()
            e[k + 1].record(stream)
        torch.cuda.synchronize()
        return float(np.median([e[k].elapsed_time(e[k + 1]) for k in range(steps)]))

    out, ref = {}, None
    for K in (64, 4, 8, 16, 32, 128):
        prm = tg.Params(num_bins=K)
        r = tg.Renderer(cam, prm, device=dev)
        s, i = tg.project(gd, cam)
        b = r.bin(s, i, "binned", sync=True)
        img = {k: v.clone() for k, v in r.rasterize(s, i, b).items()}
        buf = {k: torch.empty_like(v) for k, v in img.items()}
        bin_ms = timed(lambda: r.bin(s, i, "binned", sync=False))
        raster_ms = timed(lambda: r.rasterize(s, i, b, out=buf))

        def frame():
            s2, i2 = tg.project(gd, cam, prm, out=(s, i))
            r.rasterize(s2, i2, r.bin(s2, i2, "binned", sync=False), out=buf)
        frame_ms = timed(frame)
        if ref is None:
            ref = img
        same = bool(torch.equal(img["rgb"], ref["rgb"]) and torch.equal(img["last"], ref["last"]))
        lens = torch.diff(b.offsets[: r.tiles * K + 1].long())
        out[K] = {"bin_ms": bin_ms, "raster_ms": raster_ms, "frame_ms": frame_ms, "image_equals_k64": same,
                  "segments_ge2": int((lens >= 2).sum().item()), "longest_segment": int(lens.max().item())}
    return {int(k): out[k] for k in sorted(out)}


def scale_up(args):
    """Synthetic scale-up with the 1080p workload's structure: N = 5M ..
    30M Gaussians (seeded random subsets of one 30M-Gaussian draw on the 64
    surfaces, SH3, same 1920x1080 camera); per N the ordering stage (binned:
    range, bins, repair; global: key emission, radix sort, tile ranges), the
    raster and the whole frame, medians over the steps (the paper's
    scale-up table)."""
    import torch
    import paper_2609_03613_amd as tg
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    steps = max(min(args.steps, 10), 5)
    sizes = sorted({int(v) for v in args.scale_sizes.split(",") if v.strip()})
    top = sizes[-1]
    t0 = time.perf_counter()
    g_all, cam = scenes.scene_1080p(seed=0, n=top * 1_000_000)
    print(f"scale: generated {top}M Gaussians in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    perm = np.random.default_rng(1).permutation(top * 1_000_000)
    rows = {}
    for n_m in sizes:
        idx = np.sort(perm[: n_m * 1_000_000])
        gd = tg.to_device(scenes.subset(g_all, idx), dev)
        rb = tg.Renderer(cam, tg.Params(), device=dev)
        rg = tg.Renderer(cam, tg.Params(raster="plain", tile_order=False), device=dev)
        s, i = tg.project(gd, cam)
        bb = rb.bin(s, i, "binned", sync=True)
        bgl = rg.bin(s, i, "global", sync=True)
        M = bb.num_entries
        H, W = cam["height"], cam["width"]
        buf = {"rgb": torch.empty((H, W, 3), device=dev), "alpha": torch.empty((H, W), device=dev),
               "last": torch.empty((H, W), dtype=torch.int32, device=dev)}

        def stages(r, order):
            ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
            for k in range(steps + 2):
                e = ev[k - 2] if k >= 2 else None
                if e: e[0].record(stream)
                s2, i2 = tg.project(gd, cam, r.params, out=(s, i))
                if e: e[1].record(stream)
                b2 = r.bin(s2, i2, order, sync=(order == "global"))
                if e: e[2].record(stream)
                r.rasterize(s2, i2, b2, out=buf)
                if e: e[3].record(stream)
            torch.cuda.synchronize()
            a = np.array([[e[j].elapsed_time(e[j + 1]) for j in range(3)] + [e[0].elapsed_time(e[3])] for e in ev])
            return np.median(a, 0).tolist()

        pb, sb, rb_ms, tb = stages(rb, "binned")
        pg, sg, rg_ms, tg_ms = stages(rg, "global")
        rows[n_m] = {"entries": M, "sort_ms": {"global": sg, "binned": sb, "x": sg / sb},
                     "raster_ms": {"global": rg_ms, "binned": rb_ms, "x": rg_ms / rb_ms},
                     "total_ms": {"global": tg_ms, "binned": tb, "x": tg_ms / tb}, "project_ms": pb}
        print(f"scale: {n_m}M done ({M} entries, binned {tb:.3f} ms, global {tg_ms:.3f} ms)",
              file=sys.stderr, flush=True)
        del gd, rb, rg, s, i, bb, bgl
        torch.cuda.empty_cache()
    return {"workload": "1080p scene-shaped structure, %s M Gaussians (random subsets of one draw), SH3, "
                        "1920x1080, f=1100" % ",".join(map(str, sizes)), "rows": rows}


def _stage_times(tg, r, gd, cam, order, steps, stream):
    """Median project / ordering / raster / frame ms of `steps` frames."""
    import torch
    s, i = tg.project(gd, cam, r.params)
    b = r.bin(s, i, order, sync=True)
    out = r.rasterize(s, i, b)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for k in range(steps + 2):
        e = ev[k - 2] if k >= 2 else None
        if e: e[0].record(stream)
        tg.project(gd, cam, r.params, out=(s, i))
        if e: e[1].record(stream)
        b2 = r.bin(s, i, order, sync=(order == "global"))
        if e: e[2].record(stream)
        r.rasterize(s, i, b2, out=out)
        if e: e[3].record(stream)
    torch.cuda.synchronize()
    a = np.array([[e[j].elapsed_time(e[j + 1]) for j in range(3)] + [e[0].elapsed_time(e[3])] for e in ev])
    med = np.median(a, 0).tolist()
    return {"project": med[0], "order": med[1], "raster": med[2], "frame": med[3]}, b, out


def stress(args):
    """Depth-distribution stress (sparse, dense slab in a wide range,
    bimodal; 1920x1080) and a resolution sweep of the 1080p scene (640x360
    .. 3840x2160, focal length scaled with the width): binned against
    globally sorted frames (project, ordering, raster, whole frame), the
    entry and segment statistics, whether the paper's repair budget is
    active (kept entries above 25 % of M) and whether the images agree."""
    import torch
    import paper_2609_03613_amd as tg
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    steps = max(min(args.steps, 10), 5)

    def compare(g, cam):
        gd = tg.to_device(g, dev)
        rb = tg.Renderer(cam, tg.Params(), device=dev)
        rg = tg.Renderer(cam, tg.Params(raster="plain", tile_order=False), device=dev)
        tb, bb, ob = _stage_times(tg, rb, gd, cam, "binned", steps, stream)
        M = bb.num_entries if bb.num_entries is not None else int(bb.counters[0].item())
        bb = rb.bin(*tg.project(gd, cam), "binned", sync=True)
        lens = torch.diff(bb.offsets[: rb.tiles * 64 + 1].long())
        tgl, bg, og = _stage_times(tg, rg, gd, cam, "global", steps, stream)
        rp = tg.Renderer(cam, tg.paper_params(repair_budget=1.0), device=dev)
        sp, ip = tg.project(gd, cam)
        kept = int(rp.bin(sp, ip, "binned", sync=True).counters[3].item())
        r0 = tg.Renderer(cam, tg.Params(split_entries=0), device=dev)
        o0 = r0.rasterize(sp, ip, r0.bin(sp, ip, "binned", sync=True))
        torch.cuda.synchronize()
        row = {"entries": M, "binned_ms": tb, "global_ms": tgl,
               "raster_x": tgl["raster"] / tb["raster"], "order_x": tgl["order"] / tb["order"],
               "frame_x": tgl["frame"] / tb["frame"], "longest_segment": int(lens.max().item()),
               "entries_in_segments_over_64": float(lens[lens > 64].sum().item()) / max(M, 1),
               "paper_kept_frac": kept / max(M, 1), "paper_budget_active": kept > 0.25 * M,
               "split_tiles": bb.split()[0],
               "unsplit_equals_global": bool(torch.equal(o0["rgb"], og["rgb"])),
               "split_max_abs_diff": float((ob["rgb"] - o0["rgb"]).abs().max().item())}
        del gd
        torch.cuda.empty_cache()
        return row

    out = {"depth": {}, "resolution": {}}
    for kind in scenes.STRESS_KINDS:
        g, cam = scenes.depth_stress_scene(kind, seed=0)
        out["depth"][kind] = compare(g, cam)
        print(f"stress: {kind} done", file=sys.stderr, flush=True)
    g1, _ = scenes.scene_1080p(seed=0)
    for W, H in ((640, 360), (1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)):
        f = 1100.0 * W / 1920.0
        cam = scenes.camera(np.eye(3), np.array([0.0, 0.0, 15.0]), f, f, W / 2.0, H / 2.0, W, H)
        out["resolution"][f"{W}x{H}"] = compare(g1, cam)
        print(f"stress: {W}x{H} done", file=sys.stderr, flush=True)
    return out


def layout(args):
    """Storage layout of the Gaussians (the paper's raster-order-aware
    storage direction): the 1080p workload and the 500k training scene with
    the Gaussians in generation order (points drawn surface by surface, in
    random order on each) against Z-order of their means; per-stage median
    ms of the binned frame, and the largest image difference (the order of
    equal depths follows the Gaussian id, so only exact depth ties can move)."""
    import torch
    import paper_2609_03613_amd as tg
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    steps = max(args.steps, 10)
    out = {}
    for name, (g, cam) in (("1080p scene-shaped, 1M", scenes.scene_1080p(seed=0)),
                           ("training scene, 500k", scenes.training_scene(seed=0))):
        row, imgs = {}, {}
        for order, gg in (("generation", g), ("morton", scenes.morton_sorted(g))):
            gd = tg.to_device(gg, dev)
            r = tg.Renderer(cam, tg.Params(), device=dev)
            st, _, img = _stage_times(tg, r, gd, cam, "binned", steps, stream)
            row[order] = st
            imgs[order] = img["rgb"].clone()
            del gd
        row["raster_x"] = row["generation"]["raster"] / row["morton"]["raster"]
        row["frame_x"] = row["generation"]["frame"] / row["morton"]["frame"]
        row["max_abs_image_diff"] = float((imgs["generation"] - imgs["morton"]).abs().max().item())
        out[name] = row
        torch.cuda.empty_cache()
    return out


def workload(name):
    if name == "1080p":
        g, cam = scenes.scene_1080p(seed=0)
        desc = "1080p scene-shaped: 1M Gaussians on 64 spheres/planes, SH3, 1920x1080, f=1100"
    else:
        g, cam = scenes.small_forward(seed=0)
        desc = "small forward: 2k Gaussians, SH0, 128x128, f=128"
    return g, cam, desc


def cpu_baseline(g, cam, budget_s, gpu_image=None):
    """The FP64 oracle (project + tiled composite of every pixel) on the
    host's cores, repeated whole frames for about budget_s seconds; one frame
    on a single core in a child process; the oracle on the small forward
    workload and on the 200-Gaussian adjoint sub-case of the training scene.
    With gpu_image (rgb, alpha of the product frame), the largest difference
    to the oracle's frame over the pixels it did not flag, and their count."""
    import subprocess
    import oracle
    frames, M = 0, 0
    t0 = time.perf_counter()
    while True:
        p = oracle.project(g, cam)
        M = oracle.count_entries(p["rect"])
        ref = oracle.render(p, cam["width"], cam["height"])
        frames += 1
        el = time.perf_counter() - t0
        if el >= budget_s or frames >= 50:
            break
    out = {"value": M * frames / el, "unit": "Gaussian-tile pairs/s", "cores": oracle.num_threads(),
           "kind": "oracle", "sample": f"{frames} whole frame(s) of the same workload in {el:.1f} s "
                                      f"(FP64 projection + tiled compositing of all {cam['width']}x{cam['height']} px)",
           "ms_per_frame": 1000.0 * el / frames}
    if gpu_image is not None:
        rgb, alpha = gpu_image
        m = ref["flags"] == 0
        out["max_abs_vs_oracle"] = {"rgb": float(np.abs(rgb.astype(np.float64) - ref["rgb"])[m].max()),
                                    "alpha": float(np.abs(alpha.astype(np.float64) - ref["alpha"])[m].max())}
        out["masked_pixels"] = int((~m).sum())
        out["pixels"] = int(m.size)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--mode", "oracle-single"], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode == 0 and r.stdout.strip():
        out["single_core"] = json.loads(r.stdout.strip().splitlines()[-1])
    else:
        out["single_core"] = {"error": (r.stderr or "")[-300:]}
    # the small forward workload and the adjoint sub-case, all host cores
    gs, cs = scenes.small_forward(seed=0)
    t0 = time.perf_counter()
    k = 0
    while k < 20 or time.perf_counter() - t0 < 0.5:
        ps = oracle.project(gs, cs)
        oracle.render(ps, cs["width"], cs["height"])
        k += 1
    out["small_forward_ms_per_frame"] = 1000.0 * (time.perf_counter() - t0) / k
    gf, cf = scenes.fd_subcase()
    tgt = scenes.training_target(cf["width"], cf["height"])
    g64 = {kk: (np.asarray(v, np.float64) if kk != "sh_degree" else v) for kk, v in gf.items()}
    t0 = time.perf_counter()
    k = 0
    while k < 10 or time.perf_counter() - t0 < 0.5:
        a = oracle.adjoint(g64, cf)
        _, up = oracle.mse_upstream(a["rgb"], tgt)
        oracle.adjoint(g64, cf, d_img=up)
        k += 1
    out["adjoint_subcase_ms"] = 1000.0 * (time.perf_counter() - t0) / k
    return out


def oracle_single_core():
    """One whole 1080p oracle frame on one core (run as a child process with
    OMP_NUM_THREADS=1); prints one JSON line."""
    import oracle
    g, cam, _ = workload("1080p")
    t0 = time.perf_counter()
    p = oracle.project(g, cam)
    M = oracle.count_entries(p["rect"])
    oracle.render(p, cam["width"], cam["height"])
    el = time.perf_counter() - t0
    print(json.dumps({"cores": oracle.num_threads(), "ms_per_frame": 1000.0 * el, "value": M / el,
                      "unit": "Gaussian-tile pairs/s", "sample": "1 whole frame"}), flush=True)


def timed_frames(frame, steps, stream):
    """Runs `steps` frames with 4 HIP events each on the launch stream;
    returns (wall ms per frame, [steps, 3] stage ms, [steps] frame ms)."""
    import torch
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        frame(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = np.array([[evs[k][j].elapsed_time(evs[k][j + 1]) for j in range(3)] for k in range(steps)])
    tot = np.array([evs[k][0].elapsed_time(evs[k][3]) for k in range(steps)])
    return 1000.0 * wall / steps, st, tot


def scale_point(args, n_m=10):
    """One point of the synthetic scale-up (the 1080p structure with n_m
    million Gaussians): ordering stage, raster and whole frame, binned
    against the globally sorted comparator (sync-free, capacity sized to the
    entry count), medians of HIP-event-timed frames."""
    import torch
    import paper_2609_03613_amd as tg
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    steps = max(min(args.steps, 10), 5)
    g, cam = scenes.scene_1080p(seed=0, n=n_m * 1_000_000)
    gd = tg.to_device(g, dev)
    del g
    rb = tg.Renderer(cam, tg.Params(), device=dev)
    rg = tg.Renderer(cam, tg.Params(raster="plain", tile_order=False), device=dev)
    s, i = tg.project(gd, cam)
    M = rb.bin(s, i, "binned", sync=True).num_entries
    rg.bin(s, i, "global", capacity=int(M * 1.02) + 1024, sync=True)
    H, W = cam["height"], cam["width"]
    buf = {"rgb": torch.empty((H, W, 3), device=dev), "alpha": torch.empty((H, W), device=dev),
           "last": torch.empty((H, W), dtype=torch.int32, device=dev)}

    def run(r, order):
        def frame(e=None):
            if e: e[0].record(stream)
            tg.project(gd, cam, r.params, out=(s, i))
            if e: e[1].record(stream)
            b = r.bin(s, i, order, sync=False)
            if e: e[2].record(stream)
            r.rasterize(s, i, b, out=buf)
            if e: e[3].record(stream)
        for _ in range(2):
            frame()
        _, st, tot = timed_frames(frame, steps, stream)
        med = np.median(st, 0)
        return {"order_ms": float(med[1]), "raster_ms": float(med[2]), "frame_ms": float(np.median(tot))}

    b = run(rb, "binned")
    gl = run(rg, "global")
    del gd, rb, rg, s, i
    torch.cuda.empty_cache()
    return {"workload": f"1080p scene-shaped structure, {n_m}M Gaussians, SH3, 1920x1080, f=1100",
            "gaussians": n_m * 1_000_000, "entries": M, "binned": b, "global": gl,
            "order_x": gl["order_ms"] / b["order_ms"], "raster_x": gl["raster_ms"] / b["raster_ms"],
            "frame_x": gl["frame_ms"] / b["frame_ms"], "pairs_per_s": M / (b["frame_ms"] * 1e-3)}


def main():
    args = parse()
    if args.mode == "oracle-single":
        return oracle_single_core()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path would shard by screen "
              f"tiles, but multi-GPU runs are not implemented", file=sys.stderr)
        sys.exit(2)
    if args.mode == "kernels":
        return kernels_only(args)
    if args.mode == "train":
        print(json.dumps({"mode": "train", **train_step(args)}), flush=True)
        return
    if args.mode == "batch":
        print(json.dumps({"mode": "batch", **batched(args)}), flush=True)
        return
    if args.mode == "batch-replay":
        print(json.dumps({"mode": "batch-replay", **batch_replay(args)}), flush=True)
        return
    if args.mode == "learned":
        print(json.dumps({"mode": "learned", **learned_bins(args)}), flush=True)
        return
    if args.mode == "stress":
        print(json.dumps({"mode": "stress", **stress(args)}), flush=True)
        return
    if args.mode == "scale":
        print(json.dumps({"mode": "scale", **scale_up(args)}), flush=True)
        return
    if args.mode == "layout":
        print(json.dumps({"mode": "layout", **layout(args)}), flush=True)
        return
    if args.mode == "repair":
        import torch
        import paper_2609_03613_amd as tg
        g, cam, desc = workload(args.config)
        gd = tg.to_device(g, torch.device("cuda:0"))
        print(json.dumps({"mode": "repair", "workload": desc, "variants": repair_ablation(args, gd, cam)}),
              flush=True)
        return
    import torch
    import paper_2609_03613_amd as tg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    g, cam, desc = workload(args.config)
    gd = tg.to_device(g, dev)
    stream = torch.cuda.current_stream()
    H, W = cam["height"], cam["width"]

    # the product: binned stream, wave raster gathering by id and culling per
    # 8x8 block, heaviest tiles first, the longest tiles split
    rb = tg.Renderer(cam, tg.Params(raster="wave", packed=0), device=dev)
    # the comparator: globally sorted stream, one workgroup per tile gathering
    # batches by id, tiles in raster order
    rg = tg.Renderer(cam, tg.Params(raster="plain", packed=0, tile_order=False), device=dev)
    # the comparator's stream through the product raster (tile order + split):
    # separates what binning earns from what the raster kernel earns
    rgw = tg.Renderer(cam, tg.Params(raster="wave", packed=0), device=dev)
    # the comparator as the library first shipped it: host read of the entry
    # count before the sort
    rgs = tg.Renderer(cam, tg.Params(raster="plain", packed=0, tile_order=False), device=dev)

    # first frames size the entry buffers; the sync-free global streams get a
    # capacity of the entry count + 2 % (their sort runs over the capacity)
    splats, info = tg.project(gd, cam)
    M = rb.bin(splats, info, "binned", sync=True).num_entries
    cap_g = int(M * 1.02) + 1024
    for r in (rg, rgw, rgs):
        assert r.bin(splats, info, "global", capacity=cap_g, sync=True).num_entries == M
    torch.cuda.synchronize()

    def mk():
        return {"rgb": torch.empty((H, W, 3), dtype=torch.float32, device=dev),
                "alpha": torch.empty((H, W), dtype=torch.float32, device=dev),
                "last": torch.empty((H, W), dtype=torch.int32, device=dev)}

    bufs = {k: mk() for k in ("binned", "global", "global_product_raster", "global_host_sync")}

    def frame_fn(r, order, out, sync=False):
        def frame(evs=None):
            if evs: evs[0].record(stream)
            s, i = tg.project(gd, cam, r.params, out=(splats, info))
            if evs: evs[1].record(stream)
            b = r.bin(s, i, order, sync=sync)
            if evs: evs[2].record(stream)
            r.rasterize(s, i, b, out=out)
            if evs: evs[3].record(stream)
        return frame

    frames = {"binned": frame_fn(rb, "binned", bufs["binned"]),
              "global": frame_fn(rg, "global", bufs["global"]),
              "global_product_raster": frame_fn(rgw, "global", bufs["global_product_raster"]),
              "global_host_sync": frame_fn(rgs, "global", bufs["global_host_sync"], sync=True)}
    for _ in range(args.warmup):
        for f in frames.values():
            f()
    torch.cuda.synchronize()
    timing = {k: timed_frames(f, args.steps, stream) for k, f in frames.items()}
    frame_ms = {k: v[0] for k, v in timing.items()}
    stage = {k: np.median(v[1], 0).tolist() for k, v in timing.items()}

    # raster kernel alone, back to back on prepared streams (HIP events on the
    # launch stream around every launch)
    def raster_only(r, b, out):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        evs[0].record(stream)
        for k in range(args.steps):
            r.rasterize(splats, info, b, out=out)
            evs[k + 1].record(stream)
        torch.cuda.synchronize()
        return np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])

    tg.project(gd, cam, out=(splats, info))
    bb = rb.bin(splats, info, "binned", sync=False)
    bgl = rg.bin(splats, info, "global", sync=False)
    bglw = rgw.bin(splats, info, "global", sync=False)
    ras_b = raster_only(rb, bb, bufs["binned"])
    ras_g = raster_only(rg, bgl, bufs["global"])
    ras_gw = raster_only(rgw, bglw, bufs["global_product_raster"])
    same_product = bool(torch.equal(bufs["binned"]["rgb"], bufs["global_product_raster"]["rgb"]) and
                        torch.equal(bufs["binned"]["last"], bufs["global_product_raster"]["last"]))

    # ablation: the same streams through the other kernels and layouts; each
    # binned variant re-bins with its own options, timed separately
    import copy
    bb_noorder = copy.copy(bb)
    bb_noorder.tile_order = None
    ablation = {"binned wave cull-in-raster (product)": float(np.median(ras_b)),
                "binned wave cull-in-raster, raster-order tiles": float(np.median(raster_only(rb, bb_noorder,
                                                                                             bufs["binned"]))),
                "global wave cull-in-raster, tile order + split (product raster)": float(np.median(ras_gw))}
    bin_ms = {}
    for name, prm in [("binned wave records+masks", tg.Params(raster="wave", packed=1)),
                      ("binned wave masks", tg.Params(raster="wave", packed=2)),
                      ("binned plain gather-by-id", tg.Params(raster="plain", packed=0))]:
        rv = tg.Renderer(cam, prm, device=dev)
        bv = rv.bin(splats, info, "binned", sync=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            rv.bin(splats, info, "binned", sync=False)
        e1.record(stream)
        torch.cuda.synchronize()
        bin_ms[name] = e0.elapsed_time(e1) / args.steps
        ablation[name] = float(np.median(raster_only(rv, bv, bufs["binned"])))
        del rv, bv
    ablation["global plain gather-by-id (comparator)"] = float(np.median(ras_g))

    # instrumented launches (outside the timed region): algorithmic work
    cb = rb.rasterize(splats, info, bb, counts=True)
    cg = rg.rasterize(splats, info, bgl, counts=True)
    torch.cuda.synchronize()
    n_support = int(cb["n_support"].sum().item())
    n_visit_b = int(cb["n_visit"].sum().item())
    n_visit_g = int(cg["n_visit"].sum().item())
    # the product equals the comparator bit for bit, with and without the
    # heavy-tile quad walk (the same per-pixel chain)
    r_unsplit = tg.Renderer(cam, tg.Params(raster="wave", packed=0, split_entries=0), device=dev)
    cu = r_unsplit.rasterize(splats, info, r_unsplit.bin(splats, info, "binned", sync=True), counts=True)
    torch.cuda.synchronize()
    same = bool(torch.equal(cu["rgb"], cg["rgb"]) and torch.equal(cu["last"], cg["last"]))
    split_diff = float((cb["rgb"] - cu["rgb"]).abs().max().item())
    split_last_equal = bool(torch.equal(cb["last"], cu["last"]))
    split_bitwise = bool(torch.equal(cb["rgb"], cu["rgb"]) and torch.equal(cb["alpha"], cu["alpha"])
                         and split_last_equal)
    product_same = bool(torch.equal(cb["rgb"], cg["rgb"]) and torch.equal(cb["last"], cg["last"]))
    n_split = list(bb.split())
    gpu_image = (cb["rgb"].cpu().numpy(), cb["alpha"].cpu().numpy())
    del cb, cg, cu, r_unsplit

    raster_ms_b = float(np.median(ras_b))
    raster_ms_g = float(np.median(ras_g))
    raster_ms_gw = float(np.median(ras_gw))
    t_mean = float(np.mean(ras_b)) * 1e-3
    flops = n_support * FLOPS_PER_TEST
    achieved = flops / t_mean
    traffic, issue = profiled_counters()
    fb = frame_ms["binned"]
    result = {
        "metric": "raster-kernel ms/frame at 1080p, binned vs global-sort; Gaussian-tile pairs/s",
        "value": M / (fb * 1e-3),
        "unit": "Gaussian-tile pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fb,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "gaussians": int(g["means"].shape[0]), "width": W, "height": H,
                   "tile": 16, "bins": 64, "entries": M},
        "raster_ms": {"binned": raster_ms_b, "global": raster_ms_g, "speedup": raster_ms_g / raster_ms_b,
                      "binned_p10_p90": [float(np.percentile(ras_b, 10)), float(np.percentile(ras_b, 90))],
                      "global_p10_p90": [float(np.percentile(ras_g, 10)), float(np.percentile(ras_g, 90))],
                      "global_product_raster": raster_ms_gw},
        "raster_pairs_per_s": {"binned": M / (raster_ms_b * 1e-3), "global": M / (raster_ms_g * 1e-3)},
        "frame_ms": {"binned": fb, "global": frame_ms["global"], "speedup": frame_ms["global"] / fb,
                     "global_product_raster": frame_ms["global_product_raster"],
                     "global_host_sync": frame_ms["global_host_sync"]},
        "fps": {"binned": 1000.0 / fb, "global": 1000.0 / frame_ms["global"]},
        "binning_attributable": {
            "note": "the same product raster (wave walk, heaviest tiles first, long-tail tiles in the quad walk) on the binned "
                    "and on the globally sorted stream: what the ordering stage itself earns",
            "ordering_stage_x": stage["global_product_raster"][1] / stage["binned"][1],
            "frame_same_raster_x": frame_ms["global_product_raster"] / fb,
            "raster_same_kernel_x": raster_ms_gw / raster_ms_b,
            "images_equal": same_product},
        "stage_ms_median": {
            "binned": dict(zip(["project", "bin+repair", "raster"], stage["binned"])),
            "global": dict(zip(["project", "emit+sort+ranges", "raster"], stage["global"])),
            "global_product_raster": dict(zip(["project", "emit+sort+ranges+tile order", "raster"],
                                              stage["global_product_raster"])),
            "global_host_sync": dict(zip(["project", "emit+count read+sort+ranges", "raster"],
                                         stage["global_host_sync"])),
        },
        "tests_per_pixel": {"support": n_support / (W * H), "visit_binned": n_visit_b / (W * H),
                            "visit_global": n_visit_g / (W * H)},
        "images_bitwise_equal": same,
        "product_equals_comparator": product_same,
        "heavy_tile_split": {"tiles": n_split[0], "min_entries": n_split[1], "waves_per_block": 4,
                             "walk": "quad: a 4x4 quarter per wavefront, 4 lanes per pixel, 4 entries per step",
                             "bitwise_equal_to_unsplit": split_bitwise,
                             "max_abs_diff_vs_unsplit": split_diff, "last_equal": split_last_equal},
        "raster_ablation_ms": ablation,
        "bin_stage_ms_by_variant": bin_ms,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_FLOPS / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_FLOPS, "traffic": traffic,
                     "kernel": "raster_split_kernel<1,false> (binned, gather by id, per-block cull, long-tail "
                               "tiles in the quad walk)",
                     "work": f"{n_support} alpha-supported pixel tests x {FLOPS_PER_TEST} fp32 ops / mean launch "
                             f"{t_mean * 1e6:.1f} us",
                     "frac_vs_64_lanes_per_cu": flops / t_mean / PEAK_LANE_OPS_64,
                     "frac_with_visits": n_visit_b * FLOPS_PER_TEST / t_mean / PEAK_FP32_FLOPS,
                     "valu_issue": issue},
    }
    if not args.no_scale:
        result["scale_point"] = scale_point(args)
    if not args.no_repair:
        result["repair_ablation"] = repair_ablation(args, gd, cam)
    if not args.no_ksweep:
        result["k_sweep"] = k_sweep(args, gd, cam)
    if not args.no_train:
        result["training_step"] = train_step(args)
    if not args.no_batch:
        result["batched"] = batched(args)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(g, cam, args.cpu_seconds, gpu_image)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
