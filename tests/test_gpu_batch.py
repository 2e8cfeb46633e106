"""Batched multi-camera rendering: one persistent raster launch over all
views, captured in a HIP graph, and the tile/bin autotuner.

Bars: every view's rgb / alpha / last bitwise equal to a per-view
tgs_rasterize with the same arguments (eager batch and every graph replay);
images within 1e-4 of the FP64 oracle on unflagged pixels."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import scenes
from helpers import image_compare, to_np

pytestmark = pytest.mark.gpu

tg = pytest.importorskip("paper_2609_03613_amd")


def dev():
    return torch.device("cuda:0")


def small_views(n_views, scale=0.25, seed=0):
    cams = scenes.ring_cameras(n_views, seed=seed)
    out = []
    for c in cams:
        W, H = max(1, int(round(c["width"] * scale))), max(1, int(round(c["height"] * scale)))
        s = W / c["width"]
        out.append(scenes.camera(c["R"], c["t"], c["fx"] * s, c["fy"] * s, W / 2.0, H / 2.0, W, H))
    return out


MIXED = [dict(tile_size=16, num_bins=64), dict(tile_size=8, num_bins=16), dict(tile_size=32, num_bins=128),
         dict(tile_size=16, num_bins=32), dict(tile_size=32, num_bins=8), dict(tile_size=8, num_bins=64)]


def per_view_reference(g, cams, params, bg):
    outs = []
    for c, p in zip(cams, params):
        # the persistent raster walks every block in one wavefront, as the
        # per-view raster does without the heavy-tile split
        r = tg.Renderer(c, dataclasses.replace(p, split_entries=0), device=dev())
        s, i = tg.project(g, c, p)
        b = r.bin(s, i, "binned")
        outs.append({k: to_np(v) for k, v in r.rasterize(s, i, b, bg=bg).items()})
    torch.cuda.synchronize()
    return outs


def test_batch_equals_per_view_and_oracle():
    gnp, _ = scenes.batched_scene(seed=1, n=30000)
    cams = small_views(6)
    params = [tg.Params(**m) for m in MIXED]
    bg = (0.1, 0.2, 0.3)
    g = tg.to_device(gnp, dev())
    br = tg.BatchRenderer(cams, params, device=dev(), bg=bg)
    outs = br.frame(g, sync=True)
    torch.cuda.synchronize()
    ref = per_view_reference(g, cams, params, bg)
    for v, (o, r) in enumerate(zip(outs, ref)):
        for k in ("rgb", "alpha", "last"):
            assert np.array_equal(to_np(o[k]), r[k]), (v, k)
    for v in (0, 1):
        c = cams[v]
        orc = oracle.render(oracle.project(gnp, c), c["width"], c["height"], bg=bg)
        e_rgb, e_a, nflag = image_compare(to_np(outs[v]["rgb"]), to_np(outs[v]["alpha"]), orc)
        assert e_rgb <= 1e-4 and e_a <= 1e-4, (v, e_rgb, e_a, nflag)


def test_batch_graph_replays_match_eager():
    gnp, _ = scenes.batched_scene(seed=2, n=20000)
    cams = small_views(5, seed=2)
    params = [tg.Params(**m) for m in MIXED[:5]]
    g = tg.to_device(gnp, dev())
    br = tg.BatchRenderer(cams, params, device=dev())
    br.capture(g)
    ref = per_view_reference(g, cams, params, (0.0, 0.0, 0.0))
    for rep in range(3):
        # unrelated eager work between the replays
        tg.Renderer(cams[0], device=dev()).render(g)
        for o in br.outs:
            o["rgb"].fill_(-1.0)
        br.replay()
        torch.cuda.synchronize()
        assert not br.overflowed()
        for v, (o, r) in enumerate(zip(br.outs, ref)):
            for k in ("rgb", "alpha", "last"):
                assert np.array_equal(to_np(o[k]), r[k]), (rep, v, k)


def test_batch_single_view_and_mixed_orders():
    gnp, cam = scenes.small_forward(seed=3)
    g = tg.to_device(gnp, dev())
    p = tg.Params()
    r = tg.Renderer(cam, p, device=dev())
    s, i = tg.project(g, cam, p)
    bb = r.bin(s, i, "binned")
    bgl = r.bin(s, i, "global")
    ref = {k: to_np(v) for k, v in r.rasterize(s, i, bb).items()}
    br = tg.BatchRenderer([cam, cam], [p, p], device=dev())
    outs = br.rasterize([(s, i), (s, i)], [bb, bgl])
    torch.cuda.synchronize()
    for o in outs:
        for k in ("rgb", "alpha", "last"):
            assert np.array_equal(to_np(o[k]), ref[k]), k


def test_batch_argument_errors():
    cam = scenes.small_forward()[1]
    with pytest.raises(ValueError):
        tg.BatchRenderer([cam] * 17, device=dev())
    with pytest.raises(tg.TileGSError):
        tg.BatchRenderer([cam], [tg.Params(tile_size=12)], device=dev())


def test_autotuner_picks_valid_schedule_and_caches(tmp_path):
    from paper_2609_03613_amd import autotune
    gnp, _ = scenes.batched_scene(seed=4, n=20000)
    cam = small_views(1, scale=0.5, seed=4)[0]
    g = tg.to_device(gnp, dev())
    path = str(tmp_path / "tune.json")
    cands = ((8, 16), (16, 64), (32, 32))
    p, rec = autotune.tune(g, cam, cache_path=path, candidates=cands, reps=2)
    assert not rec["cached"]
    assert (p.tile_size, p.num_bins) in cands
    assert rec["ms"] == min(v["ms"] for v in rec["table"].values())
    assert p.sub_bins in autotune.SUB_BINS and len(rec["table"]) == len(cands) * len(autotune.SUB_BINS)
    p2, rec2 = autotune.tune(g, cam, cache_path=path, candidates=cands, reps=2)
    assert rec2["cached"] and (p2.tile_size, p2.num_bins, p2.sub_bins) == (p.tile_size, p.num_bins, p.sub_bins)
    # the tuned schedule renders the same image up to rounding
    a = tg.render(g, cam, p)
    b = tg.render(g, cam)
    torch.cuda.synchronize()
    assert (a["rgb"] - b["rgb"]).abs().max().item() <= 1e-5


@pytest.mark.parametrize("degree", [0, 3])
def test_project_views_equals_per_view_projection(degree):
    # one launch per four cameras, each lane reading its Gaussian once: the
    # splat and info lines of every view equal tgs_project's bit for bit
    # (mixed tile sizes and footprints; 6 views = a full and a partial launch)
    gnp, _ = scenes.batched_scene(seed=7, n=50000)
    if degree == 3:
        rng = np.random.default_rng(7)
        gnp = dict(gnp, sh=rng.normal(0, 0.2, size=(50000, 16, 3)).astype(np.float32), sh_degree=3)
    cams = small_views(6, scale=0.5, seed=7)
    params = [tg.Params(tile_size=ts, footprint=fp) for ts, fp in
              ((16, "opacity"), (8, "opacity"), (32, "three_sigma"), (16, "three_sigma"), (32, "opacity"),
               (8, "three_sigma"))]
    g = tg.to_device(gnp, dev())
    n = 50000
    outs = [(torch.full((n, 16), -1.0, device=dev()), torch.full((n, 4), -1, dtype=torch.int32, device=dev()))
            for _ in cams]
    tg.project_views(g, cams, params, outs)
    torch.cuda.synchronize()
    for v, (c, p) in enumerate(zip(cams, params)):
        s, i = tg.project(g, c, p)
        torch.cuda.synchronize()
        assert torch.equal(outs[v][0], s) and torch.equal(outs[v][1], i), v
        assert int((i[:, 3] > 0).sum()) > 1000, v
