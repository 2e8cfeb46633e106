"""Heavy-tile split of the WAVE raster: the tiles with at least
split_entries entries get four wavefronts per 8x8 block, one 4x4 quarter
each, in the quad walk (four lanes per pixel, four entries per step, the
per-pixel chain of the one-lane walk). The scenes here are uniformly dense,
so the bound relative to the mean tile (split_mean_factor) is turned off to
force the split; the default bound is checked on its own.

Bars: images within 1e-4 of the FP64 oracle with last ids and contribution
counts equal on unflagged pixels; against the unsplit raster bitwise equal
(rgb, alpha, transmittance, last ids, contribution and support counts),
with at most as many visited entries (the finer quarter cull) and at least
the supported ones; scenes dense enough that pixels stop; overflow still
yields NaN; no split without a dispatch order."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from helpers import image_compare, to_np

pytestmark = pytest.mark.gpu

tg = pytest.importorskip("paper_2609_03613_amd")

TOL = 1e-4


def dev():
    return torch.device("cuda:0")


def dense(seed, n, grow):
    g, cam = scenes.small_forward(seed=seed, n=n)
    g["log_scales"] = (g["log_scales"] + grow).astype(np.float32)
    g["logits"] = (g["logits"] + grow).astype(np.float32)
    return g, cam


CASES = [  # (scene, split_entries)
    ("dense_stop", 256),      # most pixels reach the stop, inside later quarters
    ("dense_open", 256),      # long tiles, few stops
    ("training", 512),
]


def scene_of(name):
    if name == "dense_stop":
        return dense(2, 3000, 2.0)
    if name == "dense_open":
        return dense(3, 6000, 1.0)
    return scenes.training_scene(seed=5, n=40000, width=320, height=208)


@pytest.mark.parametrize("case", CASES)
def test_split_matches_oracle_and_unsplit(case):
    name, split = case
    g, cam = scene_of(name)
    W, H = int(cam["width"]), int(cam["height"])
    proj = oracle.project(g, cam)
    ref = oracle.render(proj, W, H)
    gd = tg.to_device(g, dev())
    rs = tg.Renderer(cam, tg.Params(split_entries=split, split_mean_factor=0), device=dev())
    r0 = tg.Renderer(cam, tg.Params(split_entries=0), device=dev())
    s, i = tg.project(gd, cam)
    bs = rs.bin(s, i, "binned")
    b0 = r0.bin(s, i, "binned")
    out = rs.rasterize(s, i, bs, counts=True, trans=True)
    out0 = r0.rasterize(s, i, b0, counts=True, trans=True)
    torch.cuda.synchronize()
    ns, thr = bs.split()
    offs = to_np(bs.offsets).view(np.uint32).astype(np.int64)
    tiles = rs.tiles
    counts = offs[64::64][:tiles] - offs[0:tiles * 64:64]
    assert thr == split and ns == int((counts >= split).sum()) > 0
    e_rgb, e_a, nflag = image_compare(to_np(out["rgb"]), to_np(out["alpha"]), ref)
    assert e_rgb <= TOL and e_a <= TOL, (e_rgb, e_a, nflag)
    m = ref["flags"] == 0
    assert m.mean() > 0.98
    assert np.array_equal(to_np(out["n_contrib"])[m], ref["ncontrib"][m])
    assert np.array_equal(to_np(out["n_support"])[m], ref["nsupport"][m])
    last = to_np(out["last"])
    ref_last = np.where(ref["last_pos"] >= 0, ref["last_pos"], -1)
    assert np.array_equal(last[m], ref_last[m])
    # against the unsplit raster: the same per-pixel chain, bit for bit
    for key in ("rgb", "alpha", "trans", "last", "n_contrib", "n_support"):
        assert torch.equal(out[key], out0[key]), key
    nv, nv0 = to_np(out["n_visit"]), to_np(out0["n_visit"])
    assert np.all(nv <= nv0) and np.all(nv >= to_np(out["n_support"]))
    if name == "dense_stop":
        # pixels that reach the stop, and quarters that visit fewer entries
        stop = (ref["alpha"] > 1 - 2e-4)
        assert stop.mean() > 0.05
        assert (nv < nv0).any()


def test_split_global_order_and_no_order():
    g, cam = dense(4, 5000, 1.5)
    gd = tg.to_device(g, dev())
    s, i = tg.project(gd, cam)
    imgs = {}
    for name, prm, order in [("binned", tg.Params(split_entries=256, split_mean_factor=0), "binned"),
                             ("global", tg.Params(split_entries=256, split_mean_factor=0), "global"),
                             ("no order", tg.Params(split_entries=256, split_mean_factor=0, tile_order=False), "binned"),
                             ("unsplit", tg.Params(split_entries=0), "binned")]:
        r = tg.Renderer(cam, prm, device=dev())
        out = r.rasterize(s, i, r.bin(s, i, order))
        torch.cuda.synchronize()
        imgs[name] = (to_np(out["rgb"]), to_np(out["last"]))
    # same split tiles in both orders; without a dispatch order nothing is split
    assert np.array_equal(imgs["binned"][0], imgs["global"][0])
    assert np.array_equal(imgs["no order"][0], imgs["unsplit"][0])
    assert np.array_equal(imgs["binned"][0], imgs["unsplit"][0])
    assert np.array_equal(imgs["binned"][1], imgs["unsplit"][1])


def test_split_overflow_writes_nan():
    g, cam = dense(5, 4000, 1.5)
    gd = tg.to_device(g, dev())
    r = tg.Renderer(cam, tg.Params(split_entries=256, split_mean_factor=0), device=dev())
    s, i = tg.project(gd, cam)
    full = r.bin(s, i, "binned", sync=True)
    M = full.num_entries
    small = tg.Binned("binned", M // 2, r.tiles, 64, 0, dev())
    r._binned[1] = small
    b = r.bin(s, i, "binned", sync=False)
    out = r.rasterize(s, i, b)
    torch.cuda.synchronize()
    assert int(b.counters[2].item()) == 1
    assert torch.isnan(out["rgb"]).all() and torch.isnan(out["alpha"]).all()


def test_split_cap_is_deterministic():
    # more than 1024 tiles reach split_entries: the threshold is raised by
    # powers of two until at most 1024 remain, a set that does not depend on
    # the order inside a count bucket, so repeated frames are bitwise equal
    g, cam = scenes.training_scene(seed=6, n=300000, width=1297, height=840)
    gd = tg.to_device(g, dev())
    r = tg.Renderer(cam, tg.Params(split_entries=256, split_mean_factor=0), device=dev())
    r0 = tg.Renderer(cam, tg.Params(split_entries=0), device=dev())
    s, i = tg.project(gd, cam)
    outs = []
    for _ in range(3):
        b = r.bin(s, i, "binned")
        outs.append({k: v.clone() for k, v in r.rasterize(s, i, b).items()})
        torch.cuda.synchronize()
        ns, thr = b.split()
        offs = to_np(b.offsets).view(np.uint32).astype(np.int64)
        counts = offs[64::64][:r.tiles] - offs[0:r.tiles * 64:64]
        assert int((counts >= 256).sum()) > 1024
        assert thr > 256 and thr & (thr - 1) == 0 and ns == int((counts >= thr).sum()) <= 1024
        assert int((counts >= thr // 2).sum()) > 1024
    for o in outs[1:]:
        assert torch.equal(o["rgb"], outs[0]["rgb"]) and torch.equal(o["last"], outs[0]["last"])
    u = r0.rasterize(s, i, r0.bin(s, i, "binned"))
    torch.cuda.synchronize()
    assert torch.equal(outs[0]["rgb"], u["rgb"]) and torch.equal(outs[0]["last"], u["last"])


def expected_split(counts, split, factor):
    """(tiles, threshold) by the documented rule: the smallest power of two
    >= split and >= factor x the mean of the non-empty tiles (the mean bound
    only when their 8x8 blocks fill the GPU, 8192 wavefronts) leaving at most
    1024 tiles; none when the mean bound applies and the longest tiles' bit
    length puts them below twice it."""
    nonempty = int((counts > 0).sum())
    filled = 4 * nonempty >= 8192
    rel = factor * int(counts.sum()) // nonempty if nonempty and filled else 0
    longest = 1 << (int(counts.max()).bit_length() - 1) if counts.max() > 0 else 0
    if rel and longest < 2 * rel:
        return 0, 0
    h = split.bit_length() - 1
    while h < 31 and (1 << h) < rel:
        h += 1
    while h <= 31:
        c = int((counts >= (1 << h)).sum())
        if c <= 1024:
            return c, 1 << h
        h += 1
    return 0, 0


def test_split_relative_bound():
    # the default factor (2 x the mean entries of the non-empty tiles, when
    # the longest tiles reach twice that): a uniformly dense scene that fills
    # the GPU has no long tail and splits nothing; the surface scene at
    # 1080p has one and splits the tiles past the bound; with too few tiles
    # to fill the GPU, the bound from the mean is skipped
    cases = [("training", scenes.training_scene(seed=7, n=300000, width=1297, height=840)),
             ("surfaces", scenes.scene_1080p(seed=0)),
             ("small", dense(2, 3000, 2.0))]
    for name, (g, cam) in cases:
        gd = tg.to_device(g, dev())
        r = tg.Renderer(cam, tg.Params(split_entries=256), device=dev())
        r0 = tg.Renderer(cam, tg.Params(split_entries=0), device=dev())
        s, i = tg.project(gd, cam)
        b = r.bin(s, i, "binned")
        out = r.rasterize(s, i, b)
        u = r0.rasterize(s, i, r0.bin(s, i, "binned"))
        torch.cuda.synchronize()
        ns, thr = b.split()
        offs = to_np(b.offsets).view(np.uint32).astype(np.int64)
        counts = offs[64::64][:r.tiles] - offs[0:r.tiles * 64:64]
        assert (ns, thr) == expected_split(counts, 256, 2), name
        nonempty = int((counts > 0).sum())
        mean = counts.sum() / max(nonempty, 1)
        if name == "training":
            assert 4 * nonempty >= 8192 and ns == 0 and thr == 0
        elif name == "surfaces":
            assert 4 * nonempty >= 8192 and ns > 0 and thr >= 2 * mean
        else:
            assert 4 * nonempty < 8192 and thr == 256 and ns > 0
        assert torch.equal(out["rgb"], u["rgb"]) and torch.equal(out["last"], u["last"])


@pytest.mark.parametrize("W,H", [(203, 77), (134, 42), (18, 9)])
def test_split_ragged_image(W, H):
    # image sizes that cut tiles, 8x8 blocks and 4x4 quarters (quarters
    # partly or wholly outside the image, whose lanes composite nothing and
    # write nothing): the quad walk on every non-empty tile equals the
    # unsplit raster bit for bit (the visit count bounded by it: the quarter
    # cull visits fewer entries), and the oracle within 1e-4
    g, _ = dense(11, 2500, 1.5)
    cam = scenes.camera(np.eye(3), np.zeros(3), 0.5 * W, 0.5 * W, W / 2.0, H / 2.0, W, H)
    proj = oracle.project(g, cam)
    ref = oracle.render(proj, W, H)
    gd = tg.to_device(g, dev())
    rs = tg.Renderer(cam, tg.Params(split_entries=256, split_mean_factor=0), device=dev())
    r0 = tg.Renderer(cam, tg.Params(split_entries=0), device=dev())
    s, i = tg.project(gd, cam)
    bs = rs.bin(s, i, "binned")
    out = rs.rasterize(s, i, bs, counts=True, trans=True)
    out0 = r0.rasterize(s, i, r0.bin(s, i, "binned"), counts=True, trans=True)
    torch.cuda.synchronize()
    ns, thr = bs.split()
    offs = to_np(bs.offsets).view(np.uint32).astype(np.int64)
    counts = offs[64::64][:rs.tiles] - offs[0:rs.tiles * 64:64]
    assert ns == int((counts >= 256).sum()) > 0 and thr == 256
    for key in ("rgb", "alpha", "trans", "last", "n_contrib", "n_support"):
        assert torch.equal(out[key], out0[key]), key
    nv, nv0 = to_np(out["n_visit"]), to_np(out0["n_visit"])
    assert np.all(nv <= nv0) and np.all(nv >= to_np(out["n_support"]))
    e_rgb, e_a, nflag = image_compare(to_np(out["rgb"]), to_np(out["alpha"]), ref)
    assert e_rgb <= TOL and e_a <= TOL, (e_rgb, e_a, nflag)
