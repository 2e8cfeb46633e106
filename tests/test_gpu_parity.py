"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars: integer and index results (entry keys, global order, tile ranges, depth
range, bin offsets, the repaired stream) bit-exact; images within 1e-4 per
channel of the FP64 oracle on every pixel the oracle did not flag as
threshold-ambiguous; the binned and globally sorted paths, and every raster
variant, bitwise identical to each other.
"""
import numpy as np
import pytest
import torch

import oracle
import scenes
from helpers import decode_info, image_compare, to_np

pytestmark = pytest.mark.gpu

tg = pytest.importorskip("paper_2609_03613_amd")

TOL = 1e-4


def dev():
    return torch.device("cuda:0")


def run_bin(splats_np, info_np, cam, order, params=None, capacity=None):
    r = tg.Renderer(cam, params or tg.Params(), device=dev())
    s = torch.as_tensor(splats_np).to(dev())
    i = torch.as_tensor(np.ascontiguousarray(info_np).view(np.int32)).to(dev())
    b = r.bin(s, i, order, capacity=capacity)
    torch.cuda.synchronize()
    return r, s, i, b


def cam_for(W, H, f=100.0):
    return scenes.camera(np.eye(3), np.zeros(3), f, f, W / 2, H / 2, W, H)


# ---------------------------------------------------------------------------
# projection
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["small", "training_d3", "surface_d3", "guard"])
def test_project_matches_oracle(case):
    if case == "guard":
        # large Gaussians up to 2.2x the half FOV off axis: many take the
        # frustum guard and still reach the image
        g, cam = scenes.guard_scene(seed=0)
    elif case == "small":
        g, cam = scenes.small_forward(seed=0)
    elif case == "training_d3":
        g, cam = scenes.training_scene(seed=0, n=20000)
    else:
        g, cam = scenes.scene_1080p(seed=0, n=50000)
    ref = oracle.project(g, cam)
    splats, info = tg.project(tg.to_device(g, dev()), cam)
    torch.cuda.synchronize()
    s = to_np(splats).astype(np.float64)
    depth, rect = decode_info(to_np(info))
    vis_ref = (ref["flags"] & oracle.VISIBLE) > 0
    vis = (rect[:, 2] > rect[:, 0]) & (rect[:, 3] > rect[:, 1])
    amb = (ref["flags"] & (oracle.AMBIG_RECT | oracle.AMBIG_VIS)) > 0
    assert np.array_equal(vis[~amb], vis_ref[~amb])
    v = vis & vis_ref
    assert v.sum() > (0.25 if case == "guard" else 0.5) * len(v)
    # depth key: bit-exact (same IEEE binary64 operations, one rounding)
    assert np.array_equal(depth[v].view(np.uint32), ref["depth_key"][v].view(np.uint32))
    ok = v & ~amb
    assert np.array_equal(rect[ok], ref["rect"][ok].astype(np.int64))
    mean = s[:, 0:2] + s[:, 2:4]
    np.testing.assert_allclose(mean[v], ref["mean2d"][v], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(s[v, 4:7], ref["conic"][v], rtol=2e-7, atol=1e-12 * np.abs(ref["conic"][v]).max())
    np.testing.assert_allclose(s[v, 7], ref["opacity"][v], rtol=2e-7)
    np.testing.assert_allclose(s[v, 8:11], ref["rgb"][v], rtol=2e-7, atol=1e-7)
    # largest axis scale (word 11, the near-depth key's s_max): one rounding
    # of a binary64 exp on both sides
    np.testing.assert_allclose(s[v, 11], ref["smax"][v], rtol=1.2e-7, atol=0)


# ---------------------------------------------------------------------------
# ordering: bit-exact against the oracle's integer schedule
# ---------------------------------------------------------------------------

SCHED_CASES = [
    # (n, W, H, K, seed, tie_fraction, hidden_fraction, max_sigma)
    (3000, 128, 96, 64, 0, 0.0, 0.0, 12.0),
    (5000, 200, 120, 8, 1, 0.2, 0.1, 20.0),   # ragged image, ties, hidden splats
    (20000, 512, 384, 64, 2, 0.05, 0.05, 8.0),  # V > S: sampled depth range
    (4000, 64, 64, 1, 3, 0.1, 0.0, 40.0),     # K = 1: segments are whole tiles
    (1, 16, 16, 64, 4, 0.0, 0.0, 2.0),        # one splat
]


@pytest.mark.parametrize("case", SCHED_CASES)
def test_schedule_bit_exact(case):
    n, W, H, K, seed, ties, hidden, sig = case
    splats, info = scenes.random_splats(n, W, H, seed=seed, tie_fraction=ties, hidden_fraction=hidden,
                                        max_sigma_px=sig)
    cam = cam_for(W, H)
    depth, rect = scenes.info_depth(info), scenes.info_rects(info)
    tx, ty = (W + 15) // 16, (H + 15) // 16
    ref = oracle.schedule(depth, rect, tx, ty, K=K, znear=cam["znear"], zfar=cam["zfar"])
    p = tg.Params(num_bins=K)
    _, _, _, bg = run_bin(splats, info, cam, "global", p)
    assert bg.num_entries == ref["M"]
    M = ref["M"]
    assert np.array_equal(to_np(bg.keys)[:M].view(np.uint64), ref["keys"])
    assert np.array_equal(to_np(bg.vals)[:M].view(np.uint32), ref["vals"])
    assert np.array_equal(to_np(bg.offsets).view(np.uint32), ref["tile_offsets"])
    _, _, _, bb = run_bin(splats, info, cam, "binned", p)
    assert bb.num_entries == M
    assert np.array_equal(to_np(bb.zrange).view(np.uint32), ref["zrange"].view(np.uint32))
    assert np.array_equal(to_np(bb.offsets).view(np.uint32), ref["bin_offsets"])
    assert np.array_equal(to_np(bb.pairs)[:M].view(np.uint64), ref["stream"])
    c = to_np(bb.counters)
    assert c[0] == M and c[2] == 0


def test_tail_segments_bit_exact():
    # one 16x16 tile covered by 20k splats with K = 1: a single segment of
    # more than 8192 entries goes through the global-memory tail sort, and a
    # second tile gets a 2049..8192 segment
    n = 26000
    rng = np.random.default_rng(9)
    splats, info = scenes.random_splats(n, 32, 16, seed=9, tie_fraction=0.3, max_sigma_px=1.0)
    rect = np.zeros((n, 4), np.int64)
    rect[:, 2] = 1
    rect[:, 3] = 1
    rect[20000:, 0] = 1
    rect[20000:, 2] = 2
    info = scenes.make_info(scenes.info_depth(info), rect)
    cam = cam_for(32, 16)
    ref = oracle.schedule(scenes.info_depth(info), rect, 2, 1, K=1)
    # packed = 2 (block masks) keeps whole segments in the repair queues (no
    # sub-bins), so the > 8192 segment reaches the global-memory tail sort;
    # the default splits it into sub-segments first
    for p in (tg.Params(num_bins=1, packed=2), tg.Params(num_bins=1)):
        _, _, _, bb = run_bin(splats, info, cam, "binned", p)
        assert np.array_equal(to_np(bb.pairs)[:n].view(np.uint64), ref["stream"])
        assert np.array_equal(to_np(bb.offsets).view(np.uint32), ref["bin_offsets"])
    del rng


# The staged group sort (exact repair, sub-bins): 8 tiles in one row make
# one group of 8 x 64 segments. A group of at most 4096 entries is staged in
# LDS, where sub-segments of 2..128 entries are put in order; longer ones
# (depth clusters: one shared depth on one tile) are staged and then queued
# for the repair sorts; a larger group takes the unstaged path (up to 70,000
# entries here, several sweeps of the group sort's 8192-entry batches).
STAGE_CASES = [
    # (n, widest rect in tiles, tie fraction, cluster sizes)
    (1200, 3, 0.2, ()),
    (1500, 2, 0.0, (700,)),
    (3000, 1, 0.1, (2100, 300, 129, 128)),
    (4096, 1, 0.0, (64,)),
    (12000, 8, 0.3, (3000, 1000, 200)),
    (16384, 1, 0.0, ()),
    (16385, 1, 0.1, (5000,)),
    (40000, 2, 0.2, (20000, 3000, 129)),
    (70000, 1, 0.1, ()),
]


@pytest.mark.parametrize("case", STAGE_CASES)
def test_staged_group_sort(case):
    n, widest, ties, clusters = case
    W, H = 128, 16
    splats, info = scenes.random_splats(n, W, H, seed=n, tie_fraction=ties, max_sigma_px=2.0)
    rng = np.random.default_rng(n)
    rect = np.zeros((n, 4), np.int64)
    x0 = rng.integers(0, 8, n)
    rect[:, 0] = x0
    rect[:, 2] = np.minimum(x0 + rng.integers(1, widest + 1, n), 8)
    rect[:, 3] = 1
    depth = scenes.info_depth(info).copy()
    at = 0
    for k, size in enumerate(clusters):
        # one shared depth per cluster, all on tile k: one sub-segment of that size
        depth[at:at + size] = depth[at]
        rect[at:at + size, 0] = k
        rect[at:at + size, 2] = k + 1
        at += size
    info = scenes.make_info(depth, rect)
    cam = cam_for(W, H)
    ref = oracle.schedule(depth, rect, 8, 1, K=64, znear=cam["znear"], zfar=cam["zfar"])
    M = ref["M"]
    _, _, _, bb = run_bin(splats, info, cam, "binned", tg.Params(num_bins=64))
    assert bb.num_entries == M
    assert np.array_equal(to_np(bb.offsets).view(np.uint32), ref["bin_offsets"])
    assert np.array_equal(to_np(bb.pairs)[:M].view(np.uint64), ref["stream"])
    c = to_np(bb.counters)
    assert c[2] == 0
    # the path this case is meant to take, and its sub-segments (the bins at
    # 8 K): each cluster is one sub-segment of at least its size
    assert (M <= 4096) == (n <= 4096)
    sub = np.diff(oracle.schedule(depth, rect, 8, 1, K=512, znear=cam["znear"], zfar=cam["zfar"])["bin_offsets"]
                  .astype(np.int64))
    for size in clusters:
        assert (sub >= size).sum() >= sum(1 for s2 in clusters if s2 >= size)


@pytest.mark.parametrize("sub_bins", [1, 2, 4, 8])
@pytest.mark.parametrize("case", [STAGE_CASES[2], STAGE_CASES[7], STAGE_CASES[8]])
def test_sub_bin_counts_bit_exact(case, sub_bins):
    # any number of sub-bins gives the same stream (the sub-bins only split
    # the work between the group sort and the repair): staged and unstaged
    # groups, whole segments queued at one sub-bin
    n, widest, ties, clusters = case
    W, H = 128, 16
    splats, info = scenes.random_splats(n, W, H, seed=n + sub_bins, tie_fraction=ties, max_sigma_px=2.0)
    rng = np.random.default_rng(n + sub_bins)
    rect = np.zeros((n, 4), np.int64)
    x0 = rng.integers(0, 8, n)
    rect[:, 0] = x0
    rect[:, 2] = np.minimum(x0 + rng.integers(1, widest + 1, n), 8)
    rect[:, 3] = 1
    depth = scenes.info_depth(info).copy()
    at = 0
    for k, size in enumerate(clusters):
        depth[at:at + size] = depth[at]
        rect[at:at + size, 0] = k
        rect[at:at + size, 2] = k + 1
        at += size
    info = scenes.make_info(depth, rect)
    cam = cam_for(W, H)
    ref = oracle.schedule(depth, rect, 8, 1, K=64, znear=cam["znear"], zfar=cam["zfar"])
    M = ref["M"]
    _, _, _, bb = run_bin(splats, info, cam, "binned", tg.Params(num_bins=64, sub_bins=sub_bins))
    assert bb.num_entries == M and to_np(bb.counters)[2] == 0
    assert np.array_equal(to_np(bb.offsets).view(np.uint32), ref["bin_offsets"])
    assert np.array_equal(to_np(bb.pairs)[:M].view(np.uint64), ref["stream"])


@pytest.mark.parametrize("per_tile", [False, True])
def test_per_entry_atomic_path_bit_exact(per_tile):
    # 8-pixel tiles at 2560x1440 (57,600 tiles) with K = 1024: a group of
    # tiles would exceed the group sort's 4096 counters, so binning takes the
    # per-entry atomic count / offsets / scatter path instead
    n, W, H, ts, kmax = 3000, 2560, 1440, 8, 1024
    splats, info = scenes.random_splats(n, W, H, tile_size=ts, seed=41, tie_fraction=0.1, hidden_fraction=0.05,
                                        max_sigma_px=6.0)
    cam = cam_for(W, H, f=1000.0)
    tx, ty = W // ts, H // ts
    depth, rect = scenes.info_depth(info), scenes.info_rects(info)
    s = torch.as_tensor(splats).to(dev())
    i = torch.as_tensor(info.view(np.int32)).to(dev())
    if per_tile:
        kt = np.random.default_rng(5).choice([1, 2, 64, 256, 1024], size=tx * ty).astype(np.int32)
        ref = oracle.schedule_tiles(depth, rect, tx, ty, kt, znear=cam["znear"], zfar=cam["zfar"])
        p = tg.Params(tile_size=ts, num_bins=kmax, per_tile_bins=torch.as_tensor(kt).to(dev()))
    else:
        ref = oracle.schedule(depth, rect, tx, ty, K=kmax, znear=cam["znear"], zfar=cam["zfar"])
        p = tg.Params(tile_size=ts, num_bins=kmax)
    r = tg.Renderer(cam, p, device=dev())
    b = r.bin(s, i, "binned")
    torch.cuda.synchronize()
    M = ref["M"]
    S = len(ref["bin_offsets"]) - 1
    assert b.num_entries == M
    assert np.array_equal(to_np(b.offsets).view(np.uint32)[:S + 1], ref["bin_offsets"])
    assert np.array_equal(to_np(b.pairs)[:M].view(np.uint64), ref["stream"])


def test_empty_and_invisible():
    cam = cam_for(40, 24)
    for n in (0, 5):
        splats, info = scenes.random_splats(n, 40, 24, seed=1, hidden_fraction=1.0)
        for order in ("global", "binned"):
            r, s, i, b = run_bin(splats, info, cam, order)
            assert b.num_entries == 0
            out = r.rasterize(s, i, b, bg=(0.25, 0.5, 0.75))
            torch.cuda.synchronize()
            assert np.all(to_np(out["rgb"]) == np.array([0.25, 0.5, 0.75], np.float32))
            assert np.all(to_np(out["alpha"]) == 0) and np.all(to_np(out["last"]) == -1)


# ---------------------------------------------------------------------------
# raster: images against the FP64 oracle; all variants bitwise equal
# ---------------------------------------------------------------------------

VARIANTS = [("global", "plain", 0), ("global", "wave", 0), ("binned", "plain", 0), ("binned", "wave", 0),
            ("binned", "plain", 1), ("binned", "wave", 1), ("binned", "plain", 2), ("binned", "wave", 2)]


def render_variant(g_splats, g_info, cam, order, raster, packed, K=64, bg=(0.0, 0.0, 0.0)):
    p = tg.Params(num_bins=K, raster=raster, packed=packed)
    r = tg.Renderer(cam, p, device=dev())
    b = r.bin(g_splats, g_info, order)
    out = r.rasterize(g_splats, g_info, b, bg=bg, counts=True)
    torch.cuda.synchronize()
    return {k: to_np(v) for k, v in out.items()}, b


@pytest.mark.parametrize("seed,W,H", [(0, 128, 96), (1, 203, 77), (2, 16, 16), (3, 1, 1)])
def test_raster_synthetic_splats(seed, W, H):
    n = max(1, (W * H) // 8)
    splats, info = scenes.random_splats(n, W, H, seed=seed, tie_fraction=0.05, hidden_fraction=0.05)
    cam = cam_for(W, H)
    ref = oracle.render(oracle.splats_to_proj(splats, info), W, H, bg=(0.1, 0.2, 0.3))
    s = torch.as_tensor(splats).to(dev())
    i = torch.as_tensor(info.view(np.int32)).to(dev())
    outs = {}
    for order, raster, packed in VARIANTS:
        out, b = render_variant(s, i, cam, order, raster, packed, bg=(0.1, 0.2, 0.3))
        outs[(order, raster, packed)] = out
        e_rgb, e_a, nflag = image_compare(out["rgb"], out["alpha"], ref)
        assert e_rgb <= TOL and e_a <= TOL, (order, raster, packed, e_rgb, e_a, nflag)
        mask = ref["flags"] == 0
        assert np.array_equal(out["n_contrib"][mask], ref["ncontrib"][mask])
        # last: the stream position of the oracle's list (same global order)
        assert np.array_equal(out["last"][mask], ref["last_pos"][mask])
        assert np.array_equal(out["n_support"][mask], ref["nsupport"][mask])
        if raster == "plain":
            assert np.array_equal(out["n_visit"][mask], ref["nvisit"][mask])
        else:
            assert np.all(out["n_visit"][mask] <= ref["nvisit"][mask])
            assert np.all(out["n_visit"][mask] >= ref["nsupport"][mask])
    base = outs[VARIANTS[0]]
    for k, out in outs.items():
        for key in ("rgb", "alpha", "last", "n_contrib"):
            assert np.array_equal(out[key], base[key]), (k, key)


@pytest.mark.parametrize("seed", [0, 1])
def test_end_to_end_small_forward(seed):
    g, cam = scenes.small_forward(seed=seed)
    ref = oracle.render(oracle.project(g, cam), 128, 128)
    gd = tg.to_device(g, dev())
    imgs = {}
    for order in ("global", "binned"):
        out = tg.render(gd, cam, order=order, counts=True)
        torch.cuda.synchronize()
        e_rgb, e_a, nflag = image_compare(to_np(out["rgb"]), to_np(out["alpha"]), ref)
        assert e_rgb <= TOL and e_a <= TOL, (order, e_rgb, e_a)
        assert nflag <= 20
        mask = ref["flags"] == 0
        assert np.array_equal(to_np(out["n_contrib"])[mask], ref["ncontrib"][mask])
        imgs[order] = to_np(out["rgb"])
    assert np.array_equal(imgs["global"], imgs["binned"])


def test_end_to_end_large_splats_terminate():
    # larger, denser splats so that pixels reach the transmittance stop
    g, cam = scenes.small_forward(seed=2, n=3000)
    g["log_scales"] = (g["log_scales"] + 2.0).astype(np.float32)
    g["logits"] = (g["logits"] + 2.0).astype(np.float32)
    ref = oracle.render(oracle.project(g, cam), 128, 128)
    assert (ref["alpha"] > 1 - 2e-4).mean() > 0.05
    out = tg.render(tg.to_device(g, dev()), cam, order="binned", counts=True)
    torch.cuda.synchronize()
    e_rgb, e_a, nflag = image_compare(to_np(out["rgb"]), to_np(out["alpha"]), ref)
    assert e_rgb <= TOL and e_a <= TOL, (e_rgb, e_a, nflag)


def test_determinism():
    g, cam = scenes.training_scene(seed=3, n=30000, width=300, height=200)
    gd = tg.to_device(g, dev())
    r = tg.Renderer(cam, device=dev())
    a = r.render(gd, "binned")
    pa = to_np(a["binned"].pairs).copy()
    ia = to_np(a["rgb"]).copy()
    b = r.render(gd, "binned")
    assert np.array_equal(pa, to_np(b["binned"].pairs))
    assert np.array_equal(ia, to_np(b["rgb"]))


def test_capacity_overflow():
    splats, info = scenes.random_splats(2000, 128, 128, seed=5)
    cam = cam_for(128, 128)
    M = oracle.count_entries(scenes.info_rects(info))
    p = tg.Params()
    r = tg.Renderer(cam, p, device=dev())
    s = torch.as_tensor(splats).to(dev())
    i = torch.as_tensor(info.view(np.int32)).to(dev())
    # without synchronisation: counters[2] is raised and the raster writes NaN
    b = tg.Binned("binned", M // 2, r.tiles, p.num_bins, p.packed, dev())
    r._binned[1] = b
    b2 = r.bin(s, i, "binned", sync=False)
    out = r.rasterize(s, i, b2)
    torch.cuda.synchronize()
    c = to_np(b2.counters)
    assert c[0] == M and c[2] == 1
    assert np.all(np.isnan(to_np(out["rgb"])))
    # with synchronisation the wrapper grows the buffers and succeeds
    b3 = r.bin(s, i, "binned", sync=True)
    assert b3.num_entries == M and b3.capacity >= M


def test_invalid_arguments_raise():
    cam = cam_for(32, 32)
    splats, info = scenes.random_splats(10, 32, 32, seed=0)
    with pytest.raises(tg.TileGSError):
        tg.Renderer(cam, tg.Params(tile_size=12), device=dev()).bin(
            torch.as_tensor(splats).to(dev()), torch.as_tensor(info.view(np.int32)).to(dev()))


BUCKET_EDGES = [2, 3, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1024, 1025, 2048, 2049, 4096, 4097,
                8192, 8193]


def test_repair_bucket_edges_and_records():
    # one tile per segment length at every bucket boundary of the repair
    # sorts (K = 1, so a segment is a whole tile); random depths with ties
    lens = BUCKET_EDGES
    W = 16 * len(lens)
    n = sum(lens)
    splats, info = scenes.random_splats(n, W, 16, seed=11, tie_fraction=0.3, max_sigma_px=1.0)
    rect = np.zeros((n, 4), np.int64)
    tile = np.repeat(np.arange(len(lens)), lens)
    rng = np.random.default_rng(1)
    perm = rng.permutation(n)  # interleave the tiles in id order
    rect[perm, 0] = tile
    rect[perm, 2] = tile + 1
    rect[:, 3] = 1
    info = scenes.make_info(scenes.info_depth(info), rect)
    cam = cam_for(W, 16)
    for K in (1, 4):
        ref = oracle.schedule(scenes.info_depth(info), rect, len(lens), 1, K=K)
        _, _, _, bb = run_bin(splats, info, cam, "binned", tg.Params(num_bins=K, packed=1))
        pairs = to_np(bb.pairs)[:n].view(np.uint64)
        assert np.array_equal(pairs, ref["stream"]), K
        assert np.array_equal(to_np(bb.offsets).view(np.uint32), ref["bin_offsets"])
        # packed records: the entry's splat staged for its tile
        rec = to_np(bb.records)[:n]
        gid = (pairs & np.uint64(0xFFFFFFFF)).astype(np.int64)
        t_of = np.repeat(np.arange(len(lens)), np.diff(ref["bin_offsets"][::K].astype(np.int64)))
        ox = (t_of * 16).astype(np.float32)
        sp = splats[gid]
        k = np.float32(-0.72134752044448170)
        assert np.array_equal(rec[:, 0], (sp[:, 0] - ox) + sp[:, 2])
        assert np.array_equal(rec[:, 1], (sp[:, 1] - np.float32(0.0)) + sp[:, 3])
        assert np.array_equal(rec[:, 2], k * sp[:, 4])
        assert np.array_equal(rec[:, 3], np.float32(2.0 * k) * sp[:, 5])
        assert np.array_equal(rec[:, 4], k * sp[:, 6])
        assert np.array_equal(rec[:, 5:9], sp[:, 7:11])
        assert np.array_equal(rec[:, 9].view(np.uint32), gid.astype(np.uint32))
        check_block_masks(to_np(bb.masks)[:n], sp, t_of, W, 16)


def check_block_masks(masks, sp, tiles, W, H, tiles_x=None):
    """Bit w of an entry's mask must be set whenever some pixel of 8x8 block w
    of its tile reaches alpha >= 1/255 (safety of the cull, float64), and is
    clear for blocks outside the image."""
    tiles_x = tiles_x or (W + 15) // 16
    ly, lx = np.mgrid[0:16, 0:16]
    for i in range(len(masks)):
        t = int(tiles[i])
        tx, ty = t % tiles_x, t // tiles_x
        mx = float(sp[i, 0]) + float(sp[i, 2]) - 16 * tx
        my = float(sp[i, 1]) + float(sp[i, 3]) - 16 * ty
        a, b, c, o = (float(v) for v in sp[i, 4:8])
        dx, dy = mx - (lx + 0.5), my - (ly + 0.5)
        q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
        inimg = (16 * tx + lx < W) & (16 * ty + ly < H)
        tau = 2 * np.log(255 * o)
        for w in range(4):
            blk = (lx // 8 == (w & 1)) & (ly // 8 == (w >> 1)) & inimg
            bit = (int(masks[i]) >> w) & 1
            if blk.any() and (q[blk] <= tau).any():
                assert bit == 1, (i, w)
            if not blk.any():
                assert bit == 0, (i, w)


@pytest.mark.parametrize("ts", [8, 32])
def test_tile_sizes(ts):
    # 8- and 32-pixel tiles (WAVE raster, gather by id): projection rects in
    # those tile units, the schedule bit-exact against the oracle on the same
    # tile grid, both orders bitwise equal, and images within rounding of the
    # 16-pixel path (the per-pixel sequence of composited entries does not
    # depend on the tile size; the tile-relative mean's rounding does)
    g, cam = scenes.small_forward(seed=1, n=3000)
    W, H = cam["width"], cam["height"]
    ref_p = oracle.project(g, cam, tile_size=ts)
    gd = tg.to_device(g, dev())
    p = tg.Params(tile_size=ts, num_bins=32)
    splats, info = tg.project(gd, cam, p)
    torch.cuda.synchronize()
    depth, rect = decode_info(to_np(info))
    vis_ref = (ref_p["flags"] & oracle.VISIBLE) > 0
    amb = (ref_p["flags"] & (oracle.AMBIG_RECT | oracle.AMBIG_VIS)) > 0
    ok = vis_ref & ~amb
    assert np.array_equal(rect[ok], ref_p["rect"][ok].astype(np.int64))
    tx, ty = (W + ts - 1) // ts, (H + ts - 1) // ts
    ref_s = oracle.schedule(depth, rect, tx, ty, K=32, znear=cam["znear"], zfar=cam["zfar"])
    r = tg.Renderer(cam, p, device=dev())
    outs = {}
    for order in ("global", "binned"):
        b = r.bin(splats, info, order)
        M = ref_s["M"]
        assert b.num_entries == M
        if order == "binned":
            assert np.array_equal(to_np(b.offsets).view(np.uint32), ref_s["bin_offsets"])
            assert np.array_equal(to_np(b.pairs)[:M].view(np.uint64), ref_s["stream"])
        else:
            assert np.array_equal(to_np(b.offsets).view(np.uint32), ref_s["tile_offsets"])
        out = r.rasterize(splats, info, b, counts=True)
        torch.cuda.synchronize()
        outs[order] = {k: to_np(v) for k, v in out.items()}
    ref = oracle.render(oracle.project(g, cam), W, H)
    e_rgb, e_a, _ = image_compare(outs["binned"]["rgb"], outs["binned"]["alpha"], ref)
    assert e_rgb <= TOL and e_a <= TOL
    base = tg.render(gd, cam, order="binned")
    torch.cuda.synchronize()
    for key in ("rgb", "alpha", "last", "n_contrib"):
        assert np.array_equal(outs["global"][key], outs["binned"][key]), key
    assert np.abs(outs["binned"]["rgb"] - to_np(base["rgb"])).max() <= 1e-5


@pytest.mark.parametrize("W,H,ts", [(16384, 24, 8), (24, 16384, 16), (16384, 40, 32)])
def test_maximum_image_extent(W, H, ts):
    # the largest accepted width or height (16384 px): 2048 tile columns of
    # 8 px, 1024 tile rows of 16 px, 512 columns of 32 px, with a ragged
    # last tile row or column. Schedule bit-exact against the oracle on the
    # same tile grid; the product image (binned, wave raster, tile order and
    # split), the globally sorted stream through the same raster and, with
    # 16-pixel tiles, the comparator (one workgroup per tile) within 1e-4 of
    # the oracle and bitwise equal to each other
    n = 6000
    splats, info = scenes.random_splats(n, W, H, tile_size=ts, seed=W + H + ts, tie_fraction=0.05,
                                        hidden_fraction=0.05, max_sigma_px=6.0)
    cam = cam_for(W, H)
    depth, rect = decode_info(info.view(np.int32))
    tx, ty = (W + ts - 1) // ts, (H + ts - 1) // ts
    ref_s = oracle.schedule(depth, rect, tx, ty, K=32, znear=cam["znear"], zfar=cam["zfar"])
    ref = oracle.render(oracle.splats_to_proj(splats, info), W, H, tile_size=ts, bg=(0.1, 0.2, 0.3))
    s = torch.as_tensor(splats).to(dev())
    i = torch.as_tensor(info.view(np.int32)).to(dev())
    outs = {}
    legs = [("binned", "wave"), ("global", "wave")] + ([("global", "plain")] if ts == 16 else [])
    for order, raster in legs:
        r = tg.Renderer(cam, tg.Params(tile_size=ts, num_bins=32, raster=raster), device=dev())
        b = r.bin(s, i, order)
        M = ref_s["M"]
        assert b.num_entries == M
        if order == "binned":
            assert np.array_equal(to_np(b.offsets).view(np.uint32), ref_s["bin_offsets"])
            assert np.array_equal(to_np(b.pairs)[:M].view(np.uint64), ref_s["stream"])
        else:
            assert np.array_equal(to_np(b.offsets).view(np.uint32), ref_s["tile_offsets"])
        out = r.rasterize(s, i, b, bg=(0.1, 0.2, 0.3), counts=True)
        torch.cuda.synchronize()
        o = outs[(order, raster)] = {k: to_np(v) for k, v in out.items()}
        e_rgb, e_a, nflag = image_compare(o["rgb"], o["alpha"], ref)
        assert e_rgb <= TOL and e_a <= TOL, (order, raster, e_rgb, e_a, nflag)
        mask = ref["flags"] == 0
        assert np.array_equal(o["n_contrib"][mask], ref["ncontrib"][mask])
        assert np.array_equal(o["n_support"][mask], ref["nsupport"][mask])
    for leg, o in outs.items():
        for key in ("rgb", "alpha", "last", "n_contrib"):
            assert np.array_equal(o[key], outs[legs[0]][key]), (leg, key)


def test_images_identical_across_bin_counts():
    # the paper reports image quality independent of the bin count (depth
    # bin count ablation); with exact repair every K gives the same stream
    # as the global sort, so the images are bitwise identical for every K
    # (1 .. 1024; K = 1024 takes one-tile groups without sub-bins) and to
    # the globally sorted frame, in the product raster
    g, cam = scenes.scene_1080p(seed=4, n=200_000)
    gd = tg.to_device(g, dev())
    splats, info = tg.project(gd, cam)
    torch.cuda.synchronize()
    ref = tg.Renderer(cam, tg.Params(), device=dev())
    bg = ref.bin(splats, info, "global")
    base = {k: to_np(v) for k, v in ref.rasterize(splats, info, bg, counts=True).items()}
    M = bg.num_entries
    assert M > 100_000
    for K in (1, 2, 8, 64, 256, 1024):
        r = tg.Renderer(cam, tg.Params(num_bins=K), device=dev())
        b = r.bin(splats, info, "binned")
        assert b.num_entries == M
        out = r.rasterize(splats, info, b, counts=True)
        torch.cuda.synchronize()
        for key in ("rgb", "alpha", "last", "n_contrib", "n_support"):
            assert np.array_equal(to_np(out[key]), base[key]), (K, key)


def effective_bins(kt, kmax):
    """Per-tile bin counts as the library applies them: clamped to
    1..kmax and rounded down to a power of two."""
    k = np.clip(np.asarray(kt, np.int64), 1, kmax)
    return (2 ** np.floor(np.log2(k))).astype(np.int32)


@pytest.mark.parametrize("ts", [16, 8])
def test_per_tile_bins_bit_exact(ts):
    # variable bin counts per tile (segments numbered by a prefix sum):
    # seg_base, bin offsets and the repaired stream bit-exact against the
    # oracle, images bitwise equal to the uniform-K path, backward unchanged
    n, W, H = 6000, 203, 130
    splats, info = scenes.random_splats(n, W, H, tile_size=ts, seed=31, tie_fraction=0.1, hidden_fraction=0.05)
    cam = cam_for(W, H)
    tx, ty = (W + ts - 1) // ts, (H + ts - 1) // ts
    T = tx * ty
    rng = np.random.default_rng(ts)
    kt = rng.choice([0, 1, 2, 3, 5, 16, 64, 100, 256, 1000], size=T).astype(np.int32)
    kmax = 256
    keff = effective_bins(kt, kmax)
    depth, rect = scenes.info_depth(info), scenes.info_rects(info)
    ref = oracle.schedule_tiles(depth, rect, tx, ty, keff, znear=cam["znear"], zfar=cam["zfar"])
    s = torch.as_tensor(splats).to(dev())
    i = torch.as_tensor(info.view(np.int32)).to(dev())
    p = tg.Params(tile_size=ts, num_bins=kmax, per_tile_bins=torch.as_tensor(kt).to(dev()))
    r = tg.Renderer(cam, p, device=dev())
    b = r.bin(s, i, "binned")
    torch.cuda.synchronize()
    M = ref["M"]
    S = int(ref["seg_base"][-1])
    assert b.num_entries == M
    assert np.array_equal(to_np(b.seg_base).view(np.uint32), ref["seg_base"])
    assert np.array_equal(to_np(b.offsets).view(np.uint32)[:S + 1], ref["bin_offsets"])
    assert np.array_equal(to_np(b.pairs)[:M].view(np.uint64), ref["stream"])
    out = r.rasterize(s, i, b, bg=(0.2, 0.1, 0.0), counts=True)
    r_u = tg.Renderer(cam, tg.Params(tile_size=ts, num_bins=32), device=dev())
    b_u = r_u.bin(s, i, "binned")
    out_u = r_u.rasterize(s, i, b_u, bg=(0.2, 0.1, 0.0), counts=True)
    torch.cuda.synchronize()
    for k in ("rgb", "alpha", "last", "n_contrib"):
        assert torch.equal(out[k], out_u[k]), k
    # a second call with other counts reuses the buffers
    kt2 = np.full(T, 4, np.int32)
    r.set_per_tile_bins(torch.as_tensor(kt2).to(dev()))
    b2 = r.bin(s, i, "binned")
    ref2 = oracle.schedule_tiles(depth, rect, tx, ty, kt2, znear=cam["znear"], zfar=cam["zfar"])
    torch.cuda.synchronize()
    assert np.array_equal(to_np(b2.offsets).view(np.uint32)[:4 * T + 1], ref2["bin_offsets"])
    assert np.array_equal(to_np(b2.pairs)[:M].view(np.uint64), ref2["stream"])
    # backward over the per-tile stream equals the uniform one up to the
    # order of the float atomic sums
    d = torch.as_tensor(np.random.default_rng(1).normal(size=(H, W, 3)).astype(np.float32)).to(dev())
    g1 = r.rasterize_backward(s, i, b2, d, None)
    g2 = r_u.rasterize_backward(s, i, b_u, d, None)
    torch.cuda.synchronize()
    a1, a2 = to_np(g1).astype(np.float64), to_np(g2).astype(np.float64)
    scale = np.abs(a2).max(axis=0, keepdims=True) + 1e-30
    assert np.all(np.abs(a1 - a2) <= 1e-4 * (np.abs(a2) + 1e-3 * scale))


@pytest.mark.parametrize("slack", [0, 1, 4000])
def test_global_order_without_host_count(slack):
    # GLOBAL without the host entry count sorts every slot of the capacity,
    # the unused ones padded past the last tile: the stream, the ranges and
    # the image equal the oracle's and the synchronised path's
    n, W, H = 5000, 200, 120
    splats, info = scenes.random_splats(n, W, H, seed=9, tie_fraction=0.2, hidden_fraction=0.1)
    cam = cam_for(W, H)
    depth, rect = scenes.info_depth(info), scenes.info_rects(info)
    ref = oracle.schedule(depth, rect, 13, 8, znear=cam["znear"], zfar=cam["zfar"])
    M = ref["M"]
    r = tg.Renderer(cam, tg.Params(), device=dev())
    s = torch.as_tensor(splats).to(dev())
    i = torch.as_tensor(info.view(np.int32)).to(dev())
    r._binned[0] = tg.Binned("global", M + slack, r.tiles, 64, 0, dev())
    b = r.bin(s, i, "global", sync=False)
    out = r.rasterize(s, i, b)
    torch.cuda.synchronize()
    assert int(to_np(b.counters)[0]) == M and int(to_np(b.counters)[2]) == 0
    assert np.array_equal(to_np(b.keys)[:M].view(np.uint64), ref["keys"])
    assert np.array_equal(to_np(b.vals)[:M].view(np.uint32), ref["vals"])
    assert np.array_equal(to_np(b.offsets).view(np.uint32), ref["tile_offsets"])
    rs = tg.Renderer(cam, tg.Params(), device=dev())
    want = rs.rasterize(s, i, rs.bin(s, i, "global", sync=True))
    torch.cuda.synchronize()
    assert torch.equal(out["rgb"], want["rgb"]) and torch.equal(out["last"], want["last"])


def test_global_order_without_host_count_overflow():
    splats, info = scenes.random_splats(2000, 128, 128, seed=5)
    cam = cam_for(128, 128)
    M = oracle.count_entries(scenes.info_rects(info))
    r = tg.Renderer(cam, tg.Params(), device=dev())
    s = torch.as_tensor(splats).to(dev())
    i = torch.as_tensor(info.view(np.int32)).to(dev())
    r._binned[0] = tg.Binned("global", M // 2, r.tiles, 64, 0, dev())
    b = r.bin(s, i, "global", sync=False)
    out = r.rasterize(s, i, b)
    torch.cuda.synchronize()
    c = to_np(b.counters)
    assert c[0] == M and c[2] == 1
    assert np.all(np.isnan(to_np(out["rgb"])))


@pytest.mark.parametrize("ts", [8, 16, 32])
def test_three_sigma_footprint(ts):
    # the baseline's 3-sigma tile rule: rects equal to the oracle's (outside
    # its rounding flags), images within 1e-4 of the oracle's tiled render
    # with the same rects, binned == global bitwise
    g, cam = scenes.training_scene(seed=6, n=20000, width=320, height=208)
    W, H = cam["width"], cam["height"]
    ref = oracle.project(g, cam, tile_size=ts, footprint="three_sigma")
    gd = tg.to_device(g, dev())
    p = tg.Params(tile_size=ts, footprint="three_sigma", num_bins=32)
    splats, info = tg.project(gd, cam, p)
    torch.cuda.synchronize()
    depth, rect = decode_info(to_np(info))
    vis = (rect[:, 2] > rect[:, 0]) & (rect[:, 3] > rect[:, 1])
    amb = (ref["flags"] & (oracle.AMBIG_RECT | oracle.AMBIG_VIS)) > 0
    vis_ref = (ref["flags"] & oracle.VISIBLE) > 0
    assert np.array_equal(vis[~amb], vis_ref[~amb])
    ok = vis & vis_ref & ~amb
    assert np.array_equal(rect[ok], ref["rect"][ok].astype(np.int64))
    # no opacity cut: Gaussians below 1/255 keep their tiles
    assert np.any(vis & (ref["opacity"] < 1 / 255))
    want = oracle.render(ref, W, H, tile_size=ts)
    r = tg.Renderer(cam, p, device=dev())
    imgs = {}
    for order in ("binned", "global"):
        out = r.rasterize(splats, info, r.bin(splats, info, order))
        torch.cuda.synchronize()
        e_rgb, e_a, nflag = image_compare(to_np(out["rgb"]), to_np(out["alpha"]), want)
        assert e_rgb <= TOL and e_a <= TOL, (ts, order, e_rgb, e_a, nflag)
        imgs[order] = to_np(out["rgb"])
    assert np.array_equal(imgs["binned"], imgs["global"])
    # the cut at the 3-sigma tiles changes the image against the
    # opacity-aware footprint
    ro = tg.Renderer(cam, tg.Params(tile_size=ts, num_bins=32), device=dev())
    full = ro.render(gd)
    torch.cuda.synchronize()
    assert float(np.abs(to_np(full["rgb"]) - imgs["binned"]).max()) > 1e-3
