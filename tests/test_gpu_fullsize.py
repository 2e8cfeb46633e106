"""Parity at the full size of the 1080p workload (1M Gaussians on 64
spheres / planes, SH degree 3, 1920x1080, f = 1100) in the launch
configuration the benchmark times (16 px tiles, K = 64, WAVE raster, ids
gathered from the splats, heaviest tiles first).

The oracle handles this size whole: the projection of every Gaussian, the
global and binned streams bit for bit (about 2.2M entries), the
selective-repair choices of the paper mode, and every pixel of the image,
end to end and stage-isolated.
"""
import functools

import numpy as np
import pytest
import torch

import oracle
import scenes
from helpers import decode_info, image_compare, proj_to_splats, to_np

pytestmark = pytest.mark.gpu

tg = pytest.importorskip("paper_2609_03613_amd")

TOL = 1e-4
K = 64


def dev():
    return torch.device("cuda:0")


@functools.lru_cache(maxsize=None)
def workload():
    g, cam = scenes.scene_1080p(seed=0)
    proj = oracle.project(g, cam)
    return g, cam, proj


@functools.lru_cache(maxsize=None)
def oracle_schedule():
    _, cam, proj = workload()
    splats, info = proj_to_splats(proj)
    depth, rect = scenes.info_depth(info), scenes.info_rects(info)
    ref = oracle.schedule(depth, rect, 120, 68, K=K, znear=cam["znear"], zfar=cam["zfar"])
    return splats, info, ref


def test_fullsize_projection():
    g, cam, ref = workload()
    splats, info = tg.project(tg.to_device(g, dev()), cam)
    torch.cuda.synchronize()
    s = to_np(splats).astype(np.float64)
    depth, rect = decode_info(to_np(info))
    vis_ref = (ref["flags"] & oracle.VISIBLE) > 0
    vis = (rect[:, 2] > rect[:, 0]) & (rect[:, 3] > rect[:, 1])
    amb = (ref["flags"] & (oracle.AMBIG_RECT | oracle.AMBIG_VIS)) > 0
    assert np.array_equal(vis[~amb], vis_ref[~amb])
    v = vis & vis_ref
    assert np.array_equal(depth[v].view(np.uint32), ref["depth_key"][v].view(np.uint32))
    ok = v & ~amb
    assert np.array_equal(rect[ok], ref["rect"][ok].astype(np.int64))
    np.testing.assert_allclose(s[v, 0:2] + s[v, 2:4], ref["mean2d"][v], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(s[v, 7], ref["opacity"][v], rtol=2e-7)
    np.testing.assert_allclose(s[v, 8:11], ref["rgb"][v], rtol=2e-7, atol=1e-7)
    print(f"visible {int(v.sum())}, ambiguous {int(amb.sum())}")


def test_fullsize_schedule_bit_exact():
    splats, info, ref = oracle_schedule()
    _, cam, _ = workload()
    M = ref["M"]
    assert M > 2_000_000
    r = tg.Renderer(cam, tg.Params(), device=dev())
    s = torch.as_tensor(splats).to(dev())
    i = torch.as_tensor(np.ascontiguousarray(info).view(np.int32)).to(dev())
    bg = r.bin(s, i, "global")
    bb = r.bin(s, i, "binned")
    torch.cuda.synchronize()
    assert bg.num_entries == M and bb.num_entries == M
    assert np.array_equal(to_np(bg.keys)[:M].view(np.uint64), ref["keys"])
    assert np.array_equal(to_np(bg.vals)[:M].view(np.uint32), ref["vals"])
    assert np.array_equal(to_np(bg.offsets).view(np.uint32), ref["tile_offsets"])
    assert np.array_equal(to_np(bb.zrange).view(np.uint32), ref["zrange"].view(np.uint32))
    assert np.array_equal(to_np(bb.offsets).view(np.uint32), ref["bin_offsets"])
    assert np.array_equal(to_np(bb.pairs)[:M].view(np.uint64), ref["stream"])
    # heaviest-first dispatch order: a permutation of the tiles, non-increasing bit length of the counts,
    # then the number of split tiles and their threshold (split_entries = 2048;
    # 2 x the mean of the 2529 non-empty tiles is below it, and the longest
    # tiles, 4096..7004 entries, reach twice that bound)
    order = to_np(bb.dispatch_order()).view(np.uint32)
    assert np.array_equal(np.sort(order), np.arange(120 * 68))
    cnt = np.diff(ref["tile_offsets"].astype(np.int64))
    blen = np.where(cnt[order] > 0, np.floor(np.log2(np.maximum(cnt[order], 1))) + 1, 0)
    assert np.all(np.diff(blen) <= 0)
    ns, thr = bb.split()
    assert ns == int((cnt >= 2048).sum()) > 0 and thr == 2048


def test_fullsize_image_full_frame():
    # every one of the 2,073,600 pixels, rgb and alpha: end to end (the
    # oracle's binary64 projection and compositing against the product
    # frame: binned order, heaviest tiles first, longest tiles split) and
    # stage-isolated (the oracle composites the GPU's own binary32 splats)
    g, cam, proj = workload()
    W, H = 1920, 1080
    want = oracle.render(proj, W, H)
    gd = tg.to_device(g, dev())
    r = tg.Renderer(cam, tg.Params(), device=dev())
    splats, info = tg.project(gd, cam)
    imgs, lasts, alphas = {}, {}, {}
    for order in ("binned", "global"):
        b = r.bin(splats, info, order)
        out = r.rasterize(splats, info, b)
        torch.cuda.synchronize()
        imgs[order] = to_np(out["rgb"])
        lasts[order] = to_np(out["last"])
        alphas[order] = to_np(out["alpha"])
        e_rgb, e_a, masked = image_compare(imgs[order], alphas[order], want)
        print(f"{order}: end to end max |d rgb| {e_rgb:.3e}, |d alpha| {e_a:.3e}, masked {masked} of {W * H}")
        assert masked <= 1e-2 * W * H
        assert e_rgb <= TOL and e_a <= TOL, (order, e_rgb, e_a)
    iso = oracle.render(oracle.splats_to_proj(to_np(splats), to_np(info).view(np.uint32)), W, H)
    e_rgb, e_a, masked = image_compare(imgs["binned"], alphas["binned"], iso)
    print(f"stage-isolated max |d rgb| {e_rgb:.3e}, |d alpha| {e_a:.3e}, masked {masked}")
    assert e_rgb <= TOL and e_a <= TOL and masked <= 1e-2 * W * H
    # the last composited entry: the oracle's stream position equals the
    # GPU's wherever the pixel is not flagged
    m = iso["flags"] == 0
    assert np.array_equal(lasts["binned"][m], iso["last_pos"][m])
    # both orders, with and without the heavy-tile split, and the
    # comparator kernel give the same image bit for bit
    assert np.array_equal(imgs["binned"], imgs["global"]) and np.array_equal(lasts["binned"], lasts["global"])
    r0 = tg.Renderer(cam, tg.Params(split_entries=0), device=dev())
    rp = tg.Renderer(cam, tg.Params(raster="plain", tile_order=False), device=dev())
    u = r0.rasterize(splats, info, r0.bin(splats, info, "binned"))
    c = rp.rasterize(splats, info, rp.bin(splats, info, "global"))
    torch.cuda.synchronize()
    assert torch.equal(u["rgb"], c["rgb"]) and torch.equal(u["last"], c["last"])
    assert np.array_equal(imgs["binned"], to_np(u["rgb"])) and np.array_equal(alphas["binned"], to_np(u["alpha"]))
    assert np.array_equal(lasts["binned"], to_np(u["last"]))


def test_fullsize_paper_mode_selection():
    splats, info, _ = oracle_schedule()
    _, cam, _ = workload()
    depth, rect = scenes.info_depth(info), scenes.info_rects(info)
    key = oracle.near_keys(depth, splats[:, 11], 1.0, 0.25, cam["znear"], cam["zfar"])
    ref = oracle.schedule_keyed(depth, key, rect, 120, 68, K=K, znear=cam["znear"], zfar=cam["zfar"])
    T = 120 * 68
    sel, used = oracle.repair_select(ref["bin_offsets"], T, K, 0.25)
    r = tg.Renderer(cam, tg.paper_params(), device=dev())
    s = torch.as_tensor(splats).to(dev())
    i = torch.as_tensor(np.ascontiguousarray(info).view(np.int32)).to(dev())
    b = r.bin(s, i, "binned")
    torch.cuda.synchronize()
    M = ref["M"]
    assert np.array_equal(to_np(b.zrange).view(np.uint32), ref["zrange"].view(np.uint32))
    assert np.array_equal(to_np(b.offsets).view(np.uint32), ref["bin_offsets"])
    assert np.array_equal(to_np(b.repaired)[:T * K], sel)
    assert int(to_np(b.counters)[3]) == used
    pairs = to_np(b.pairs)[:M].view(np.uint64)
    lens = np.diff(ref["bin_offsets"].astype(np.int64))
    seg = np.repeat(np.arange(T * K), lens)
    assert np.array_equal(pairs[np.lexsort((pairs, seg))], ref["stream"])
    on = np.repeat(sel.astype(bool), lens)
    assert np.array_equal(pairs[on], ref["stream"][on])
    print(f"paper mode at 1080p: {int(sel.sum())} segments, {used} of {M} entries repaired")
