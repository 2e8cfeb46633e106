"""Oracle parity at the stated sizes of the remaining workloads, in the
launch configurations the benchmark times:

- the training step: 500k Gaussians (SH3) at 1297x840, with 16-pixel tiles
  and K = 64 and with the autotuned 32-pixel tiles and K = 128, every
  Gaussian's gradient line against the oracle's compositing adjoint of the
  same splats, and every Gaussian's parameter gradients against the oracle's
  projection adjoint;
- the 4K evaluation scene of the learned bins: 6M Gaussians (SH3) at
  3840x2160, the global and binned streams (22M entries) bit for bit and
  65,536 random pixels end to end;
- the scale-up point: 10M Gaussians of the 1080p structure, the binned stream
  (about 22M entries, sub-segments past the 8192-entry LDS sort included) bit
  for bit and 65,536 pixels;
- the batched frame: 3M Gaussians on 16 ring cameras (640x360 .. 2560x1440),
  one persistent launch, 8192 random pixels of every view end to end.

Bars as elsewhere: integer results bit-exact; images within 1e-4 of the FP64
oracle on pixels it did not flag; gradients within 1e-3 per gradient column as
|gpu - ref| / (|ref| + 1e-3 max |ref|), with the upstream gradient zeroed on
flagged pixels. The oracle flags a pixel when one of its alpha tests lies
within the binary32 rounding bound of the 1/255 cut or its stop test within
2e-4 relative of 1e-4; with tens of alpha-supported tests per pixel that is
0.1-0.5 % of the pixels here (reported; held below 1 % so that the mask
cannot hide a broken image).
"""
import functools

import numpy as np
import pytest
import torch

import oracle
import scenes
from helpers import decode_info, image_compare, to_np

pytestmark = pytest.mark.gpu

tg = pytest.importorskip("paper_2609_03613_amd")

TOL = 1e-4
GRAD_TOL = 1e-3
KEYS = ("means", "log_scales", "quats", "logits", "sh")
AMBIG = oracle.PIX_AMBIG_ALPHA | oracle.PIX_AMBIG_STOP | oracle.PIX_AMBIG_GAUSS


def dev():
    return torch.device("cuda:0")


def grad_err(gpu, ref):
    gpu = np.asarray(gpu, np.float64).reshape(len(ref), -1)
    ref = np.asarray(ref, np.float64).reshape(len(ref), -1)
    scale = np.abs(ref).max(axis=0, keepdims=True)
    err = np.abs(gpu - ref) / (np.abs(ref) + 1e-3 * scale + 1e-30)
    return float(err.max())


# ---------------------------------------------------------------------------
# training step: 500k Gaussians, SH3, 1297x840
# ---------------------------------------------------------------------------

# the paper's tile size and bins, and the ones the autotuner picks for this camera
@pytest.mark.parametrize("ts,K", [(16, 64), (32, 128)])
def test_training_step_gradients_full_size(ts, K):
    g, cam = scenes.training_scene(seed=0)
    W, H = cam["width"], cam["height"]
    n = len(g["logits"])
    target = scenes.training_target(W, H)
    gd = tg.to_device(g, dev())
    p = tg.Params(tile_size=ts, num_bins=K)
    r = tg.Renderer(cam, p, device=dev())
    splats, info = tg.project(gd, cam, p)
    b = r.bin(splats, info, "binned", fresh=True)
    fwd = r.rasterize(splats, info, b, trans=True)
    torch.cuda.synchronize()
    assert b.num_entries > (7_000_000 if ts == 16 else 2_500_000)
    proj = oracle.splats_to_proj(to_np(splats), to_np(info).view(np.uint32))
    ref_fwd = oracle.render(proj, W, H, tile_size=ts)
    e_rgb, e_a, _ = image_compare(to_np(fwd["rgb"]), to_np(fwd["alpha"]), ref_fwd)
    assert e_rgb <= TOL and e_a <= TOL, (e_rgb, e_a)
    mask = (ref_fwd["flags"] & AMBIG) == 0
    assert mask.mean() > 0.99
    # the loss gradient of mean((rgb - target)^2) at the oracle's image, in
    # binary32 so that both sides see the same upstream values
    up = (2.0 * (ref_fwd["rgb"] - target) / ref_fwd["rgb"].size * mask[..., None]).astype(np.float32)
    ref = oracle.composite_adjoint(proj, W, H, tile_size=ts, d_img=up)
    up_d = torch.as_tensor(up).to(dev())
    # the benchmark's step (forward state saved), and the recomputed walk
    d_saved = to_np(r.rasterize_backward(splats, info, b, up_d, saved=fwd))
    d_walk = to_np(r.rasterize_backward(splats, info, b, up_d))
    torch.cuda.synchronize()
    for name, d in (("saved", d_saved), ("recomputed", d_walk)):
        errs = [grad_err(d[:, k], ref["d_proj"][:, k]) for k in range(9)]
        print(name, "gradient-line errors", ["%.2e" % e for e in errs])
        assert max(errs) <= GRAD_TOL, (name, errs)
    # projection backward of every Gaussian: fed the oracle's gradient lines
    # (rounded to binary32) against the oracle's projection adjoint of the
    # same lines, and end to end (the GPU's own lines). Gaussians whose
    # visibility or rect the oracle finds within rounding of an edge are left
    # out on both sides.
    pflags = oracle.project(g, cam, tile_size=ts)["flags"]
    keep = (pflags & (oracle.AMBIG_RECT | oracle.AMBIG_VIS)) == 0
    d32 = np.zeros((n, 12), np.float32)
    d32[:, :9] = ref["d_proj"]
    d32[~keep] = 0.0
    want = oracle.project_adjoint(g, cam, d32[:, :9].astype(np.float64))
    got = tg.project_backward(gd, cam, torch.as_tensor(d32).to(dev()))
    dg = d_saved.copy()
    dg[~keep] = 0.0
    want_e2e = oracle.project_adjoint(g, cam, np.where(keep[:, None], ref["d_proj"], 0.0))
    got_e2e = tg.project_backward(gd, cam, torch.as_tensor(dg).to(dev()))
    torch.cuda.synchronize()
    for k in KEYS:
        e = grad_err(to_np(got[k]), want[k])
        e2 = grad_err(to_np(got_e2e[k]), want_e2e[k])
        print(k, "projection backward %.2e, end to end %.2e" % (e, e2))
        assert e <= 1e-4, (k, e)
        assert e2 <= GRAD_TOL, (k, e2)


# ---------------------------------------------------------------------------
# 6M Gaussians at 3840x2160 and the 10M scale-up point at 1080p
# ---------------------------------------------------------------------------

def _stream_and_pixels(g, cam, n_pix=65536, seed=3, check_global=True):
    W, H = cam["width"], cam["height"]
    tx, ty = (W + 15) // 16, (H + 15) // 16
    gd = tg.to_device(g, dev())
    r = tg.Renderer(cam, tg.Params(), device=dev())
    splats, info = tg.project(gd, cam)
    bb = r.bin(splats, info, "binned")
    out = r.rasterize(splats, info, bb)
    torch.cuda.synchronize()
    depth, rect = decode_info(to_np(info))
    ref = oracle.schedule(depth, rect, tx, ty, K=64, znear=cam["znear"], zfar=cam["zfar"])
    M = ref["M"]
    assert bb.num_entries == M
    assert np.array_equal(to_np(bb.zrange).view(np.uint32), ref["zrange"].view(np.uint32))
    assert np.array_equal(to_np(bb.offsets).view(np.uint32), ref["bin_offsets"])
    assert np.array_equal(to_np(bb.pairs)[:M].view(np.uint64), ref["stream"])
    lens = np.diff(ref["bin_offsets"].astype(np.int64))
    if check_global:
        rg = tg.Renderer(cam, tg.Params(raster="plain", tile_order=False), device=dev())
        bgl = rg.bin(splats, info, "global")
        torch.cuda.synchronize()
        assert bgl.num_entries == M
        assert np.array_equal(to_np(bgl.keys)[:M].view(np.uint64), ref["keys"])
        assert np.array_equal(to_np(bgl.vals)[:M].view(np.uint32), ref["vals"])
        assert np.array_equal(to_np(bgl.offsets).view(np.uint32), ref["tile_offsets"])
        del bgl, rg
    rgb, alpha = to_np(out["rgb"]), to_np(out["alpha"])
    del bb, out, splats, info, gd, r
    torch.cuda.empty_cache()
    rng = np.random.default_rng(seed)
    pix = np.stack([rng.integers(0, W, n_pix), rng.integers(0, H, n_pix)], 1)
    want = oracle.render(oracle.project(g, cam), W, H, pix=pix)
    m = want["flags"] == 0
    e_rgb = float(np.abs(rgb[pix[:, 1], pix[:, 0]] - want["rgb"])[m].max())
    e_a = float(np.abs(alpha[pix[:, 1], pix[:, 0]] - want["alpha"])[m].max())
    e_masked = float(np.abs(rgb[pix[:, 1], pix[:, 0]] - want["rgb"])[~m].max(initial=0.0))
    print(f"M = {M}, longest segment {int(lens.max())}, pixels: max |d rgb| {e_rgb:.3e}, "
          f"|d alpha| {e_a:.3e}, masked {int((~m).sum())} of {n_pix} (max |d rgb| there {e_masked:.2e})")
    assert (~m).sum() <= 1e-2 * n_pix
    assert e_rgb <= TOL and e_a <= TOL
    return M, lens


def test_4k_6M_stream_and_pixels():
    g, cam = scenes.learned_eval_scene(seed=0)
    M, _ = _stream_and_pixels(g, cam)
    assert M > 20_000_000


def test_scale_up_10M_stream_and_pixels():
    g, cam = scenes.scene_1080p(seed=0, n=10_000_000)
    M, lens = _stream_and_pixels(g, cam, check_global=False)
    assert M > 20_000_000
    # the long-segment tail sort (more than 8192 entries in one bin) runs here
    assert int(lens.max()) > 8192


# ---------------------------------------------------------------------------
# batched frame: 3M Gaussians, 16 ring cameras
# ---------------------------------------------------------------------------

BATCH_PARAMS = [dict(tile_size=32, num_bins=128), dict(tile_size=16, num_bins=64), dict(tile_size=32, num_bins=64),
                dict(tile_size=8, num_bins=32)]


@functools.lru_cache(maxsize=None)
def batched_frame():
    g, cams = scenes.batched_scene(seed=0)
    gd = tg.to_device(g, dev())
    params = [tg.Params(**BATCH_PARAMS[v % len(BATCH_PARAMS)]) for v in range(len(cams))]
    br = tg.BatchRenderer(cams, params, device=dev())
    br.capture(gd)
    br.replay()
    torch.cuda.synchronize()
    assert not br.overflowed()
    outs = [{k: to_np(v) for k, v in o.items()} for o in br.outs]
    return g, cams, params, outs, sum(br.entries)


@pytest.mark.parametrize("view", range(16))
def test_batched_3M_16_views_against_oracle(view):
    g, cams, params, outs, entries = batched_frame()
    assert entries > 200_000_000
    c = cams[view]
    W, H = c["width"], c["height"]
    rng = np.random.default_rng(100 + view)
    pix = np.stack([rng.integers(0, W, 8192), rng.integers(0, H, 8192)], 1)
    want = oracle.render(oracle.project(g, c, tile_size=params[view].tile_size), W, H,
                         tile_size=params[view].tile_size, pix=pix)
    m = want["flags"] == 0
    o = outs[view]
    e_rgb = float(np.abs(o["rgb"][pix[:, 1], pix[:, 0]] - want["rgb"])[m].max())
    e_a = float(np.abs(o["alpha"][pix[:, 1], pix[:, 0]] - want["alpha"])[m].max())
    e_masked = float(np.abs(o["rgb"][pix[:, 1], pix[:, 0]] - want["rgb"])[~m].max(initial=0.0))
    print(f"view {view} {W}x{H}: max |d rgb| {e_rgb:.3e}, |d alpha| {e_a:.3e}, masked {int((~m).sum())} "
          f"(max |d rgb| there {e_masked:.2e})")
    assert (~m).sum() <= 1e-2 * len(pix)
    assert e_rgb <= TOL and e_a <= TOL
