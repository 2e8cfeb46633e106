"""GPU parity of the learned bin-count proposal against the FP64 reference
(oracle/mlp.py): tile features, logits and choices, the training step's
loss and gradient and the SGD update, the fallback, and that images do not
depend on the proposed counts."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from oracle import mlp
from helpers import to_np

pytestmark = pytest.mark.gpu

tg = pytest.importorskip("paper_2609_03613_amd")
from paper_2609_03613_amd import bins  # noqa: E402


def dev():
    return torch.device("cuda:0")


def rel_err(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max() + 1e-30
    return float(np.max(np.abs(got - ref) / (np.abs(ref) + 1e-3 * scale)))


def test_tile_features_match_oracle():
    n, W, H = 5000, 210, 150
    splats, info = scenes.random_splats(n, W, H, seed=41, tie_fraction=0.05)
    cam = scenes.camera(np.eye(3), np.zeros(3), 100.0, 100.0, W / 2, H / 2, W, H)
    tx, ty = (W + 15) // 16, (H + 15) // 16
    kt = (2 ** np.random.default_rng(3).integers(0, 9, size=tx * ty)).astype(np.int32)
    ref_s = oracle.schedule_tiles(scenes.info_depth(info), scenes.info_rects(info), tx, ty, kt,
                                  znear=cam["znear"], zfar=cam["zfar"])
    ref = mlp.tile_features(ref_s["bin_offsets"], ref_s["seg_base"], ref_s["M"])
    r = tg.Renderer(cam, tg.Params(num_bins=256, per_tile_bins=torch.as_tensor(kt).to(dev())), device=dev())
    s = torch.as_tensor(splats).to(dev())
    i = torch.as_tensor(info.view(np.int32)).to(dev())
    b = r.bin(s, i, "binned")
    f = to_np(bins.tile_features(r, b))
    assert np.abs(f - ref).max() <= 2e-5 * (1 + np.abs(ref)).max()
    # uniform K
    r2 = tg.Renderer(cam, tg.Params(num_bins=32), device=dev())
    b2 = r2.bin(s, i, "binned")
    ref2s = oracle.schedule(scenes.info_depth(info), scenes.info_rects(info), tx, ty, K=32,
                            znear=cam["znear"], zfar=cam["zfar"])
    ref2 = mlp.tile_features(ref2s["bin_offsets"], np.arange(tx * ty + 1) * 32, ref2s["M"])
    f2 = to_np(bins.tile_features(r2, b2))
    assert np.abs(f2 - ref2).max() <= 2e-5 * (1 + np.abs(ref2)).max()


def test_proposal_matches_oracle_and_fallback():
    rng = np.random.default_rng(5)
    w = rng.normal(0.0, 0.3, size=mlp.NUM_PARAMS).astype(np.float32)
    x = rng.normal(0.0, 1.0, size=(3000, 16)).astype(np.float32)
    z_ref, _ = mlp.forward(w.astype(np.float64), x.astype(np.float64))
    wt = torch.as_tensor(w).to(dev())
    xt = torch.as_tensor(x).to(dev())
    logits = torch.empty((3000, 8), dtype=torch.float32, device=dev())
    k = to_np(bins.propose_bins(wt, xt, logits=logits))
    # binary32 dot products of length <= 64 through three layers
    assert np.abs(to_np(logits) - z_ref).max() <= 2e-5 * np.abs(z_ref).max()
    srt = np.sort(z_ref, axis=1)
    clear = srt[:, -1] - srt[:, -2] > 1e-4
    assert np.array_equal(k[clear], mlp.choose_bins(w.astype(np.float64), x.astype(np.float64))[clear])
    assert clear.mean() > 0.95
    bad = w.copy()
    bad[100] = np.nan
    kb = to_np(bins.propose_bins(torch.as_tensor(bad).to(dev()), xt, fallback=64))
    assert np.all(kb == 64)


def test_training_step_matches_oracle():
    rng = np.random.default_rng(7)
    T = 2500
    w = rng.normal(0.0, 0.3, size=mlp.NUM_PARAMS).astype(np.float32)
    x = rng.normal(0.0, 1.0, size=(T, 16)).astype(np.float32)
    r = rng.uniform(0.0, 1.0, size=(T, 8)).astype(np.float32)
    r -= r.min(axis=1, keepdims=True)
    w64, x64, r64 = w.astype(np.float64), x.astype(np.float64), r.astype(np.float64)
    g_ref = mlp.grad(w64, x64, r64)
    L_ref = mlp.loss(w64, x64, r64)
    xt, rt = torch.as_tensor(x).to(dev()), torch.as_tensor(r).to(dev())
    # lr = momentum = 0 and a zero velocity: the velocity returns the gradient
    tr = bins.Trainer(w, device=dev())
    loss = tr.step(xt, rt, 0.0, 0.0)
    torch.cuda.synchronize()
    assert abs(float(loss.item()) - L_ref) <= 1e-5 * abs(L_ref)
    # binary32 sums over 2500 tiles of terms of both signs (float atomics
    # per 512-tile chunk): relative to |g| + 1e-3 max |g|
    assert rel_err(to_np(tr.v), g_ref) <= 5e-4
    assert np.array_equal(to_np(tr.w), w)
    # two momentum steps against the reference update
    tr = bins.Trainer(w, device=dev())
    wr, vr = w64, np.zeros_like(w64)
    for _ in range(2):
        tr.step(xt, rt, 0.05, 0.9)
        wr, vr = mlp.sgd_step(wr, vr, mlp.grad(wr, x64, r64), 0.05, 0.9)
    torch.cuda.synchronize()
    assert rel_err(to_np(tr.v), vr) <= 5e-4
    assert np.abs(to_np(tr.w) - wr).max() <= 1e-6 * (1 + np.abs(wr).max())


def test_learned_bins_leave_images_unchanged():
    g, cam = scenes.scene_1080p(seed=3, n=40000, width=480, height=270, focal=275.0)
    gd = tg.to_device(g, dev())
    w = bins.init_weights(seed=1)
    rng = np.random.default_rng(0)
    w[-8:] = rng.normal(size=8)          # a network that prefers varied counts
    w[-8 - 64 * 8:-8] = rng.normal(0, 0.5, size=64 * 8)
    lb = bins.LearnedBins(cam, weights=w, device=dev(), judge=False)
    base = tg.render(gd, cam)
    outs = [lb.render(gd) for _ in range(3)]
    torch.cuda.synchronize()
    kt = to_np(lb.kt)
    assert len(np.unique(kt)) > 1
    for o in outs:
        for k in ("rgb", "alpha", "last"):
            assert torch.equal(o[k], base[k]), k
    # without weights: the fixed K
    lb0 = bins.LearnedBins(cam, weights=None, device=dev())
    assert torch.equal(lb0.render(gd)["rgb"], base["rgb"])


def modelled_cost(binned, r, c_seg, c_b):
    """Bin + repair cost of a stream under the cost model fitted at
    training (per-segment cost plus per-entry costs of the repair-length
    buckets)."""
    from paper_2609_03613_amd.train_bins import bucket_entries
    T = r.tiles
    if binned.seg_base is not None:
        sb = to_np(binned.seg_base).astype(np.int64)
    else:
        sb = np.arange(T + 1) * r.params.num_bins
    off = to_np(binned.offsets).view(np.uint32).astype(np.int64)[: sb[-1] + 1]
    lens = np.diff(off)
    kt = np.diff(sb)
    total = c_seg * sb[-1]
    for K in np.unique(kt):
        rows = np.flatnonzero(kt == K)
        L = np.stack([lens[sb[t]:sb[t] + K] for t in rows])
        total += float((bucket_entries(L) @ c_b).sum())
    return total


def test_trained_network_gain():
    # Held-out scenes of the scene-shaped structure (seeds outside the
    # training range). Three things are measured:
    # - the cost model fitted at training to the method's own timings: the
    #   committed network's per-tile counts must lower the modelled bin +
    #   repair cost against the fixed K = 64 (what it was trained to do);
    # - the network alone (judge off), HIP-event-timed bin stage per frame
    #   including features and proposal: reported, not bounded. On MI355X it
    #   is slower than the fixed K (the per-tile segment machinery costs more
    #   than the repair it saves, whose cost hardly depends on K with the
    #   sub-bin repair);
    # - the frame loop with the judge on (the product configuration): it must
    #   not lose more than its probing costs against the fixed K (ratio >=
    #   0.97 over 128 frames, probes included), and it must keep the faster
    #   mode. Frames run back to back, as in a frame loop, so the host-side
    #   judge runs ahead of the GPU.
    # Images are identical in every mode.
    w = bins.load_weights()
    assert w is not None, "committed weights missing or invalid"
    with np.load(bins.WEIGHTS_PATH, allow_pickle=False) as z:
        c_seg, c_b = float(z["c_seg"]), np.asarray(z["c_bucket"], np.float64)
    stream = torch.cuda.current_stream()
    ratios, raw, judged = [], [], []

    def per_frame_ms(fn, k, warm=8):
        # k frames back to back (the host runs ahead, as in a frame loop):
        # GPU time between events around all of them / k
        for _ in range(warm):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    for seed in (2000, 2001):
        g, cam = scenes.scene_1080p(seed=seed)
        gd = tg.to_device(g, dev())
        fixed = tg.Renderer(cam, tg.Params(), device=dev())
        s, i = tg.project(gd, cam, fixed.params)
        bf = fixed.bin(s, i, "binned")
        net = bins.LearnedBins(cam, weights=w, device=dev(), judge=False)
        for _ in range(3):
            r, bl = net.bin(s, i, sync=True)
        ratios.append(modelled_cost(bl, r, c_seg, c_b) / modelled_cost(bf, fixed, c_seg, c_b))
        a = r.rasterize(s, i, bl)
        b = fixed.rasterize(s, i, bf)
        torch.cuda.synchronize()
        assert torch.equal(a["rgb"], b["rgb"]) and torch.equal(a["last"], b["last"])
        t_fixed = per_frame_ms(lambda: fixed.bin(s, i, "binned", sync=False), 32)
        t_net = per_frame_ms(lambda: net.bin(s, i, sync=False), 32)
        raw.append(t_fixed / t_net)
        # the judge decides within its first frames (warm-up), then probes
        # the other mode every 32nd frame: those probes are in the mean
        lb = bins.LearnedBins(cam, weights=w, device=dev(), judge=True, warm=4, probe_every=32)
        t_judged = per_frame_ms(lambda: lb.bin(s, i, sync=False), 128, warm=16)
        t_fixed2 = per_frame_ms(lambda: fixed.bin(s, i, "binned", sync=False), 32)
        judged.append(max(t_fixed, t_fixed2) / t_judged)
        # the judge must keep the faster mode; within 5 % of each other the
        # two are a tie at the timing noise of separate measurements, and
        # either choice is right
        t_ref = min(t_fixed, t_fixed2)
        faster = "learned" if t_net < t_ref else "fixed"
        if abs(t_net - t_ref) > 0.05 * t_ref:
            assert lb.choice() == faster, (lb.choice(), t_net, t_fixed, t_fixed2)
        rj, bj = lb.bin(s, i, sync=True)
        c = rj.rasterize(s, i, bj)
        torch.cuda.synchronize()
        assert torch.equal(c["rgb"], b["rgb"]) and torch.equal(c["last"], b["last"])
    print(f"modelled cost learned / fixed K=64: {ratios}; measured bin-stage speed-up, network alone: {raw}, "
          f"with the judge: {judged}")
    assert max(ratios) < 0.97
    assert min(judged) >= 0.97
