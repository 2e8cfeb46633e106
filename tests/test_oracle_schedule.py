"""Pins of the oracle's integer schedule: emitted keys, global order, per-tile
ranges, robust depth range, log-depth bins, counts, offsets and the
tile-bin-major stream (supplement: depth-range and bin-construction
algorithms, log-depth-bin equation).

Brute force in plain Python on tiny inputs, numpy's sort/partition as an
independent order-statistics routine, closed forms of the bit-pattern
logarithm at powers of two, and the invariants the paper states (each tile
walks one contiguous interval; counts sum to M).
"""
import struct

import numpy as np
import pytest

import oracle
import scenes


def f32(x):
    return float(np.float32(x))


def bits(x):
    return struct.unpack("<I", struct.pack("<f", x))[0]


def tiny_case(seed, n=60, tx=5, ty=4, ties=True):
    rng = np.random.default_rng(seed)
    depth = rng.uniform(1.0, 9.0, size=n).astype(np.float32)
    if ties:
        depth[rng.integers(0, n, 10)] = depth[rng.integers(0, n, 10)]
    x0 = rng.integers(0, tx, n)
    y0 = rng.integers(0, ty, n)
    x1 = np.minimum(tx, x0 + rng.integers(0, 3, n))
    y1 = np.minimum(ty, y0 + rng.integers(0, 3, n))
    return depth, np.stack([x0, y0, x1, y1], 1).astype(np.int32)


@pytest.mark.parametrize("seed", range(4))
def test_global_list_brute_force(seed):
    tx, ty = 5, 4
    depth, rect = tiny_case(seed, tx=tx, ty=ty)
    entries = []
    for g in range(len(depth)):
        for y in range(rect[g, 1], rect[g, 3]):
            for x in range(rect[g, 0], rect[g, 2]):
                entries.append((y * tx + x, float(depth[g]), g))
    entries.sort()
    s = oracle.schedule(depth, rect, tx, ty, K=4)
    assert s["M"] == len(entries)
    assert [int(k >> 32) for k in s["keys"]] == [e[0] for e in entries]
    assert [int(k & 0xFFFFFFFF) for k in s["keys"]] == [bits(e[1]) for e in entries]
    assert s["vals"].tolist() == [e[2] for e in entries]
    for t in range(tx * ty):
        n_t = sum(1 for e in entries if e[0] == t)
        assert s["tile_offsets"][t + 1] - s["tile_offsets"][t] == n_t
        assert all(e[0] == t for e in entries[s["tile_offsets"][t]:s["tile_offsets"][t + 1]])


def test_depth_range_all_samples():
    # 101 depths 1..101 (<= S, all sampled): ranks floor(0.01 * 100) = 1 and
    # ceil(0.99 * 100) = 99 give 2 and 100; span 98, pad 4.9.
    depth = np.arange(1, 102, dtype=np.float32)[::-1].copy()
    rect = np.tile(np.array([[0, 0, 1, 1]], np.int32), (101, 1))
    zr = oracle.depth_range(depth, rect, znear=0.01, zfar=1e10)
    span = f32(f32(100.0) - f32(2.0))
    assert zr[0] == pytest.approx(0.01)  # 2 - 4.9 < znear
    assert zr[1] == f32(f32(100.0) + f32(f32(0.05) * span))
    zr = oracle.depth_range(depth, rect, znear=0.01, zfar=103.0)
    assert zr[1] == np.float32(103.0)


def test_depth_range_sampling_and_order_statistics():
    # V > S: the samples are the visible ids at ranks floor(i V / S); the order
    # statistics are then compared with numpy's sort.
    rng = np.random.default_rng(5)
    n, S = 30000, 8192
    depth = rng.lognormal(2.0, 0.5, n).astype(np.float32)
    rect = np.tile(np.array([[0, 0, 1, 1]], np.int32), (n, 1))
    hidden = rng.random(n) < 0.2
    rect[hidden, 2] = 0  # empty rect: not visible
    vis = np.nonzero(~hidden)[0]
    V = len(vis)
    sample = np.sort(depth[vis[(np.arange(S, dtype=np.int64) * V) // S]])
    lo = sample[int(np.floor(0.01 * (S - 1)))]
    hi = sample[int(np.ceil(0.99 * (S - 1)))]
    span = np.float32(hi - lo)
    pad = np.float32(np.float32(0.05) * span)
    zr = oracle.depth_range(depth, rect)
    assert zr[0] == np.float32(lo - pad)
    assert zr[1] == np.float32(hi + pad)
    # ranks agree with numpy's selection routine
    assert np.partition(sample, 81)[81] == sample[81]


def test_depth_range_degenerate():
    rect = np.array([[0, 0, 1, 1]] * 5, np.int32)
    zr = oracle.depth_range(np.full(5, 3.0, np.float32), rect)
    assert zr[0] == np.float32(np.float32(3.0) - np.float32(np.float32(0.05) * np.float32(1e-6)))
    zr = oracle.depth_range(np.full(5, 3.0, np.float32), np.zeros((5, 4), np.int32), znear=0.5, zfar=7.0)
    assert list(zr) == [0.5, 7.0]  # nothing visible


def test_bin_map_powers_of_two_closed_form():
    # With zmin = 1 and zmax = 2^k the bit-pattern logarithm is exact at
    # powers of two: 2^j falls in bin floor(K j / k).
    K, k = 64, 8
    for j in range(k + 1):
        b = oracle.bin_of(2.0 ** j, 1.0, 2.0 ** k, K)
        assert b == min(K - 1, (K * j) // k)


def test_bin_map_properties():
    rng = np.random.default_rng(0)
    z = np.sort(rng.uniform(0.5, 40.0, 5000).astype(np.float32))
    for K in (1, 4, 64, 256):
        b = [oracle.bin_of(v, 2.0, 30.0, K) for v in z]
        assert all(b[i] <= b[i + 1] for i in range(len(b) - 1))  # monotone in depth
        assert min(b) == 0 and max(b) == K - 1
        assert oracle.bin_of(1.0, 2.0, 30.0, K) == 0 and oracle.bin_of(31.0, 2.0, 30.0, K) == K - 1
    # log-like: the ratio of bin edges is about constant across octaves
    b = np.array([oracle.bin_of(v, 1.0, 16.0, 64) for v in (1.0, 2.0, 4.0, 8.0, 16.0)])
    assert b.tolist() == [0, 16, 32, 48, 63]
    assert oracle.bin_of(5.0, 5.0, 5.0, 16) == 0  # empty range


@pytest.mark.parametrize("seed", range(3))
def test_counts_offsets_and_stream_brute_force(seed):
    tx, ty, K = 5, 4, 8
    depth, rect = tiny_case(seed, n=80, tx=tx, ty=ty)
    s = oracle.schedule(depth, rect, tx, ty, K=K)
    zmin, zmax = s["zrange"]
    cnt = np.zeros(tx * ty * K, np.int64)
    segs = {}
    for g in range(len(depth)):
        b = oracle.bin_of(depth[g], zmin, zmax, K)
        for y in range(rect[g, 1], rect[g, 3]):
            for x in range(rect[g, 0], rect[g, 2]):
                q = (y * tx + x) * K + b
                cnt[q] += 1
                segs.setdefault(q, []).append((bits(float(depth[g])), g))
    off = np.concatenate([[0], np.cumsum(cnt)])
    np.testing.assert_array_equal(s["bin_offsets"], off)
    assert off[-1] == s["M"]
    for q, items in segs.items():
        want = [(d << 32) | g for d, g in sorted(items)]
        assert s["stream"][off[q]:off[q + 1]].tolist() == want


@pytest.mark.parametrize("K", [1, 2, 16, 64])
def test_exact_stream_equals_global_list(K):
    # Bins are monotone in the depth bits, so sorting every (tile, bin) segment
    # by (depth bits, id) reproduces the global (tile, depth, id) list tile by
    # tile; and each tile's bins form the tile's one contiguous interval.
    g, cam = scenes.small_forward(seed=1, n=1500)
    p = oracle.project(g, cam)
    s = oracle.schedule(p["depth_key"], p["rect"], 8, 8, K=K)
    glob = ((s["keys"] & np.uint64(0xFFFFFFFF)) << np.uint64(32)) | s["vals"].astype(np.uint64)
    np.testing.assert_array_equal(s["stream"], glob)
    bo = s["bin_offsets"]
    np.testing.assert_array_equal(bo[0::K], s["tile_offsets"])


def test_empty_schedule():
    s = oracle.schedule(np.zeros(0, np.float32), np.zeros((0, 4), np.int32), 3, 2, K=4)
    assert s["M"] == 0
    assert s["bin_offsets"].tolist() == [0] * 25
    assert s["tile_offsets"].tolist() == [0] * 7


@pytest.mark.parametrize("seed", range(3))
def test_per_tile_bins_brute_force(seed):
    # tile t has K_t bins numbered from seg_base[t] = K_0 + ... + K_{t-1};
    # counts, offsets and sorted segments written out by hand
    tx, ty = 5, 4
    depth, rect = tiny_case(seed, n=80, tx=tx, ty=ty)
    rng = np.random.default_rng(seed + 10)
    kt = (2 ** rng.integers(0, 7, size=tx * ty)).astype(np.int32)
    s = oracle.schedule_tiles(depth, rect, tx, ty, kt)
    zmin, zmax = s["zrange"]
    base = np.concatenate([[0], np.cumsum(kt)])
    np.testing.assert_array_equal(s["seg_base"], base)
    cnt = np.zeros(base[-1], np.int64)
    segs = {}
    for g in range(len(depth)):
        for y in range(rect[g, 1], rect[g, 3]):
            for x in range(rect[g, 0], rect[g, 2]):
                t = y * tx + x
                q = base[t] + oracle.bin_of(depth[g], zmin, zmax, int(kt[t]))
                cnt[q] += 1
                segs.setdefault(q, []).append((bits(float(depth[g])), g))
    off = np.concatenate([[0], np.cumsum(cnt)])
    np.testing.assert_array_equal(s["bin_offsets"], off)
    for q, items in segs.items():
        assert s["stream"][off[q]:off[q + 1]].tolist() == [(d << 32) | g for d, g in sorted(items)]


def test_per_tile_bins_special_cases():
    g, cam = scenes.small_forward(seed=2, n=1500)
    p = oracle.project(g, cam)
    uni = oracle.schedule(p["depth_key"], p["rect"], 8, 8, K=16)
    # the same K in every tile is the uniform schedule
    same = oracle.schedule_tiles(p["depth_key"], p["rect"], 8, 8, np.full(64, 16, np.int32))
    np.testing.assert_array_equal(same["bin_offsets"], uni["bin_offsets"])
    np.testing.assert_array_equal(same["stream"], uni["stream"])
    # any per-tile choice keeps the stream equal to the global list (bins are
    # monotone in depth) and each tile's range unchanged
    kt = (2 ** np.random.default_rng(4).integers(0, 9, size=64)).astype(np.int32)
    var = oracle.schedule_tiles(p["depth_key"], p["rect"], 8, 8, kt)
    np.testing.assert_array_equal(var["stream"], uni["stream"])
    np.testing.assert_array_equal(var["bin_offsets"][var["seg_base"]], uni["tile_offsets"])


def test_rects_outside_the_grid_are_rejected():
    # a rect in another tile size's units (8-pixel tiles handed to a 16-pixel
    # grid) reaches past the tile lists: the tiled render, the schedule and
    # the compositing adjoint refuse it instead of indexing past their arrays;
    # so does a pixel outside the image
    W, H = 160, 40
    splats, info = scenes.random_splats(300, W, H, tile_size=8, seed=3)
    proj = oracle.splats_to_proj(splats, info)
    assert proj["rect"][:, 2].max() > (W + 15) // 16
    oracle.render(proj, W, H, tile_size=8)
    with pytest.raises(AssertionError):
        oracle.render(proj, W, H, tile_size=16)
    depth, rect = scenes.info_depth(info), scenes.info_rects(info)
    oracle.schedule(depth, rect, (W + 7) // 8, (H + 7) // 8, K=8)
    with pytest.raises(AssertionError):
        oracle.schedule(depth, rect, (W + 15) // 16, (H + 15) // 16, K=8)
    d_img = np.zeros((H, W, 3))
    oracle.composite_adjoint(proj, W, H, tile_size=8, d_img=d_img)
    with pytest.raises(AssertionError):
        oracle.composite_adjoint(proj, W, H, tile_size=16, d_img=d_img)
    with pytest.raises(AssertionError):
        oracle.render(proj, W, H, tile_size=8, pix=np.array([[W, 0]], np.int32))
