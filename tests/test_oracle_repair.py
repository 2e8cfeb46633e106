"""Pins of the oracle's selective-repair mode: the near-depth binning key
(supplement, Algorithm "Robust depth-range estimation", near-depth mode),
the keep rules (Table "Exact-repair selection rules") and the first-fit
entry budget (supplement, Algorithm "Selective repair selection and local
exact sorting"), and compositing over a given traversal order.

Pins: hand-worked selections whose expected sets were written out from the
rule table (boundary cases of every threshold and a budget walk-through),
exact binary32 values of the shifted key, brute force in plain Python for
the keyed schedule on tiny inputs, and closed-form two-Gaussian composites
for the traversal order.
"""
import struct

import numpy as np
import pytest

import oracle
import scenes


def bits(x):
    return struct.unpack("<I", struct.pack("<f", float(x)))[0]


def offsets_of(lengths):
    return np.concatenate([[0], np.cumsum(np.asarray(lengths, np.int64))]).astype(np.uint32)


# ---------------------------------------------------------------------------
# near-depth key
# ---------------------------------------------------------------------------

def test_near_key_exact_values():
    z = np.array([8.0, 8.0, 8.0, 8.0, 0.02, 0.02], np.float32)
    smax = np.array([0.0, 1.0, 3.0, 1e6, 1.0, 0.001], np.float32)
    k = oracle.near_keys(z, smax, alpha=1.0, gamma=0.25, znear=0.015, zfar=100.0)
    # min(alpha s, gamma z): 0 -> z; 1 < 2 -> z - 1; 3 > 2 -> z - 2 (= 0.75 z);
    # huge -> 0.75 z; 0.02 - 0.005 = 0.015 = znear (clamped from below at
    # most to znear); 0.02 - 0.001 = 0.019
    assert k.tolist() == [8.0, 7.0, 6.0, 6.0, np.float32(0.02) - np.float32(0.005), np.float32(0.019)]
    assert k[4] >= np.float32(0.015)
    # alpha = 0 leaves every key at its depth
    assert np.array_equal(oracle.near_keys(z, smax, alpha=0.0, znear=0.015, zfar=100.0), z)
    # clamps: below max(znear, 1e-4) and above zfar
    lo = oracle.near_keys(np.array([0.01], np.float32), np.array([1.0], np.float32), znear=1e-6, zfar=10.0)
    assert lo[0] == np.float32(0.0075)
    lo = oracle.near_keys(np.array([1e-4], np.float32), np.array([1.0], np.float32), znear=1e-6, zfar=10.0)
    assert lo[0] == np.float32(1e-4)
    hi = oracle.near_keys(np.array([50.0], np.float32), np.array([0.0], np.float32), znear=0.01, zfar=20.0)
    assert hi[0] == np.float32(20.0)


def test_near_key_monotone_per_scale_not_across_scales():
    z = np.linspace(0.5, 40.0, 4001).astype(np.float32)
    for s in (0.0, 0.01, 0.3, 2.0, 50.0):
        k = oracle.near_keys(z, np.full_like(z, s), znear=0.01, zfar=1e4)
        assert np.all(np.diff(k.astype(np.float64)) >= 0.0), s
    # a larger Gaussian slightly behind a small one gets the nearer key: the
    # key order can disagree with the depth order, so bins formed on it are
    # not monotone in the depth
    k = oracle.near_keys(np.array([10.0, 10.5], np.float32), np.array([0.0, 1.0], np.float32), znear=0.01, zfar=1e4)
    assert k[1] < k[0]


# ---------------------------------------------------------------------------
# keep rules and budget
# ---------------------------------------------------------------------------

# (bin lengths of one tile with K = 4, expected kept flags) -- worked by hand
# from the rule table; the comment names the rule that decides each segment.
RULE_CASES = [
    ([0, 0, 320, 680], [0, 0, 1, 1]),     # (i) at 320; (i)
    ([0, 0, 319, 1000], [0, 0, 0, 1]),    # 319: (i) no, share 24 % no, (iv) no (> 256)
    ([0, 0, 45, 55], [0, 0, 1, 1]),       # (iii) at exactly 45 %
    ([0, 0, 44, 56], [0, 0, 0, 1]),       # 44 %: no rule
    ([0, 0, 129, 1161], [0, 0, 1, 1]),    # (iv) at 129 and exactly 10 %
    ([0, 0, 128, 1152], [0, 0, 0, 1]),    # 128 is below the (iv) range; share 10 % < 45 %
    ([0, 0, 257, 2313], [0, 0, 0, 1]),    # 257 is above the (iv) range; 10 % share
    ([16, 1000, 0, 0], [1, 1, 0, 0]),     # (v) at 16 in bin 0; (i)
    ([0, 15, 9, 1000], [0, 0, 0, 1]),     # bin 1 with 15 < 16; 9: share < 45 %
    ([0, 0, 16, 1000], [0, 0, 0, 1]),     # bin 2: (v) does not apply
    ([0, 16, 0, 1000], [0, 1, 0, 1]),     # (v) in bin 1
    ([2, 0, 0, 0], [1, 0, 0, 0]),         # two entries, 100 % share
    ([1, 0, 0, 0], [0, 0, 0, 0]),         # one entry: never repaired
    ([0, 0, 0, 513], [0, 0, 0, 1]),       # (ii) / (i)
]


def test_keep_rules_boundaries():
    lengths = [l for c, _ in RULE_CASES for l in c]
    expect = [e for _, es in RULE_CASES for e in es]
    sel, used = oracle.repair_select(offsets_of(lengths), len(RULE_CASES), 4, budget_frac=1.0)
    assert sel.tolist() == expect
    assert used == sum(l for l, e in zip(lengths, expect) if e)


def test_budget_first_fit_walkthrough():
    # tiles (K = 4): [16, 0, 3, 300] [1, 15, 200, 700] [2, 2, 0, 0]; M = 1239
    # kept: seg 0 (v), seg 3 (iii: 300 of 319), seg 6 (iv: 200 of 916),
    # seg 7 (i), seg 8 and 9 (iii: 2 of 4). B = floor(0.25 * 1239) = 309.
    # First fit: 16 -> 16; 300 would give 316 > 309: skipped; 200 -> 216;
    # 700 skipped; 2 -> 218; 2 -> 220.
    off = offsets_of([16, 0, 3, 300, 1, 15, 200, 700, 2, 2, 0, 0])
    sel, used = oracle.repair_select(off, 3, 4, budget_frac=0.25)
    assert np.nonzero(sel)[0].tolist() == [0, 6, 8, 9] and used == 220
    sel, used = oracle.repair_select(off, 3, 4, budget_frac=1.0)
    assert np.nonzero(sel)[0].tolist() == [0, 3, 6, 7, 8, 9] and used == 1220
    # a budget of zero selects nothing (every kept segment has >= 2 entries)
    sel, used = oracle.repair_select(off, 3, 4, budget_frac=0.0)
    assert not sel.any() and used == 0
    # B = floor(0.0145 * 1239) = 17: 16 fits, then only the 2-entry segments
    # would, and 16 + 2 = 18 > 17
    sel, used = oracle.repair_select(off, 3, 4, budget_frac=0.0145)
    assert np.nonzero(sel)[0].tolist() == [0] and used == 16


def test_selection_within_budget_and_first_fit_property():
    rng = np.random.default_rng(3)
    T, K = 40, 8
    lengths = rng.choice([0, 1, 2, 3, 5, 16, 40, 150, 330, 600], size=T * K,
                         p=[.3, .15, .1, .1, .1, .08, .07, .05, .03, .02])
    off = offsets_of(lengths)
    M = int(off[-1])
    _, used_all = oracle.repair_select(off, T, K, budget_frac=1.0)
    kept, _ = oracle.repair_select(off, T, K, budget_frac=1.0)
    for frac in (0.0, 0.05, 0.1, 0.25, 0.5):
        sel, used = oracle.repair_select(off, T, K, budget_frac=frac)
        B = int(np.floor(frac * M))
        assert used <= B and used == int(lengths[sel.astype(bool)].sum())
        assert np.all(sel <= kept)
        # first fit: every kept segment left out did not fit the budget
        # given what was taken before it
        taken = 0
        for q in range(T * K):
            if sel[q]:
                taken += int(lengths[q])
            elif kept[q]:
                assert taken + int(lengths[q]) > B
    assert used_all == int(lengths[kept.astype(bool)].sum())


# ---------------------------------------------------------------------------
# keyed schedule
# ---------------------------------------------------------------------------

def tiny(seed, n=80, tx=5, ty=4):
    rng = np.random.default_rng(seed)
    depth = rng.uniform(1.0, 9.0, size=n).astype(np.float32)
    depth[rng.integers(0, n, 10)] = depth[rng.integers(0, n, 10)]
    smax = np.exp(rng.uniform(np.log(0.01), np.log(3.0), size=n)).astype(np.float32)
    x0 = rng.integers(0, tx, n)
    y0 = rng.integers(0, ty, n)
    x1 = np.minimum(tx, x0 + rng.integers(0, 3, n))
    y1 = np.minimum(ty, y0 + rng.integers(0, 3, n))
    return depth, smax, np.stack([x0, y0, x1, y1], 1).astype(np.int32)


@pytest.mark.parametrize("seed", range(3))
def test_keyed_schedule_brute_force(seed):
    tx, ty, K = 5, 4, 8
    depth, smax, rect = tiny(seed, tx=tx, ty=ty)
    key = oracle.near_keys(depth, smax, znear=0.01, zfar=1e10)
    s = oracle.schedule_keyed(depth, key, rect, tx, ty, K=K)
    # the range comes from the keys, not the depths
    assert np.array_equal(s["zrange"], oracle.depth_range(key, rect))
    zmin, zmax = s["zrange"]
    segs = [[] for _ in range(tx * ty * K)]
    for g in range(len(depth)):
        for y in range(rect[g, 1], rect[g, 3]):
            for x in range(rect[g, 0], rect[g, 2]):
                b = oracle.bin_of(key[g], zmin, zmax, K)
                segs[(y * tx + x) * K + b].append((bits(depth[g]) << 32) | g)
    stream = [v for sg in segs for v in sorted(sg)]
    assert s["stream"].tolist() == stream
    assert s["bin_offsets"].tolist() == offsets_of([len(sg) for sg in segs]).tolist()
    # every tile holds the same entries as its globally sorted list
    g = oracle.schedule(depth, rect, tx, ty, K=K)
    for t in range(tx * ty):
        a = sorted(s["stream"][s["bin_offsets"][t * K]:s["bin_offsets"][t * K + K]].tolist())
        e = g["keys"][g["tile_offsets"][t]:g["tile_offsets"][t + 1]] & 0xFFFFFFFF
        ids = g["vals"][g["tile_offsets"][t]:g["tile_offsets"][t + 1]]
        assert a == sorted(((e.astype(np.uint64) << np.uint64(32)) | ids.astype(np.uint64)).tolist())


# ---------------------------------------------------------------------------
# compositing over a given order
# ---------------------------------------------------------------------------

def two_gaussians():
    # both means on the centre of pixel (3, 2) of an 8x8 image, so q = 0
    # there and alpha = min(0.99, opacity)
    return {"mean2d": np.array([[3.5, 2.5], [3.5, 2.5]]), "conic": np.array([[0.5, 0.0, 0.5]] * 2),
            "opacity": np.array([0.5, 0.8]), "rgb": np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]),
            "depth_key": np.array([1.0, 2.0], np.float32), "rect": np.array([[0, 0, 1, 1]] * 2, np.int32),
            "flags": np.array([1, 1], np.uint8)}


def test_render_stream_closed_form():
    p = two_gaussians()
    pix = np.array([[3, 2]], np.int32)
    fwd = oracle.render_stream(p, 8, 8, [0, 2], [0, 1], tile_size=16, pix=pix)
    rev = oracle.render_stream(p, 8, 8, [0, 2], [1, 0], tile_size=16, pix=pix)
    # front to back: C = a0 c0 + (1 - a0) a1 c1; alpha = 1 - (1 - a0)(1 - a1)
    np.testing.assert_allclose(fwd["rgb"][0], [0.5, 0.5 * 0.8, 0.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(rev["rgb"][0], [0.2 * 0.5, 0.8, 0.0], rtol=0, atol=1e-15)
    assert abs(fwd["alpha"][0] - 0.9) < 1e-15 and abs(rev["alpha"][0] - 0.9) < 1e-15
    assert fwd["last_gid"][0] == 1 and rev["last_gid"][0] == 0


def test_render_stream_in_depth_order_is_render():
    n, W, H = 300, 48, 40
    splats, info = scenes.random_splats(n, W, H, seed=5, max_sigma_px=6.0)
    proj = oracle.splats_to_proj(splats, info)
    tx, ty = 3, 3
    s = oracle.schedule(proj["depth_key"], proj["rect"], tx, ty, K=4)
    ref = oracle.render(proj, W, H)
    got = oracle.render_stream(proj, W, H, s["tile_offsets"], s["vals"])
    for k in ("rgb", "alpha", "last_gid", "ncontrib", "nvisit"):
        assert np.array_equal(ref[k], got[k]), k
