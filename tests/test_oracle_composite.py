"""Pins of the oracle's compositing (the per-pixel definition of the image).

Closed forms (one Gaussian, a stack of identical layers, two ordered layers,
the 0.99 clamp and the 1/255 cut), invariants (transmittance bound, colour
bound, permutation invariance) and brute force (every Gaussian sorted per
pixel) against the tiled traversal.
"""
import math

import numpy as np
import pytest

import oracle
import scenes


def records(mean2d, conic, opacity, rgb, depth, rect):
    n = len(opacity)
    return {
        "mean2d": np.asarray(mean2d, np.float64).reshape(n, 2),
        "conic": np.asarray(conic, np.float64).reshape(n, 3),
        "opacity": np.asarray(opacity, np.float64),
        "rgb": np.asarray(rgb, np.float64).reshape(n, 3),
        "depth_key": np.asarray(depth, np.float32),
        "rect": np.asarray(rect, np.int32).reshape(n, 4),
        "flags": np.ones(n, np.uint8),
    }


def test_single_isotropic_gaussian_image():
    # image = min(0.99, o exp(-r^2 / (2 s^2))) * c where that is >= 1/255, else 0
    W = H = 48
    s2, o, c = 9.0, 0.8, np.array([0.2, 0.7, 1.3])
    m = (20.3, 26.6)
    rec = records([m], [1 / s2, 0, 1 / s2], [o], [c], [5.0], [[0, 0, 3, 3]])
    out = oracle.render(rec, W, H)
    ys, xs = np.mgrid[0:H, 0:W] + 0.5
    a = np.minimum(0.99, o * np.exp(-0.5 * ((xs - m[0]) ** 2 + (ys - m[1]) ** 2) / s2))
    a = np.where(a >= 1 / 255, a, 0.0)
    np.testing.assert_allclose(out["rgb"], a[..., None] * c, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(out["alpha"], a, rtol=1e-13, atol=1e-15)
    assert np.array_equal(out["ncontrib"], (a > 0).astype(np.int32))


def test_stack_of_half_opaque_layers_stops_after_13():
    # 20 layers with alpha exactly 0.5 at the pixel centre: after k layers
    # T = 2^-k; the 14th would give 2^-14 < 1e-4 <= 2^-13, so exactly 13
    # layers are composited and rgb = c (1 - 2^-13).
    n = 20
    c = np.array([0.9, 0.4, 0.1])
    px = (8.5, 8.5)
    depth = np.linspace(1.0, 3.0, n)[::-1]  # reversed: gid order != depth order
    rec = records([px] * n, [[0.5, 0.0, 0.5]] * n, [0.5] * n, [c] * n, depth, [[0, 0, 1, 1]] * n)
    out = oracle.render(rec, 16, 16, pix=[[8, 8]])
    np.testing.assert_allclose(out["rgb"][0], c * (1 - 2.0 ** -13), rtol=1e-14)
    assert out["alpha"][0] == pytest.approx(1 - 2.0 ** -13, rel=1e-14)
    assert out["ncontrib"][0] == 13
    # the 13th nearest layer is the last composited one
    assert out["last_gid"][0] == np.argsort(depth)[12]
    assert out["nvisit"][0] == 14 and out["nsupport"][0] == 14


@pytest.mark.parametrize("swap", [False, True])
def test_two_layers_in_depth_order(swap):
    # C = a1 c1 + (1 - a1) a2 c2 with layer 1 in front
    a1, a2 = 0.6, 0.7
    c1, c2 = np.array([1.0, 0.0, 0.2]), np.array([0.0, 1.0, 0.4])
    d = [2.0, 3.0] if not swap else [3.0, 2.0]
    rec = records([(4.5, 4.5)] * 2, [[0.1, 0, 0.1]] * 2, [a1, a2], [c1, c2], d, [[0, 0, 1, 1]] * 2)
    out = oracle.render(rec, 8, 8, pix=[[4, 4]])
    if not swap:
        expect = a1 * c1 + (1 - a1) * a2 * c2
    else:
        expect = a2 * c2 + (1 - a2) * a1 * c1
    np.testing.assert_allclose(out["rgb"][0], expect, rtol=1e-14)


def test_equal_depths_break_ties_by_id():
    a1, a2 = 0.6, 0.7
    c1, c2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    rec = records([(4.5, 4.5)] * 2, [[0.1, 0, 0.1]] * 2, [a1, a2], [c1, c2], [2.0, 2.0], [[0, 0, 1, 1]] * 2)
    out = oracle.render(rec, 8, 8, pix=[[4, 4]])
    np.testing.assert_allclose(out["rgb"][0], a1 * c1 + (1 - a1) * a2 * c2, rtol=1e-14)


def test_alpha_clamp_and_cut():
    c = np.array([0.5, 0.25, 1.0])
    full = records([(4.5, 4.5)], [[0.1, 0, 0.1]], [1.0], [c], [2.0], [[0, 0, 1, 1]])
    out = oracle.render(full, 8, 8, pix=[[4, 4]])
    np.testing.assert_allclose(out["rgb"][0], 0.99 * c, rtol=1e-15)
    lo = records([(4.5, 4.5)], [[0.1, 0, 0.1]], [(1 / 255) * (1 - 1e-9)], [c], [2.0], [[0, 0, 1, 1]])
    assert np.all(oracle.render(lo, 8, 8, pix=[[4, 4]])["rgb"][0] == 0)
    hi = records([(4.5, 4.5)], [[0.1, 0, 0.1]], [(1 / 255) * (1 + 1e-9)], [c], [2.0], [[0, 0, 1, 1]])
    np.testing.assert_allclose(oracle.render(hi, 8, 8, pix=[[4, 4]])["rgb"][0], c / 255 * (1 + 1e-9), rtol=1e-14)


def test_background_is_added_with_transmittance():
    c = np.array([0.5, 0.25, 1.0])
    bg = np.array([0.1, 0.2, 0.3])
    rec = records([(4.5, 4.5)], [[0.1, 0, 0.1]], [0.4], [c], [2.0], [[0, 0, 1, 1]])
    out = oracle.render(rec, 8, 8, pix=[[4, 4], [0, 7]], bg=bg)
    np.testing.assert_allclose(out["rgb"][0], 0.4 * c + 0.6 * bg, rtol=1e-14)
    a = 0.4 * math.exp(-0.5 * 0.1 * (4.0 ** 2 + 3.0 ** 2))
    np.testing.assert_allclose(out["rgb"][1], a * c + (1 - a) * bg, rtol=1e-13)


def small_scene(seed, n=2000):
    g, cam = scenes.small_forward(seed=seed, n=n)
    return oracle.project(g, cam), cam


@pytest.mark.parametrize("seed", [0, 1])
def test_tiled_equals_brute_force(seed):
    p, cam = small_scene(seed)
    t = oracle.render(p, 128, 128, mode="tiled")
    b = oracle.render(p, 128, 128, mode="brute")
    np.testing.assert_array_equal(t["rgb"], b["rgb"])
    np.testing.assert_array_equal(t["last_gid"], b["last_gid"])
    np.testing.assert_array_equal(t["ncontrib"], b["ncontrib"])


def test_tiled_equals_brute_force_large_splats():
    # bigger, overlapping splats: many tiles per splat and early termination
    g, cam = scenes.small_forward(seed=2, n=400)
    g["log_scales"] = (g["log_scales"] + 2.5).astype(np.float32)
    g["logits"] = (g["logits"] + 2.0).astype(np.float32)
    p = oracle.project(g, cam)
    t = oracle.render(p, 128, 128)
    b = oracle.render(p, 128, 128, mode="brute")
    assert (t["alpha"] > 0.999).mean() > 0.05  # some pixels terminate
    np.testing.assert_array_equal(t["rgb"], b["rgb"])
    np.testing.assert_array_equal(t["last_gid"], b["last_gid"])


def test_transmittance_and_colour_bounds():
    g, cam = scenes.small_forward(seed=3, n=1500)
    g["log_scales"] = (g["log_scales"] + 2.0).astype(np.float32)
    p = oracle.project(g, cam)
    out = oracle.render(p, 128, 128)
    T = 1 - out["alpha"]
    assert T.min() >= 1e-4
    cmax = p["rgb"].max()
    assert np.all(out["rgb"] >= 0)
    assert np.all(out["rgb"] <= out["alpha"][..., None] * cmax + 1e-12)
    assert np.all(out["nsupport"] >= out["ncontrib"])
    assert np.all(out["nvisit"] >= out["nsupport"])


def test_permutation_invariance():
    g, cam = scenes.small_forward(seed=6, n=800)
    perm = np.random.default_rng(0).permutation(800)
    p = oracle.project(g, cam)
    q = oracle.project(scenes.subset(g, perm), cam)
    assert len(np.unique(p["depth_key"][(p["flags"] & 1) > 0])) == ((p["flags"] & 1) > 0).sum()
    a, b = oracle.render(p, 128, 128), oracle.render(q, 128, 128)
    np.testing.assert_array_equal(a["rgb"], b["rgb"])
    has = a["last_gid"] >= 0
    np.testing.assert_array_equal(a["last_gid"][has], perm[b["last_gid"][has]])


def test_last_position_matches_global_list():
    p, cam = small_scene(0)
    out = oracle.render(p, 128, 128)
    s = oracle.schedule(p["depth_key"], p["rect"], 8, 8)
    has = out["last_pos"] >= 0
    assert has.sum() > 1000
    np.testing.assert_array_equal(s["vals"][out["last_pos"][has]], out["last_gid"][has])
