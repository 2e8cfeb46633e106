"""Pins of the FP64 reference of the bin-count proposal network (oracle/mlp.py):
central finite differences of the loss, closed forms (constant logits, the
SGD step), the choice map, and the tile features written out by hand."""
import math

import numpy as np
import pytest

import scenes
from oracle import mlp
import oracle


def rand_case(T=24, seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    w = rng.normal(0.0, scale, size=mlp.NUM_PARAMS)
    x = rng.normal(0.0, 1.0, size=(T, 16))
    r = rng.uniform(0.0, 2.0, size=(T, 8))
    r -= r.min(axis=1, keepdims=True)
    return w, x, r


def test_num_params():
    assert mlp.NUM_PARAMS == 16 * 64 + 64 + 64 * 64 + 64 + 64 * 8 + 8 == 5768


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    w, x, r = rand_case(seed=seed)
    g = mlp.grad(w, x, r)
    L0 = mlp.loss(w, x, r)
    rng = np.random.default_rng(seed + 5)
    idx = rng.choice(mlp.NUM_PARAMS, size=600, replace=False)
    idx = np.concatenate([idx, np.arange(mlp.NUM_PARAMS - 8 - 64 * 8, mlp.NUM_PARAMS)])  # all of W3, b3
    gmax = np.abs(g).max()
    checked = 0
    for i in idx:
        h = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        Lp, Lm = mlp.loss(wp, x, r), mlp.loss(wm, x, r)
        if abs((Lp - L0) - (L0 - Lm)) / h > 1e-5 * gmax:  # a ReLU kink inside the stencil
            continue
        fd = (Lp - Lm) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * (abs(fd) + 1e-3 * gmax) + 5e-10, (i, g[i], fd)
        checked += 1
    assert checked >= 1000


def test_constant_logits_closed_form():
    _, x, r = rand_case(seed=3)
    w = np.zeros(mlp.NUM_PARAMS)
    b3 = np.array([0.5, -1.0, 2.0, 0.0, 0.3, -0.2, 1.1, 0.0])
    w[-8:] = b3
    p = np.exp(b3) / np.exp(b3).sum()
    assert mlp.loss(w, x, r) == pytest.approx(float(np.mean(r @ p)), rel=1e-13)
    # adding a constant to every logit changes nothing; the b3 gradient sums to 0
    w2 = w.copy()
    w2[-8:] += 7.0
    assert mlp.loss(w2, x, r) == pytest.approx(mlp.loss(w, x, r), rel=1e-13)
    assert abs(mlp.grad(w, x, r)[-8:].sum()) < 1e-15
    # and the b3 gradient is mean_t p_k (r_tk - p . r_t)
    want = np.mean(p * (r - (r @ p)[:, None]), axis=0)
    np.testing.assert_allclose(mlp.grad(w, x, r)[-8:], want, rtol=1e-12, atol=1e-15)


def test_sgd_step_closed_form():
    rng = np.random.default_rng(2)
    w, g1, g2 = rng.normal(size=(3, 10))
    v0 = np.zeros(10)
    w1, v1 = mlp.sgd_step(w, v0, g1, lr=0.1, mu=0.9)
    np.testing.assert_allclose(w1, w - 0.1 * g1)
    w2, v2 = mlp.sgd_step(w1, v1, g2, lr=0.1, mu=0.9)
    np.testing.assert_allclose(v2, 0.9 * g1 + g2)
    np.testing.assert_allclose(w2, w - 0.1 * g1 - 0.1 * (0.9 * g1 + g2))


def test_choice_map_and_ties():
    w = np.zeros(mlp.NUM_PARAMS)
    x = np.zeros((3, 16))
    assert mlp.choose_bins(w, x).tolist() == [2, 2, 2]  # all equal: the first wins
    w[-8:] = [0, 0, 0, 0, 0, 1, 0, 1]
    assert mlp.choose_bins(w, x).tolist() == [64, 64, 64]


def test_features_by_hand():
    # tile 0: K = 4, lengths [3, 0, 1, 2]; tile 1: K = 16, lengths 0..15;
    # tile 2: K = 2, empty
    lens = [[3, 0, 1, 2], list(range(16)), [0, 0]]
    seg_base = np.array([0, 4, 20, 22])
    off = np.concatenate([[0], np.cumsum(np.concatenate(lens))])
    M = int(off[-1])
    f = mlp.tile_features(off, seg_base, M)
    dens = math.log2(1 + M / 3)
    n0 = 6
    np.testing.assert_allclose(f[0, 1:9], np.array([1.5, 1.5, 0, 0, 0.5, 0.5, 1, 1]) / n0)
    assert f[0, 0] == pytest.approx(math.log2(7))
    assert f[0, 9] == pytest.approx(math.log2(4))
    assert f[0, 10] == pytest.approx(3 / 4)
    assert f[0, 11] == pytest.approx(2 / 8)
    assert f[0, 12] == pytest.approx(5 / 6)
    assert f[0, 13] == pytest.approx(math.log2(1 + 14 / 6))
    assert f[0, 14] == pytest.approx(dens) and f[0, 15] == pytest.approx(math.log2(7) - dens)
    n1 = sum(range(16))
    np.testing.assert_allclose(f[1, 1:9], np.array([2 * j + 2 * j + 1 for j in range(8)]) / n1)
    assert f[1, 10] == pytest.approx(15 / 16)
    assert f[2, 0] == 0 and not np.any(f[2, 1:10]) and f[2, 11] == pytest.approx(1 / 8)


def test_features_of_a_scene_schedule():
    g, cam = scenes.small_forward(seed=3, n=2000)
    p = oracle.project(g, cam)
    kt = (2 ** np.random.default_rng(0).integers(1, 9, size=64)).astype(np.int32)
    s = oracle.schedule_tiles(p["depth_key"], p["rect"], 8, 8, kt)
    f = mlp.tile_features(s["bin_offsets"], s["seg_base"], s["M"])
    counts = np.diff(s["bin_offsets"][s["seg_base"]])
    np.testing.assert_allclose(f[:, 0], np.log2(1 + counts))
    nz = counts > 0
    np.testing.assert_allclose(f[nz, 1:9].sum(1), 1.0, rtol=1e-12)
    np.testing.assert_allclose(f[:, 11], np.log2(kt) / 8)
