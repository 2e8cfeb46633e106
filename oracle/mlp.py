"""FP64 reference of the learned bin-count proposal: per-tile features, the
16-64-64-8 ReLU network, its expected-regret loss, the gradient and the
momentum SGD step.

TEST INFRASTRUCTURE ONLY: the test suite is the only caller. It shares no
code with the GPU library.

The paper fixes K = 64 bins per tile (section "Implementation details"; the
bin-count ablation table varies K per frame). The proposal network is an
addition that picks K_t per tile from the previous frame's per-tile depth
histogram and counts; exact repair keeps the image unchanged whatever it
picks, so only time is at stake.

Definitions (binary64 here):
  Features of tile t, from a frame's stream with K_t bins in tile t and
  segment lengths l_0 .. l_{K_t - 1}, n_t = sum l_b, M entries, T tiles:
    f0      log2(1 + n_t)
    f1..f8  8-cell depth histogram / max(n_t, 1): cell j collects bins b
            with floor(8 b / K_t) = j when K_t >= 8; a bin of a tile with
            K_t < 8 bins is spread evenly over its 8 / K_t cells
    f9      log2(1 + max_b l_b)
    f10     (number of non-empty bins) / K_t
    f11     log2(K_t) / 8
    f12     (sum of l_b over bins with l_b >= 2) / max(n_t, 1)
    f13     log2(1 + sum l_b^2 / max(n_t, 1))
    f14     log2(1 + M / T)
    f15     f0 - f14
  Network: h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), z = h2 W3 + b3,
  W1 [16, 64], W2 [64, 64], W3 [64, 8]; flat parameter vector in the order
  W1, b1, W2, b2, W3, b3 (row-major), 5768 values. Choice k -> K_t = 2^(k+1).
  Loss: L = (1/T) sum_t sum_k softmax(z_t)_k r_tk with r the per-tile
  regret of choice k (its cost minus the tile's best cost, in a common
  unit). Step: v <- mu v + g, w <- w - lr v.
"""
from __future__ import annotations

import numpy as np

SIZES = ((16, 64), (64, 64), (64, 8))
NUM_PARAMS = sum(a * b + b for a, b in SIZES)
CHOICES = 8


def unpack(w):
    w = np.asarray(w, np.float64)
    assert w.shape == (NUM_PARAMS,)
    out, o = [], 0
    for a, b in SIZES:
        W = w[o:o + a * b].reshape(a, b)
        o += a * b
        bb = w[o:o + b]
        o += b
        out.append((W, bb))
    return out


def forward(w, x):
    """Logits [T, 8] and the hidden activations."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(w)
    x = np.asarray(x, np.float64)
    a1 = x @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3 + b3
    return z, (x, a1, h1, a2, h2)


def softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss(w, x, regret):
    z, _ = forward(w, x)
    p = softmax(z)
    return float(np.mean(np.sum(p * regret, axis=1)))


def grad(w, x, regret):
    """dL/dw (flat), by the chain rule: dL/dz_tk = p_tk (r_tk - sum_j p_tj r_tj) / T."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(w)
    z, (x, a1, h1, a2, h2) = forward(w, x)
    T = z.shape[0]
    p = softmax(z)
    r = np.asarray(regret, np.float64)
    dz = p * (r - np.sum(p * r, axis=1, keepdims=True)) / T
    gW3 = h2.T @ dz
    gb3 = dz.sum(0)
    dh2 = dz @ W3.T
    da2 = dh2 * (a2 > 0)
    gW2 = h1.T @ da2
    gb2 = da2.sum(0)
    dh1 = da2 @ W2.T
    da1 = dh1 * (a1 > 0)
    gW1 = x.T @ da1
    gb1 = da1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def sgd_step(w, v, g, lr, mu):
    v = mu * np.asarray(v, np.float64) + np.asarray(g, np.float64)
    return np.asarray(w, np.float64) - lr * v, v


def choose_bins(w, x):
    """K_t = 2^(argmax_k z_tk + 1); the first maximum wins ties."""
    z, _ = forward(w, x)
    return (2 ** (np.argmax(z, axis=1) + 1)).astype(np.int32)


def tile_features(bin_offsets, seg_base, M):
    """Features [T, 16] of every tile from a frame's stream (seg_base [T + 1]
    first segment of each tile, bin_offsets [S + 1])."""
    seg_base = np.asarray(seg_base, np.int64)
    off = np.asarray(bin_offsets, np.int64)
    T = len(seg_base) - 1
    f = np.zeros((T, 16))
    dens = np.log2(1.0 + M / max(T, 1))
    for t in range(T):
        s0, s1 = seg_base[t], seg_base[t + 1]
        K = s1 - s0
        lens = (off[s0 + 1:s1 + 1] - off[s0:s1]).astype(np.float64)
        n = lens.sum()
        d = max(n, 1.0)
        hist = np.zeros(8)
        for b in range(K):
            if K >= 8:
                hist[(8 * b) // K] += lens[b]
            else:
                c = 8 // K
                hist[b * c:(b + 1) * c] += lens[b] / c
        f[t, 0] = np.log2(1.0 + n)
        f[t, 1:9] = hist / d
        f[t, 9] = np.log2(1.0 + lens.max()) if K else 0.0
        f[t, 10] = np.count_nonzero(lens) / K
        f[t, 11] = np.log2(K) / 8.0
        f[t, 12] = lens[lens >= 2].sum() / d
        f[t, 13] = np.log2(1.0 + (lens * lens).sum() / d)
        f[t, 14] = dens
        f[t, 15] = f[t, 0] - dens
    return f
