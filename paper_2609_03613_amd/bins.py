"""Learned per-tile bin counts: Python side of tgs_tile_features,
tgs_propose_bins and tgs_mlp_train_step (argument marshalling only), the
weight file, and the frame loop that feeds each frame's features to the
next frame's binning.

The network picks K_t in {2, 4, ..., 256} per tile from the previous
frame's stream; exact repair keeps the image unchanged, so a missing,
malformed or non-finite weight file falls back to the fixed K (64) and
changes only time.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from . import _lib as L
from .api import Params, Renderer, _ptr, _stream, project

WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "bin_mlp.npz")
MAX_BINS = 256
FALLBACK_BINS = 64


def load_weights(path=WEIGHTS_PATH):
    """The parameter vector (float32 [5768]) or None when the file is
    missing, malformed or not finite (the caller then uses the fixed K)."""
    try:
        with np.load(path, allow_pickle=False) as z:
            w = np.asarray(z["weights"], np.float32)
    except (OSError, KeyError, ValueError):
        return None
    if w.shape != (L.MLP_PARAMS,) or not np.all(np.isfinite(w)):
        return None
    return w


def save_weights(path, w, **meta):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, weights=np.asarray(w, np.float32), **{k: np.asarray(v) for k, v in meta.items()})


def tile_features(renderer, binned, out=None):
    """tgs_tile_features of a binned stream: [T, 16] float32."""
    if out is None:
        out = torch.empty((renderer.tiles, 16), dtype=torch.float32, device=renderer.device)
    L.check(L.lib().tgs_tile_features(ctypes.byref(binned.c()), ctypes.byref(renderer.ccam),
                                      ctypes.byref(renderer.cparams), _ptr(out), _stream()))
    return out


def propose_bins(weights, features, fallback=FALLBACK_BINS, out=None, logits=None):
    """tgs_propose_bins: per-tile bin counts int32 [T]."""
    T = int(features.shape[0])
    if out is None:
        out = torch.empty(T, dtype=torch.int32, device=features.device)
    L.check(L.lib().tgs_propose_bins(_ptr(weights), _ptr(features.contiguous()), T, int(fallback), _ptr(out),
                                     _ptr(logits), _stream()))
    return out


class Trainer:
    """Momentum SGD on the device (tgs_mlp_train_step)."""

    def __init__(self, weights, device="cuda"):
        self.w = torch.as_tensor(np.asarray(weights, np.float32)).to(device).contiguous()
        self.v = torch.zeros_like(self.w)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.ws = None
        self.device = device

    def step(self, features, regret, lr, momentum):
        T = int(features.shape[0])
        need = L.lib().tgs_mlp_train_workspace_size(T)
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        L.check(L.lib().tgs_mlp_train_step(_ptr(self.w), _ptr(self.v), _ptr(features.contiguous()),
                                           _ptr(regret.contiguous()), T, float(lr), float(momentum), _ptr(self.ws),
                                           self.ws.numel(), _ptr(self.loss), _stream()))
        return self.loss


def init_weights(seed=0):
    """He-style initialisation; the last layer starts at zero with the bias
    favouring K = 64 (choice 5), so an untrained network proposes the
    fixed K."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in ((16, 64), (64, 64), (64, 8)):
        W = rng.normal(0.0, np.sqrt(2.0 / a), size=(a, b)) if b != 8 else np.zeros((a, b))
        bb = np.zeros(b)
        if b == 8:
            bb[5] = 1.0
        parts += [W.ravel(), bb]
    return np.concatenate(parts).astype(np.float32)


class LearnedBins:
    """Frame loop with learned bin counts for one camera, judged against
    the fixed K at run time.

    Frame 1 uses the fixed K; a learned frame bins with the counts the
    network proposed from the previous frame's stream (features and
    proposal included in its cost). The judge times bin stages with HIP
    events on the launch stream, read back without waiting once they have
    completed. It alternates the two modes until each has `warm` timings
    (waiting for them once if the host has run ahead of the GPU) and keeps
    the faster by median; from then on every `probe_every`-th frame bins
    with the other mode and the frame after it with the kept one, both
    timed (the others are not), and the choice is revisited with each new
    pair, so a scene change can flip it. Without valid weights every frame
    uses the fixed K; with judge=False and weights, every frame after the
    first is learned. Exact repair keeps every image identical whichever
    mode bins it."""

    def __init__(self, cam, weights=None, device="cuda", tile_size=16, judge=True, warm=4, probe_every=64):
        self.weights = None if weights is None else torch.as_tensor(np.asarray(weights, np.float32)).to(device)
        self.fixed = Renderer(cam, Params(tile_size=tile_size, num_bins=FALLBACK_BINS), device=device)
        self.learned = Renderer(cam, Params(tile_size=tile_size, num_bins=MAX_BINS), device=device)
        self.kt = torch.full((self.fixed.tiles,), FALLBACK_BINS, dtype=torch.int32, device=device)
        self.learned.set_per_tile_bins(self.kt)
        self.feat = torch.empty((self.fixed.tiles, 16), dtype=torch.float32, device=device)
        self.prev = None  # (renderer, binned) of the previous frame
        self.judge = judge
        self.warm = int(warm)
        self.probe_every = max(2, int(probe_every))
        self.times = {"learned": [], "fixed": []}
        self.modes = []  # the mode of every frame
        self._pending = []
        self._best = None
        self._since = 0  # frames since the decision

    def _collect(self):
        keep, new = [], False
        for mode, e0, e1 in self._pending:
            if e1.query():
                self.times[mode].append(e0.elapsed_time(e1))
                new = True
            else:
                keep.append((mode, e0, e1))
        self._pending = keep
        if new:
            tl, tf = self.times["learned"], self.times["fixed"]
            if len(tl) >= self.warm and len(tf) >= self.warm:
                self._best = "learned" if np.median(tl[-self.warm:]) < np.median(tf[-self.warm:]) else "fixed"

    def choice(self):
        """The mode the judge currently prefers ("learned" or "fixed"), or
        None while it has fewer than `warm` timings of either."""
        return self._best

    def _mode(self):
        """(mode, timed) of the next frame."""
        if self.weights is None or self.prev is None:
            return "fixed", False
        if not self.judge:
            return "learned", False
        if self._pending:
            self._collect()
        if self._best is None:
            n_l = len(self.times["learned"]) + sum(m == "learned" for m, _, _ in self._pending)
            n_f = len(self.times["fixed"]) + sum(m == "fixed" for m, _, _ in self._pending)
            if min(n_l, n_f) >= self.warm:
                # both modes probed, timings still in flight (the host runs
                # ahead of the GPU): wait for them once, to decide
                for _, _, e1 in self._pending:
                    e1.synchronize()
                self._collect()
            if self._best is None:  # still probing: the mode with fewer timings
                return ("learned" if n_l <= n_f else "fixed"), True
        self._since += 1
        k = self._since % self.probe_every
        if k == 0:
            return ("fixed" if self._best == "learned" else "learned"), True
        return self._best, k == 1

    def bin(self, splats, info, sync=False):
        """Bins one frame (learned counts or the fixed K, as the judge
        decides); returns (renderer, binned)."""
        mode, timed = self._mode()
        if timed:
            stream = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        if mode == "learned":
            r0, b0 = self.prev
            tile_features(r0, b0, out=self.feat)
            propose_bins(self.weights, self.feat, out=self.kt)
            r, b = self.learned, self.learned.bin(splats, info, "binned", sync=sync)
        else:
            r, b = self.fixed, self.fixed.bin(splats, info, "binned", sync=sync)
        if timed:
            e1.record(stream)
            self._pending.append((mode, e0, e1))
        self.modes.append(mode)
        self.prev = (r, b)
        return r, b

    def render(self, g, bg=(0.0, 0.0, 0.0)):
        s, i = project(g, self.fixed.cam, self.fixed.params)
        r, b = self.bin(s, i, sync=True)
        return r.rasterize(s, i, b, bg=bg)
