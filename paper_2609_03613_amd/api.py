"""Python entry points over the C ABI. PyTorch provides device memory and the
current HIP stream; every step of the path runs in the library's kernels.

Typical use::

    r = Renderer(camera_dict, params)
    out = r.render(gaussians, order="binned")   # dict of device tensors

``gaussians`` is a dict of CUDA tensors (means, log_scales, quats, logits, sh)
plus ``sh_degree``, in the layout of ``include/tilegs.h``.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L

ORDERS = {"global": L.ORDER_GLOBAL, "binned": L.ORDER_BINNED}
RASTERS = {"plain": L.RASTER_PLAIN, "wave": L.RASTER_WAVE}
REPAIRS = {"all": L.REPAIR_ALL, "rules": L.REPAIR_RULES, "none": L.REPAIR_NONE}
FOOTPRINTS = {"opacity": L.FOOTPRINT_OPACITY_AWARE, "three_sigma": L.FOOTPRINT_THREE_SIGMA}


@dataclass
class Params:
    """Ordering / raster options; defaults are the paper's (K = 64, 8192
    samples, 1st / 99th percentiles, 5 % pad, no per-entry geometry written
    before the raster) with the wave raster."""
    tile_size: int = 16
    num_bins: int = 64
    sample_count: int = 8192
    p_lo: float = 1.0
    p_hi: float = 99.0
    pad: float = 0.05
    raster: str = "wave"
    packed: int = 0          # 0: gather + cull in the raster, 1: records + masks, 2: masks only
    tile_order: bool = True
    per_tile_bins: object = None  # None, or a device int32 tensor [T]: bins per tile (num_bins = bound)
    repair: str = "all"      # "all" (exact), "rules" (the paper's selective repair), "none"
    repair_budget: float = 0.25
    near_shift: bool = False  # bin on z - min(alpha s_max, gamma z) instead of z
    shift_alpha: float = 1.0
    shift_gamma: float = 0.25
    split_entries: int = 2048  # tiles with this many entries take the quad walk, 16 wavefronts per tile (0: never)
    split_mean_factor: int = 2  # ... and this many times the mean of the non-empty tiles, when the longest reach twice that (0: no such bound)
    footprint: str = "opacity"  # tile rect rule: "opacity" (alpha-support box) or "three_sigma" (baseline square)
    sub_bins: int = 0  # exact repair: log-depth sub-bins per bin ordered by the binning (1, 2, 4, 8; 0: 8)

    def c(self):
        return L.Params(self.tile_size, self.num_bins, self.sample_count, self.p_lo, self.p_hi, self.pad,
                        RASTERS[self.raster], int(self.packed), _ptr(self.per_tile_bins).value,
                        REPAIRS[self.repair], float(self.repair_budget), int(bool(self.near_shift)),
                        float(self.shift_alpha), float(self.shift_gamma), int(self.split_entries),
                        int(self.split_mean_factor), FOOTPRINTS[self.footprint], int(self.sub_bins))


def paper_params(**kw):
    """The paper's selective mode: rule-based repair within a 25 % entry
    budget and bins on the near-depth key."""
    return Params(repair="rules", near_shift=True, **kw)


def camera_struct(cam):
    c = L.Camera()
    R = [float(v) for v in torch.as_tensor(cam["R"], dtype=torch.float64).reshape(9).tolist()]
    t = [float(v) for v in torch.as_tensor(cam["t"], dtype=torch.float64).reshape(3).tolist()]
    c.R = (ctypes.c_double * 9)(*R)
    c.t = (ctypes.c_double * 3)(*t)
    c.fx, c.fy, c.cx, c.cy = float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.znear, c.zfar = float(cam.get("znear", 0.01)), float(cam.get("zfar", 1e10))
    return c


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def to_device(g, device="cuda"):
    """numpy scene dict (scenes.py) -> dict of contiguous CUDA tensors."""
    out = {k: torch.as_tensor(v).to(device).contiguous() for k, v in g.items() if k != "sh_degree"}
    out["sh_degree"] = int(g["sh_degree"])
    return out


def project(g, cam, params=None, out=None):
    """tgs_project: returns (splats [n, 16] float32, info [n, 4] int32),
    written into ``out`` = (splats, info) when given."""
    params = params or Params()
    n = int(g["means"].shape[0])
    dev = g["means"].device
    if out is not None:
        splats, info = out
    else:
        splats = torch.empty((n, 16), dtype=torch.float32, device=dev)
        info = torch.empty((n, 4), dtype=torch.int32, device=dev)
    gs = L.Gaussians(_ptr(g["means"]).value, _ptr(g["log_scales"]).value, _ptr(g["quats"]).value,
                     _ptr(g["logits"]).value, _ptr(g["sh"]).value, n, int(g["sh_degree"]))
    pr = L.Projected(_ptr(splats).value, _ptr(info).value, n)
    L.check(L.lib().tgs_project(ctypes.byref(gs), ctypes.byref(camera_struct(cam)), ctypes.byref(params.c()),
                                ctypes.byref(pr), _stream()))
    return splats, info


def project_views(g, cams, params, outs):
    """tgs_project_views: the projections of g through every camera of cams
    (with params[v]) into outs[v] = (splats, info), each launch reading the
    Gaussians once for up to eight cameras."""
    nv = len(cams)
    n = int(g["means"].shape[0])
    gs = L.Gaussians(_ptr(g["means"]).value, _ptr(g["log_scales"]).value, _ptr(g["quats"]).value,
                     _ptr(g["logits"]).value, _ptr(g["sh"]).value, n, int(g["sh_degree"]))
    cc = (L.Camera * nv)(*[camera_struct(c) for c in cams])
    pp = (L.Params * nv)(*[p.c() for p in params])
    pr = (L.Projected * nv)(*[L.Projected(_ptr(s).value, _ptr(i).value, n) for s, i in outs])
    L.check(L.lib().tgs_project_views(ctypes.byref(gs), nv, ctypes.cast(cc, ctypes.c_void_p),
                                      ctypes.cast(pp, ctypes.c_void_p), ctypes.cast(pr, ctypes.c_void_p), _stream()))
    return outs


class Binned:
    """Device buffers of one entry stream (see tgs_binned)."""

    def __init__(self, order, capacity, tiles, num_bins, packed, device, tile_order=True, per_tile=False):
        self.order = ORDERS[order] if isinstance(order, str) else order
        self.capacity = int(capacity)
        cap = max(self.capacity, 1)
        kw = dict(device=device)
        self.counters = torch.zeros(4, dtype=torch.int64, **kw)
        self.zrange = torch.zeros(2, dtype=torch.float32, **kw)
        self.keys = self.vals = self.pairs = self.records = self.masks = None
        if self.order == L.ORDER_GLOBAL:
            self.keys = torch.empty(cap, dtype=torch.int64, **kw)
            self.vals = torch.empty(cap, dtype=torch.int32, **kw)
            self.offsets = torch.empty(tiles + 1, dtype=torch.int32, **kw)
        else:
            self.pairs = torch.empty(cap, dtype=torch.int64, **kw)
            self.offsets = torch.empty(tiles * num_bins + 1, dtype=torch.int32, **kw)
            if packed:
                self.masks = torch.empty(cap, dtype=torch.uint8, **kw)
            if packed == 1:
                self.records = torch.empty((cap, 12), dtype=torch.float32, **kw)
        self.tiles = int(tiles)
        self.tile_order = torch.empty(tiles + 2, dtype=torch.int32, **kw) if tile_order else None
        self.seg_base = torch.empty(tiles + 1, dtype=torch.int32, **kw) if per_tile else None
        self.repaired = (torch.empty(max(tiles * num_bins, 1), dtype=torch.uint8, **kw)
                         if self.order == L.ORDER_BINNED else None)
        self.num_entries = None

    def dispatch_order(self):
        """The tiles in dispatch order (device int32 [T]), or None."""
        return None if self.tile_order is None else self.tile_order[: self.tiles]

    def split(self):
        """(number of split tiles, their entry threshold) written by tgs_bin."""
        v = self.tile_order[self.tiles: self.tiles + 2].tolist()
        return int(v[0]), int(v[1])

    def c(self):
        return L.Binned(self.capacity, _ptr(self.keys).value, _ptr(self.vals).value, _ptr(self.pairs).value,
                        _ptr(self.offsets).value, _ptr(self.records).value, _ptr(self.masks).value,
                        _ptr(self.zrange).value,
                        _ptr(self.counters).value, _ptr(self.tile_order).value, _ptr(self.seg_base).value,
                        _ptr(self.repaired).value)


class Renderer:
    """Holds a camera, options, workspace and entry buffers (grown on demand)."""

    def __init__(self, cam, params=None, device="cuda"):
        self.cam = cam
        self.params = params or Params()
        self.ccam = camera_struct(cam)
        self.cparams = self.params.c()
        self.device = device
        ts = int(self.params.tile_size)
        self.tiles_x = (int(cam["width"]) + ts - 1) // ts
        self.tiles_y = (int(cam["height"]) + ts - 1) // ts
        self.tiles = self.tiles_x * self.tiles_y
        self._binned = {}
        self._ws = {}

    def set_per_tile_bins(self, kt):
        """Per-tile bin counts for the next tgs_bin calls (device int32 [T],
        or None for params.num_bins everywhere)."""
        self.params.per_tile_bins = kt
        self.cparams = self.params.c()

    def _new_binned(self, o, capacity):
        return Binned(o, capacity, self.tiles, self.params.num_bins, self.params.packed, self.device,
                      self.params.tile_order, per_tile=self.params.per_tile_bins is not None)

    def _workspace(self, order, n, capacity):
        need = L.lib().tgs_bin_workspace_size(n, capacity, ctypes.byref(self.ccam), ctypes.byref(self.cparams),
                                              order)
        ws = self._ws.get(order)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
            self._ws[order] = ws
        return ws

    def bin(self, splats, info, order="binned", capacity=None, sync=True, fresh=False):
        """tgs_bin. With sync, the entry count is read back and the buffers are
        grown (and the call repeated) when it exceeds their capacity. With
        fresh, new entry buffers are allocated (a stream that must outlive
        the next call, e.g. one a backward pass will read)."""
        o = ORDERS[order] if isinstance(order, str) else order
        n = int(splats.shape[0])
        pr = L.Projected(_ptr(splats).value, _ptr(info).value, n)
        b = self._binned.get(o)
        if fresh and b is not None:
            capacity = max(capacity or 0, b.capacity)
            b = None
        if b is not None and (b.seg_base is None) != (self.params.per_tile_bins is None):
            capacity = max(capacity or 0, b.capacity)
            b = None
        if b is None or (capacity is not None and b.capacity < capacity):
            b = self._new_binned(o, capacity if capacity is not None else max(1024, 4 * n))
            self._binned[o] = b
        for _ in range(2):
            ws = self._workspace(o, n, b.capacity)
            m = ctypes.c_int64(-1)
            st = L.lib().tgs_bin(ctypes.byref(pr), ctypes.byref(self.ccam), ctypes.byref(self.cparams), o,
                                 _ptr(ws), ws.numel(), ctypes.byref(b.c()),
                                 ctypes.byref(m) if sync else None, _stream())
            if st == L.TGS_ERR_CAPACITY:
                b = self._new_binned(o, int(m.value * 1.1) + 1024)
                self._binned[o] = b
                continue
            L.check(st)
            b.num_entries = int(m.value) if sync else None
            return b
        raise L.TileGSError(L.TGS_ERR_CAPACITY, "capacity still exceeded after growing")

    def rasterize(self, splats, info, binned, bg=(0.0, 0.0, 0.0), counts=False, out=None, trans=False):
        """tgs_rasterize: dict with rgb [H, W, 3], alpha [H, W], last [H, W]
        (and n_contrib, n_visit, n_support when counts; the final
        transmittance `trans` [H, W] when trans)."""
        H, W = int(self.cam["height"]), int(self.cam["width"])
        if out is None:
            out = {
                "rgb": torch.empty((H, W, 3), dtype=torch.float32, device=self.device),
                "alpha": torch.empty((H, W), dtype=torch.float32, device=self.device),
                "last": torch.empty((H, W), dtype=torch.int32, device=self.device),
            }
            if counts:
                out["n_contrib"] = torch.empty((H, W), dtype=torch.int32, device=self.device)
                out["n_visit"] = torch.empty((H, W), dtype=torch.int32, device=self.device)
                out["n_support"] = torch.empty((H, W), dtype=torch.int32, device=self.device)
            if trans:
                out["trans"] = torch.empty((H, W), dtype=torch.float32, device=self.device)
        n = int(splats.shape[0])
        pr = L.Projected(_ptr(splats).value, _ptr(info).value, n)
        bgc = (ctypes.c_float * 3)(*[float(v) for v in bg])
        L.check(L.lib().tgs_rasterize(ctypes.byref(pr), ctypes.byref(binned.c()), ctypes.byref(self.ccam),
                                      ctypes.byref(self.cparams), binned.order, bgc, _ptr(out["rgb"]),
                                      _ptr(out["alpha"]), _ptr(out["last"]), _ptr(out.get("n_contrib")),
                                      _ptr(out.get("n_visit")), _ptr(out.get("n_support")), _ptr(out.get("trans")),
                                      _stream()))
        return out

    def rasterize_backward(self, splats, info, binned, d_rgb, d_alpha=None, bg=(0.0, 0.0, 0.0), out=None,
                           saved=None):
        """tgs_rasterize_backward: gradient lines [n, 12] (dL/d mean_x, mean_y,
        conic a, b, c, opacity, r, g, b, 0, 0, 0) from dL/d rgb [H, W, 3] and
        dL/d alpha [H, W] (None = zero). saved: the forward's output dict
        with "trans" and "last" (skips the recomputed forward walk)."""
        n = int(splats.shape[0])
        if out is None:
            out = torch.empty((n, L.GRAD_WORDS), dtype=torch.float32, device=self.device)
        d_rgb = d_rgb.contiguous().float()
        d_alpha = None if d_alpha is None else d_alpha.contiguous().float()
        pr = L.Projected(_ptr(splats).value, _ptr(info).value, n)
        bgc = (ctypes.c_float * 3)(*[float(v) for v in bg])
        tr = None if saved is None else saved["trans"]
        la = None if saved is None else saved["last"]
        L.check(L.lib().tgs_rasterize_backward(ctypes.byref(pr), ctypes.byref(binned.c()), ctypes.byref(self.ccam),
                                               ctypes.byref(self.cparams), binned.order, bgc, _ptr(d_rgb),
                                               _ptr(d_alpha), _ptr(tr), _ptr(la), _ptr(out), _stream()))
        return out

    def render(self, g, order="binned", bg=(0.0, 0.0, 0.0), counts=False):
        splats, info = project(g, self.cam, self.params)
        b = self.bin(splats, info, order)
        out = self.rasterize(splats, info, b, bg=bg, counts=counts)
        out["splats"], out["info"], out["binned"] = splats, info, b
        return out


def render(g, cam, params=None, order="binned", bg=(0.0, 0.0, 0.0), counts=False):
    return Renderer(cam, params, device=g["means"].device).render(g, order=order, bg=bg, counts=counts)


def _gaussians_struct(g):
    n = int(g["means"].shape[0])
    return L.Gaussians(_ptr(g["means"]).value, _ptr(g["log_scales"]).value, _ptr(g["quats"]).value,
                       _ptr(g["logits"]).value, _ptr(g["sh"]).value, n, int(g["sh_degree"]))


def project_backward(g, cam, d_splats):
    """tgs_project_backward: dict of parameter gradients (same shapes as
    ``g``'s tensors) from the gradient lines [n, 12]."""
    gr = {k: torch.empty_like(g[k]) for k in ("means", "log_scales", "quats", "logits", "sh")}
    out = L.GaussianGrads(_ptr(gr["means"]).value, _ptr(gr["log_scales"]).value, _ptr(gr["quats"]).value,
                          _ptr(gr["logits"]).value, _ptr(gr["sh"]).value)
    L.check(L.lib().tgs_project_backward(ctypes.byref(_gaussians_struct(g)), ctypes.byref(camera_struct(cam)),
                                         _ptr(d_splats.contiguous()), ctypes.byref(out), _stream()))
    return gr


class _RenderFn(torch.autograd.Function):
    """Image (rgb, alpha) of the Gaussian parameters; backward through
    tgs_rasterize_backward and tgs_project_backward."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, logits, sh, renderer, sh_degree, order, bg):
        g = {"means": means.contiguous(), "log_scales": log_scales.contiguous(), "quats": quats.contiguous(),
             "logits": logits.contiguous(), "sh": sh.contiguous(), "sh_degree": int(sh_degree)}
        splats, info = project(g, renderer.cam, renderer.params)
        binned = renderer.bin(splats, info, order, fresh=True)
        wave = renderer.params.raster == "wave"
        out = renderer.rasterize(splats, info, binned, bg=bg, trans=wave)
        ctx.renderer, ctx.binned, ctx.bg, ctx.g = renderer, binned, bg, g
        ctx.saved = {"trans": out["trans"], "last": out["last"]} if wave else None
        ctx.save_for_backward(splats, info)
        return out["rgb"], out["alpha"]

    @staticmethod
    def backward(ctx, d_rgb, d_alpha):
        splats, info = ctx.saved_tensors
        r = ctx.renderer
        if d_rgb is None:
            d_rgb = torch.zeros((int(r.cam["height"]), int(r.cam["width"]), 3), device=splats.device)
        d_splats = r.rasterize_backward(splats, info, ctx.binned, d_rgb, d_alpha, bg=ctx.bg, saved=ctx.saved)
        gr = project_backward(ctx.g, r.cam, d_splats)
        return gr["means"], gr["log_scales"], gr["quats"], gr["logits"], gr["sh"], None, None, None, None


def render_differentiable(renderer, g, order="binned", bg=(0.0, 0.0, 0.0)):
    """(rgb [H, W, 3], alpha [H, W]) as differentiable functions of g's
    means, log_scales, quats, logits and sh tensors."""
    return _RenderFn.apply(g["means"], g["log_scales"], g["quats"], g["logits"], g["sh"], renderer,
                           int(g["sh_degree"]), order, tuple(float(v) for v in bg))


class BatchRenderer:
    """Several cameras per frame: tgs_project_views for all views (the
    Gaussians read once per eight views), per-view tgs_bin (BINNED, each view
    with its own params: tile size, bins; up to ``lanes`` views at once on
    side streams), then one tgs_rasterize_batch persistent launch for all
    views. ``capture`` records
    the whole frame in a HIP graph (torch.cuda.CUDAGraph) after an eager
    frame has sized every buffer; ``replay`` launches it."""

    def __init__(self, cams, params=None, device="cuda", bg=(0.0, 0.0, 0.0), lanes=4):
        if len(cams) > L.MAX_VIEWS:
            raise ValueError(f"at most {L.MAX_VIEWS} views per batch")
        # per-view binnings run on this many streams at once (default
        # priority), forked from and joined back into the caller's stream
        self.lanes = max(1, int(lanes))
        self._side = None
        params = params or [Params() for _ in cams]
        self.views = [Renderer(c, p, device=device) for c, p in zip(cams, params)]
        self.device = device
        self.bg = tuple(float(v) for v in bg)
        self.outs = []
        for c in cams:
            H, W = int(c["height"]), int(c["width"])
            self.outs.append({"rgb": torch.empty((H, W, 3), dtype=torch.float32, device=device),
                              "alpha": torch.empty((H, W), dtype=torch.float32, device=device),
                              "last": torch.empty((H, W), dtype=torch.int32, device=device)})
        nv = len(cams)
        self._ccams = (L.Camera * nv)(*[r.ccam for r in self.views])
        self._cparams = (L.Params * nv)(*[r.cparams for r in self.views])
        need = L.lib().tgs_batch_workspace_size(nv, ctypes.cast(self._ccams, ctypes.c_void_p),
                                                ctypes.cast(self._cparams, ctypes.c_void_p))
        if need == 0:
            raise L.TileGSError(L.TGS_ERR_INVALID_ARG, "invalid batch cameras or params")
        self.ws = torch.empty(need, dtype=torch.uint8, device=device)
        self.proj = None
        self.binned = None
        self.entries = None
        self.graph = None

    def _alloc_proj(self, n):
        if self.proj is None or int(self.proj[0][0].shape[0]) != n:
            self.proj = [(torch.empty((n, 16), dtype=torch.float32, device=self.device),
                          torch.empty((n, 4), dtype=torch.int32, device=self.device)) for _ in self.views]

    def rasterize(self, projs, binned, noalloc=False):
        """tgs_rasterize_batch over (splats, info) and Binned per view (with
        noalloc, tgs_rasterize_batch_noalloc: the library's fixed scratch
        instead of the workspace)."""
        nv = len(self.views)
        prs = (L.Projected * nv)(*[L.Projected(_ptr(s).value, _ptr(i).value, int(s.shape[0])) for s, i in projs])
        bs = (L.Binned * nv)(*[b.c() for b in binned])
        orders = (ctypes.c_int32 * nv)(*[b.order for b in binned])
        self._cparams = (L.Params * nv)(*[r.cparams for r in self.views])
        bgc = (ctypes.c_float * 3)(*self.bg)
        ptrs = lambda k: (ctypes.c_void_p * nv)(*[o[k].data_ptr() for o in self.outs])
        self._keep = (prs, bs, orders, bgc)
        args = (nv, ctypes.cast(prs, ctypes.c_void_p), ctypes.cast(bs, ctypes.c_void_p),
                ctypes.cast(self._ccams, ctypes.c_void_p), ctypes.cast(self._cparams, ctypes.c_void_p),
                ctypes.cast(orders, ctypes.c_void_p), bgc, ptrs("rgb"), ptrs("alpha"), ptrs("last"))
        if noalloc:
            L.check(L.lib().tgs_rasterize_batch_noalloc(*args, _stream()))
        else:
            L.check(L.lib().tgs_rasterize_batch(*args, _ptr(self.ws), self.ws.numel(), _stream()))
        return self.outs

    def frame(self, g, sync=False):
        """One eager frame: project and bin every view, one batched raster.
        With sync, entry counts are read back and buffers grown as needed
        (do this once before capture)."""
        self._alloc_proj(int(g["means"].shape[0]))
        project_views(g, [r.cam for r in self.views], [r.params for r in self.views], self.proj)
        if sync or self.lanes == 1 or len(self.views) == 1:
            binned = [r.bin(s, i, "binned", sync=sync) for r, (s, i) in zip(self.views, self.proj)]
        else:
            # every view has its own buffers (sized by a sync frame), so the
            # binnings of different views may overlap
            main = torch.cuda.current_stream()
            if self._side is None:
                self._side = [torch.cuda.Stream(device=self.device) for _ in range(self.lanes)]
            for st in self._side:
                st.wait_stream(main)
            binned = [None] * len(self.views)
            for v, lane in self._lane_of():
                r, (sp, ip) = self.views[v], self.proj[v]
                with torch.cuda.stream(self._side[lane]):
                    binned[v] = r.bin(sp, ip, "binned", sync=False)
            for st in self._side:
                main.wait_stream(st)
        self.binned = binned
        if sync:
            self.entries = [b.num_entries for b in binned]
        return self.rasterize(self.proj, binned)

    def _lane_of(self):
        """(view, stream) pairs: the views by decreasing entry count (pixels
        before the first sized frame), each to the least loaded stream."""
        load = [0] * self.lanes
        sizes = self.entries or [int(r.cam["width"]) * int(r.cam["height"]) for r in self.views]
        out = []
        for v in sorted(range(len(self.views)), key=lambda k: -sizes[k]):
            lane = min(range(self.lanes), key=lambda k: load[k])
            load[lane] += sizes[v]
            out.append((v, lane))
        return out

    def overflowed(self):
        return any(int(b.counters[2].item()) != 0 for b in self.binned)

    def capture(self, g):
        """Sizes the buffers with an eager frame and records one frame in a
        HIP graph (projection, binning and the batched raster of every
        view)."""
        self.frame(g, sync=True)
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.frame(g, sync=False)  # warm-up on the capture stream
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.frame(g, sync=False)
        return self.graph

    def replay(self):
        self.graph.replay()
        return self.outs
