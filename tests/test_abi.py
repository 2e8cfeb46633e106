"""The C ABI on the host: the library loads, exports every symbol the header
declares, and rejects bad arguments before launching anything (these calls
never reach the GPU)."""
import ctypes
import os
import re

import pytest

import paper_2609_03613_amd as tg
from paper_2609_03613_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "tilegs.h")).read()
    return sorted(set(re.findall(r"TGS_API\s+[\w\s\*]+?\b(tgs_\w+)\s*\(", text)))


def test_exports_match_header():
    names = header_functions()
    assert names == sorted(L.EXPORTS)
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_default_params():
    p = L.Params()
    L.lib().tgs_default_params(ctypes.byref(p))
    assert (p.tile_size, p.num_bins, p.sample_count) == (16, 64, 8192)
    assert (p.p_lo, p.p_hi) == (1.0, 99.0) and abs(p.pad - 0.05) < 1e-7
    assert p.raster == L.RASTER_WAVE and p.packed == 0
    assert p.footprint == L.FOOTPRINT_OPACITY_AWARE and (p.split_entries, p.split_mean_factor) == (2048, 2)
    assert p.sub_bins == 0
    # the binding's defaults are the library's
    q = tg.Params().c()
    for name, _ in L.Params._fields_:
        assert getattr(q, name) == getattr(p, name) or name in ("p_lo", "p_hi", "pad", "repair_budget",
                                                               "shift_alpha", "shift_gamma"), name


def cam(w=64, h=48):
    return tg.camera_struct({"R": [1, 0, 0, 0, 1, 0, 0, 0, 1], "t": [0, 0, 0], "fx": 50.0, "fy": 50.0,
                             "cx": w / 2, "cy": h / 2, "width": w, "height": h})


def status_of(fn, *args):
    return fn(*args), L.lib().tgs_last_error().decode()


def test_project_argument_errors():
    lib = L.lib()
    p = tg.Params().c()
    out = L.Projected(None, None, 0)
    g = L.Gaussians(None, None, None, None, None, 0, 5)
    st, msg = status_of(lib.tgs_project, ctypes.byref(g), ctypes.byref(cam()), ctypes.byref(p), ctypes.byref(out), None)
    assert st == L.TGS_ERR_INVALID_ARG and "sh_degree" in msg
    g = L.Gaussians(None, None, None, None, None, 10, 0)
    st, msg = status_of(lib.tgs_project, ctypes.byref(g), ctypes.byref(cam()), ctypes.byref(p), ctypes.byref(out), None)
    assert st == L.TGS_ERR_INVALID_ARG and "NULL" in msg
    bad = cam(0, 10)
    g = L.Gaussians(None, None, None, None, None, 0, 0)
    st, msg = status_of(lib.tgs_project, ctypes.byref(g), ctypes.byref(bad), ctypes.byref(p), ctypes.byref(out), None)
    assert st == L.TGS_ERR_INVALID_ARG and "image size" in msg
    c = cam()
    c.znear = 2.0
    c.zfar = 1.0
    st, msg = status_of(lib.tgs_project, ctypes.byref(g), ctypes.byref(c), ctypes.byref(p), ctypes.byref(out), None)
    assert st == L.TGS_ERR_INVALID_ARG and "znear" in msg
    for bad_p in (tg.Params(tile_size=12), tg.Params(tile_size=8, raster="plain"), tg.Params(tile_size=32, packed=1)):
        st, msg = status_of(lib.tgs_project, ctypes.byref(g), ctypes.byref(cam()), ctypes.byref(bad_p.c()),
                            ctypes.byref(out), None)
        assert st == L.TGS_ERR_UNSUPPORTED and "tile_size" in msg
    for ts in (8, 16, 32):
        assert lib.tgs_bin_workspace_size(100, 1000, ctypes.byref(cam()), ctypes.byref(tg.Params(tile_size=ts).c()),
                                          L.ORDER_BINNED) > 0


def test_bin_workspace_and_argument_errors():
    lib = L.lib()
    c = cam()
    p = tg.Params().c()
    need = lib.tgs_bin_workspace_size(1000, 5000, ctypes.byref(c), ctypes.byref(p), L.ORDER_BINNED)
    assert need >= 5000 * 4 + 12 * 64 * 4
    need_g = lib.tgs_bin_workspace_size(1000, 5000, ctypes.byref(c), ctypes.byref(p), L.ORDER_GLOBAL)
    assert need_g >= 5000 * 12
    pr = L.Projected(None, None, 0)
    need = lib.tgs_bin_workspace_size(0, 5000, ctypes.byref(c), ctypes.byref(p), L.ORDER_BINNED)
    fake = ctypes.c_void_p(0x1000)
    b = L.Binned(5000, None, None, fake.value, fake.value, fake.value, fake.value, fake.value, fake.value)
    st, msg = status_of(lib.tgs_bin, ctypes.byref(pr), ctypes.byref(c), ctypes.byref(p), L.ORDER_BINNED, fake,
                        need - 1, ctypes.byref(b), None, None)
    assert st == L.TGS_ERR_WORKSPACE and "workspace" in msg
    # a workspace that is large enough but not 256-byte aligned
    st, msg = status_of(lib.tgs_bin, ctypes.byref(pr), ctypes.byref(c), ctypes.byref(p), L.ORDER_BINNED,
                        ctypes.c_void_p(0x1010), need, ctypes.byref(b), None, None)
    assert st == L.TGS_ERR_WORKSPACE and "aligned" in msg
    # the remaining cases pass no workspace, so that even a validation bug
    # stops at the workspace check instead of launching anything
    st, _ = status_of(lib.tgs_bin, ctypes.byref(pr), ctypes.byref(c), ctypes.byref(p), 7, None, 0,
                      ctypes.byref(b), None, None)
    assert st == L.TGS_ERR_INVALID_ARG
    pk = tg.Params(num_bins=0).c()
    st, _ = status_of(lib.tgs_bin, ctypes.byref(pr), ctypes.byref(c), ctypes.byref(pk), L.ORDER_BINNED, None, 0,
                      ctypes.byref(b), None, None)
    assert st == L.TGS_ERR_INVALID_ARG
    b.masks = None
    p2 = tg.Params(packed=2).c()
    st, msg = status_of(lib.tgs_bin, ctypes.byref(pr), ctypes.byref(c), ctypes.byref(p2), L.ORDER_BINNED, None, 0,
                        ctypes.byref(b), None, None)
    assert st == L.TGS_ERR_INVALID_ARG and "masks" in msg
    p1 = tg.Params(packed=1).c()
    b.masks = fake.value
    b.records = None
    st, msg = status_of(lib.tgs_bin, ctypes.byref(pr), ctypes.byref(c), ctypes.byref(p1), L.ORDER_BINNED, None, 0,
                        ctypes.byref(b), None, None)
    assert st == L.TGS_ERR_INVALID_ARG and "records" in msg
    p3 = tg.Params(packed=3).c()
    st, msg = status_of(lib.tgs_bin, ctypes.byref(pr), ctypes.byref(c), ctypes.byref(p3), L.ORDER_BINNED, None, 0,
                        ctypes.byref(b), None, None)
    assert st == L.TGS_ERR_INVALID_ARG and "packed" in msg


def test_rasterize_argument_errors():
    lib = L.lib()
    c = cam()
    p = tg.Params().c()
    pr = L.Projected(None, None, 0)
    b = L.Binned(0, None, None, None, None, None, None, None, None)
    bg = (ctypes.c_float * 3)(0, 0, 0)
    st, msg = status_of(lib.tgs_rasterize, ctypes.byref(pr), ctypes.byref(b), ctypes.byref(c), ctypes.byref(p),
                        L.ORDER_BINNED, bg, None, None, None, None, None, None, None, None)
    assert st == L.TGS_ERR_INVALID_ARG


def test_backward_argument_errors():
    # every case fails validation before anything could be launched
    lib = L.lib()
    c = cam()
    p = tg.Params().c()
    fake = ctypes.c_void_p(0x1000).value
    pr = L.Projected(fake, fake, 10)
    b = L.Binned(100, None, None, fake, fake, None, None, fake, fake, None)
    bg = (ctypes.c_float * 3)(0, 0, 0)
    rb = lib.tgs_rasterize_backward
    st, msg = status_of(rb, ctypes.byref(pr), None, ctypes.byref(c), ctypes.byref(p), L.ORDER_BINNED, bg, fake, None,
                        None, None, fake, None)
    assert st == L.TGS_ERR_INVALID_ARG and "binned" in msg
    st, msg = status_of(rb, ctypes.byref(pr), ctypes.byref(b), ctypes.byref(c), ctypes.byref(p), L.ORDER_BINNED, bg,
                        None, None, None, None, fake, None)
    assert st == L.TGS_ERR_INVALID_ARG and "d_rgb" in msg
    st, msg = status_of(rb, ctypes.byref(pr), ctypes.byref(b), ctypes.byref(c), ctypes.byref(p), L.ORDER_BINNED, bg,
                        fake, None, None, None, None, None)
    assert st == L.TGS_ERR_INVALID_ARG and "d_splats" in msg
    st, msg = status_of(rb, ctypes.byref(pr), ctypes.byref(b), ctypes.byref(c), ctypes.byref(p), L.ORDER_BINNED, bg,
                        fake, None, fake, None, fake, None)
    assert st == L.TGS_ERR_INVALID_ARG and "trans" in msg
    st, msg = status_of(rb, ctypes.byref(pr), ctypes.byref(b), ctypes.byref(c), ctypes.byref(p), 7, bg, fake, None,
                        None, None, None, None)
    assert st == L.TGS_ERR_INVALID_ARG and "order" in msg
    b.pairs = None
    st, msg = status_of(rb, ctypes.byref(pr), ctypes.byref(b), ctypes.byref(c), ctypes.byref(p), L.ORDER_BINNED, bg,
                        fake, None, None, None, None, None)
    assert st == L.TGS_ERR_INVALID_ARG
    pb = lib.tgs_project_backward
    gr = L.GaussianGrads(fake, fake, fake, fake, fake)
    g = L.Gaussians(fake, fake, fake, fake, fake, 10, 4)
    st, msg = status_of(pb, ctypes.byref(g), ctypes.byref(c), fake, ctypes.byref(gr), None)
    assert st == L.TGS_ERR_INVALID_ARG and "sh_degree" in msg
    g = L.Gaussians(fake, fake, fake, fake, fake, 10, 3)
    st, msg = status_of(pb, ctypes.byref(g), ctypes.byref(c), None, ctypes.byref(gr), None)
    assert st == L.TGS_ERR_INVALID_ARG and "gradient" in msg
    st, msg = status_of(pb, ctypes.byref(g), ctypes.byref(c), fake, None, None)
    assert st == L.TGS_ERR_INVALID_ARG and "grads" in msg
    gr.sh = None
    st, msg = status_of(pb, ctypes.byref(g), ctypes.byref(c), fake, ctypes.byref(gr), None)
    assert st == L.TGS_ERR_INVALID_ARG
    bad = cam(20000, 10)
    gr.sh = fake
    st, msg = status_of(pb, ctypes.byref(g), ctypes.byref(bad), fake, ctypes.byref(gr), None)
    assert st == L.TGS_ERR_INVALID_ARG and "image size" in msg


def test_error_type():
    with pytest.raises(tg.TileGSError):
        L.check(L.TGS_ERR_INVALID_ARG)


def test_repair_mode_argument_errors():
    lib = L.lib()
    g = L.Gaussians(None, None, None, None, None, 0, 0)
    out = L.Projected(None, None, 0)
    p = L.Params()
    lib.tgs_default_params(ctypes.byref(p))
    assert (p.repair, p.near_shift) == (L.REPAIR_ALL, 0)
    assert abs(p.repair_budget - 0.25) < 1e-7 and p.shift_alpha == 1.0 and p.shift_gamma == 0.25
    assert p.split_entries == 2048 and p.split_mean_factor == 2
    cases = [(tg.Params(repair="rules", packed=1), L.TGS_ERR_UNSUPPORTED, "packed"),
             (tg.Params(repair="none", packed=2), L.TGS_ERR_UNSUPPORTED, "packed"),
             (tg.Params(repair="rules", repair_budget=1.5), L.TGS_ERR_INVALID_ARG, "repair_budget"),
             (tg.Params(repair="rules", repair_budget=float("nan")), L.TGS_ERR_INVALID_ARG, "repair_budget"),
             (tg.Params(near_shift=True, shift_gamma=1.0), L.TGS_ERR_INVALID_ARG, "shift_gamma"),
             (tg.Params(near_shift=True, shift_alpha=-1.0), L.TGS_ERR_INVALID_ARG, "shift_alpha"),
             (tg.Params(near_shift=True, shift_alpha=float("inf")), L.TGS_ERR_INVALID_ARG, "shift_alpha"),
             (tg.Params(split_entries=1000), L.TGS_ERR_INVALID_ARG, "split_entries"),
             (tg.Params(split_entries=128), L.TGS_ERR_INVALID_ARG, "split_entries"),
             (tg.Params(split_mean_factor=-1), L.TGS_ERR_INVALID_ARG, "split_mean_factor"),
             (tg.Params(sub_bins=3), L.TGS_ERR_INVALID_ARG, "sub_bins"),
             (tg.Params(sub_bins=16), L.TGS_ERR_INVALID_ARG, "sub_bins")]
    for bad, code, word in cases:
        st, msg = status_of(lib.tgs_project, ctypes.byref(g), ctypes.byref(cam()), ctypes.byref(bad.c()),
                            ctypes.byref(out), None)
        assert st == code and word in msg, (bad, st, msg)
    raw = tg.Params().c()
    raw.repair = 3
    st, msg = status_of(lib.tgs_project, ctypes.byref(g), ctypes.byref(cam()), ctypes.byref(raw), ctypes.byref(out),
                        None)
    assert st == L.TGS_ERR_INVALID_ARG and "repair" in msg
    raw = tg.Params(repair="rules").c()
    raw.per_tile_bins = 0x1000
    st, msg = status_of(lib.tgs_project, ctypes.byref(g), ctypes.byref(cam()), ctypes.byref(raw), ctypes.byref(out),
                        None)
    assert st == L.TGS_ERR_UNSUPPORTED and "uniform" in msg
    # the selection scan needs its own status words (one pair per 4096 segments)
    c = cam(1920, 1080)
    # (against exact repair on the same near-depth bins, which uses no sub-bins either)
    base = lib.tgs_bin_workspace_size(1000, 5000, ctypes.byref(c), ctypes.byref(tg.Params(near_shift=True).c()),
                                      L.ORDER_BINNED)
    rules = lib.tgs_bin_workspace_size(1000, 5000, ctypes.byref(c), ctypes.byref(tg.paper_params().c()),
                                       L.ORDER_BINNED)
    assert rules > base
