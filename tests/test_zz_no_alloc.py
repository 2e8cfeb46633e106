"""The allocation-free batched raster (tgs_rasterize_batch_noalloc) against
tgs_rasterize_batch with a caller workspace: same views, same streams, the
images must be bitwise equal (the same kernels run on the library's fixed
scratch instead of the workspace). Two calls in a row, the second with fewer
and smaller views, so stale control words or work items of the first call
would show; a batch too large for the fixed scratch is rejected before
anything is enqueued."""
import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu

tg = pytest.importorskip("paper_2609_03613_amd")


def dev():
    return torch.device("cuda:0")


def views(n_views, scale, seed):
    cams = scenes.ring_cameras(n_views, seed=seed)
    out = []
    for c in cams:
        W, H = max(1, int(round(c["width"] * scale))), max(1, int(round(c["height"] * scale)))
        s = W / c["width"]
        out.append(scenes.camera(c["R"], c["t"], c["fx"] * s, c["fy"] * s, W / 2.0, H / 2.0, W, H))
    return out


MIXED = [dict(tile_size=16, num_bins=64), dict(tile_size=8, num_bins=16), dict(tile_size=32, num_bins=128),
         dict(tile_size=16, num_bins=32), dict(tile_size=32, num_bins=8), dict(tile_size=8, num_bins=64)]


def both(g, cams, params):
    """(noalloc outputs, workspace outputs) of the same prepared views."""
    br = tg.BatchRenderer(cams, params, device=dev(), bg=(0.2, 0.1, 0.3))
    br.frame(g, sync=True)  # project + bin every view, size the buffers
    for o in br.outs:
        o["rgb"].fill_(-7.0)
        o["alpha"].fill_(-7.0)
        o["last"].fill_(-7)
    br.rasterize(br.proj, br.binned, noalloc=True)
    torch.cuda.synchronize()
    got = [{k: v.clone() for k, v in o.items()} for o in br.outs]
    for o in br.outs:
        o["rgb"].fill_(-9.0)
    br.rasterize(br.proj, br.binned)
    torch.cuda.synchronize()
    return got, br.outs


def test_noalloc_batch_matches_workspace_batch_twice():
    gnp, _ = scenes.batched_scene(seed=5, n=60000)
    g = tg.to_device(gnp, dev())
    # first call: six views; second call: three smaller views
    for n_views, scale, seed in ((6, 0.5, 5), (3, 0.2, 6)):
        cams = views(n_views, scale, seed)
        got, want = both(g, cams, [tg.Params(**m) for m in MIXED[:n_views]])
        for v, (a, b) in enumerate(zip(got, want)):
            for k in ("rgb", "alpha", "last"):
                assert torch.equal(a[k], b[k]), (n_views, v, k)
            assert float(a["alpha"].max()) > 0.1  # the views see the scene


def test_noalloc_batch_rejects_views_beyond_its_scratch():
    # 16 views of 8192x8192 at 8-pixel tiles: 16 x 1M blocks, far beyond
    # the fixed scratch; rejected on the host before any launch
    import ctypes
    from paper_2609_03613_amd import _lib as L
    cams = [scenes.camera(np.eye(3), np.zeros(3), 4000.0, 4000.0, 4096.0, 4096.0, 8192, 8192) for _ in range(16)]
    params = [tg.Params(tile_size=8) for _ in cams]
    nv = len(cams)
    ccams = (L.Camera * nv)(*[tg.camera_struct(c) for c in cams])
    cparams = (L.Params * nv)(*[p.c() for p in params])
    dummy = torch.zeros(16, dtype=torch.int64, device=dev())
    pr = (L.Projected * nv)(*[L.Projected(0, 0, 0) for _ in cams])
    bs = (L.Binned * nv)(*[L.Binned(0, 0, 0, 0, dummy.data_ptr(), 0, 0, 0, dummy.data_ptr(), 0, 0, 0)
                           for _ in cams])
    orders = (ctypes.c_int32 * nv)(*([L.ORDER_BINNED] * nv))
    ptrs = (ctypes.c_void_p * nv)(*([dummy.data_ptr()] * nv))
    bg = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
    st = L.lib().tgs_rasterize_batch_noalloc(nv, ctypes.cast(pr, ctypes.c_void_p), ctypes.cast(bs, ctypes.c_void_p),
                                             ctypes.cast(ccams, ctypes.c_void_p), ctypes.cast(cparams, ctypes.c_void_p),
                                             ctypes.cast(orders, ctypes.c_void_p), bg, ptrs, ptrs, ptrs, None)
    assert st == L.TGS_ERR_WORKSPACE
    assert "fixed scratch" in L.lib().tgs_last_error().decode()
    torch.cuda.synchronize()
    assert int(dummy.abs().sum()) == 0
