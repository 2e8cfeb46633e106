"""GPU parity of the backward pass against the FP64 oracle adjoint.

The paper has no backward pass; the oracle's adjoint is pinned by central
finite differences (test_oracle_adjoint.py). Bar: every gradient within
1e-3 relative of the oracle, measured per gradient array (per column of the
splat gradient lines) as |gpu - ref| / (|ref| + 1e-3 max |ref|), the floor
keeping cancellation-dominated near-zero entries from dividing by ~0.
Upstream gradients are zeroed on pixels whose forward value is
threshold-ambiguous in the oracle (alpha within rounding of 1/255, the stop
test within rounding of 1e-4, a Gaussian whose visibility or rect is
within rounding of an edge), where binary32 and binary64 may legitimately
take different discrete paths. The projection backward alone, fed the
oracle's splat gradients rounded to binary32, is held to 1e-4: the
quaternion gradient drops its radial part (the normalisation), a
cancellation that amplifies the 6e-8 input rounding by up to a few hundred.
"""
import numpy as np
import pytest
import torch

import oracle
import scenes
from helpers import to_np

pytestmark = pytest.mark.gpu

tg = pytest.importorskip("paper_2609_03613_amd")

GRAD_TOL = 1e-3
KEYS = ("means", "log_scales", "quats", "logits", "sh")
AMBIG = oracle.PIX_AMBIG_ALPHA | oracle.PIX_AMBIG_STOP | oracle.PIX_AMBIG_GAUSS


def dev():
    return torch.device("cuda:0")


def grad_err(gpu, ref):
    gpu = np.asarray(gpu, np.float64).reshape(len(ref), -1)
    ref = np.asarray(ref, np.float64).reshape(len(ref), -1)
    scale = np.abs(ref).max(axis=0, keepdims=True)
    if not np.any(scale):
        return float(np.abs(gpu).max(initial=0.0))
    err = np.abs(gpu - ref) / (np.abs(ref) + 1e-3 * scale + 1e-30)
    return float(err.max())


def cam_for(W, H, f=100.0):
    return scenes.camera(np.eye(3), np.zeros(3), f, f, W / 2, H / 2, W, H)


def upstream(W, H, mask, seed):
    rng = np.random.default_rng(seed)
    d_img = rng.normal(0.0, 1.0, size=(H, W, 3)) * mask[..., None]
    d_alpha = rng.normal(0.0, 1.0, size=(H, W)) * mask
    # the GPU receives binary32; give the oracle the same values
    return d_img.astype(np.float32), d_alpha.astype(np.float32)


def gpu_raster_backward(splats, info, cam, order, d_img, d_alpha, bg, params=None):
    """Bins and runs tgs_rasterize_backward; returns the gradient lines."""
    r = tg.Renderer(cam, params or tg.Params(), device=dev())
    s = torch.as_tensor(splats).to(dev())
    i = torch.as_tensor(np.ascontiguousarray(info).view(np.int32)).to(dev())
    b = r.bin(s, i, order)
    dr = torch.as_tensor(d_img).to(dev())
    da = None if d_alpha is None else torch.as_tensor(d_alpha).to(dev())
    out = r.rasterize_backward(s, i, b, dr, da, bg=bg)
    torch.cuda.synchronize()
    return to_np(out)


RASTER_CASES = [
    # seed, W, H, splats per pixel, max sigma (px)
    (0, 128, 96, 1 / 8, 12.0),
    (1, 203, 77, 1 / 8, 12.0),
    (2, 16, 16, 1 / 4, 6.0),
    (3, 96, 64, 2.0, 20.0),   # dense: most pixels reach the stop test
]


@pytest.mark.parametrize("seed,W,H,density,sigma", RASTER_CASES)
def test_raster_backward_matches_oracle(seed, W, H, density, sigma):
    n = max(1, int(W * H * density))
    splats, info = scenes.random_splats(n, W, H, seed=seed, tie_fraction=0.05, hidden_fraction=0.05,
                                        max_sigma_px=sigma)
    cam = cam_for(W, H)
    bg = (0.1, 0.2, 0.3)
    proj = oracle.splats_to_proj(splats, info)
    fwd = oracle.render(proj, W, H, bg=bg)
    mask = (fwd["flags"] & AMBIG) == 0
    if density >= 1:
        assert (fwd["alpha"] > 1 - 2e-4).mean() > 0.2
    d_img, d_alpha = upstream(W, H, mask, seed + 100)
    ref = oracle.composite_adjoint(proj, W, H, bg=bg, d_img=d_img, d_alpha=d_alpha)
    assert np.abs(ref["rgb"] - fwd["rgb"]).max() < 1e-12
    outs = {}
    for order in ("global", "binned"):
        g = gpu_raster_backward(splats, info, cam, order, d_img, d_alpha, bg)
        assert g.shape == (n, 12) and not np.any(g[:, 9:])
        e = [grad_err(g[:, k], ref["d_proj"][:, k]) for k in range(9)]
        assert max(e) <= GRAD_TOL, (order, e)
        outs[order] = g
    # same per-pixel contributions in both orders; only the order of the
    # float atomic sums can differ
    assert grad_err(outs["global"][:, :9], outs["binned"][:, :9]) <= 1e-4


@pytest.mark.parametrize("ts", [8, 32])
def test_raster_backward_tile_sizes(ts):
    W, H = 100, 70
    n = W * H // 6
    splats, info = scenes.random_splats(n, W, H, tile_size=ts, seed=20 + ts, hidden_fraction=0.05)
    cam = cam_for(W, H)
    proj = oracle.splats_to_proj(splats, info)
    fwd = oracle.render(proj, W, H, tile_size=ts)
    mask = (fwd["flags"] & AMBIG) == 0
    d_img, d_alpha = upstream(W, H, mask, ts)
    ref = oracle.composite_adjoint(proj, W, H, tile_size=ts, d_img=d_img, d_alpha=d_alpha)
    for order in ("global", "binned"):
        g = gpu_raster_backward(splats, info, cam, order, d_img, d_alpha, (0.0, 0.0, 0.0),
                                tg.Params(tile_size=ts, num_bins=16))
        e = [grad_err(g[:, k], ref["d_proj"][:, k]) for k in range(9)]
        assert max(e) <= GRAD_TOL, (ts, order, e)


def test_raster_backward_from_saved_forward_state():
    # the forward's saved transmittance and last position replace the
    # recomputed walk: same gradients up to the atomic summation order
    W, H, n = 150, 100, 3000
    splats, info = scenes.random_splats(n, W, H, seed=12, max_sigma_px=16.0)
    cam = cam_for(W, H)
    r = tg.Renderer(cam, device=dev())
    s = torch.as_tensor(splats).to(dev())
    i = torch.as_tensor(info.view(np.int32)).to(dev())
    b = r.bin(s, i, "binned")
    fwd = r.rasterize(s, i, b, bg=(0.3, 0.2, 0.1), trans=True)
    assert torch.allclose(1.0 - fwd["trans"], fwd["alpha"])
    d = torch.as_tensor(np.random.default_rng(2).normal(size=(H, W, 3)).astype(np.float32)).to(dev())
    da = torch.as_tensor(np.random.default_rng(3).normal(size=(H, W)).astype(np.float32)).to(dev())
    g1 = to_np(r.rasterize_backward(s, i, b, d, da, bg=(0.3, 0.2, 0.1)))
    g2 = to_np(r.rasterize_backward(s, i, b, d, da, bg=(0.3, 0.2, 0.1), saved=fwd))
    torch.cuda.synchronize()
    assert grad_err(g2[:, :9], g1[:, :9]) <= 1e-4


def test_raster_backward_without_alpha_gradient_and_repeat():
    W, H, n = 64, 48, 500
    splats, info = scenes.random_splats(n, W, H, seed=7)
    cam = cam_for(W, H)
    proj = oracle.splats_to_proj(splats, info)
    fwd = oracle.render(proj, W, H)
    mask = (fwd["flags"] & AMBIG) == 0
    d_img, _ = upstream(W, H, mask, 3)
    ref = oracle.composite_adjoint(proj, W, H, d_img=d_img)
    a = gpu_raster_backward(splats, info, cam, "binned", d_img, None, (0.0, 0.0, 0.0))
    b = gpu_raster_backward(splats, info, cam, "binned", d_img, None, (0.0, 0.0, 0.0))
    assert max(grad_err(a[:, k], ref["d_proj"][:, k]) for k in range(9)) <= GRAD_TOL
    assert grad_err(a[:, :9], b[:, :9]) <= 1e-4


def test_raster_backward_edge_cases():
    cam = cam_for(40, 24)
    r = tg.Renderer(cam, device=dev())
    # no Gaussians
    s = torch.zeros((0, 16), device=dev())
    i = torch.zeros((0, 4), dtype=torch.int32, device=dev())
    b = r.bin(s, i, "binned")
    out = r.rasterize_backward(s, i, b, torch.ones((24, 40, 3), device=dev()))
    assert out.shape == (0, 12)
    # every Gaussian invisible: all gradients zero
    splats, info = scenes.random_splats(50, 40, 24, seed=1, hidden_fraction=1.0)
    g = gpu_raster_backward(splats, info, cam, "binned", np.ones((24, 40, 3), np.float32), None, (0.0, 0.0, 0.0))
    assert not np.any(g)
    # truncated stream (overflow flag): all gradients zero
    splats, info = scenes.random_splats(2000, 128, 128, seed=5)
    cam = cam_for(128, 128)
    p = tg.Params()
    r = tg.Renderer(cam, p, device=dev())
    s = torch.as_tensor(splats).to(dev())
    i = torch.as_tensor(info.view(np.int32)).to(dev())
    M = oracle.count_entries(scenes.info_rects(info))
    r._binned[1] = tg.Binned("binned", M // 2, r.tiles, p.num_bins, p.packed, dev())
    b = r.bin(s, i, "binned", sync=False)
    out = r.rasterize_backward(s, i, b, torch.ones((128, 128, 3), device=dev()))
    torch.cuda.synchronize()
    assert to_np(b.counters)[2] == 1 and not np.any(to_np(out))


PROJ_CASES = [
    ("fd_subcase", None),
    ("training_d3", 3),
    ("training_d1", 1),
    ("small_d0", 0),
]


def scene_for(case):
    if case == "fd_subcase":
        return scenes.fd_subcase()
    if case == "small_d0":
        return scenes.small_forward(seed=4, n=3000)
    g, cam = scenes.training_scene(seed=5, n=20000, width=320, height=208)
    deg = int(case[-1])
    g = dict(g)
    g["sh"] = np.ascontiguousarray(g["sh"][:, : (deg + 1) ** 2])
    g["sh_degree"] = deg
    return g, cam


def oracle_grads(g, cam, target, bg=(0.0, 0.0, 0.0)):
    """Oracle adjoint for L = sum over unflagged pixels of (rgb - target)^2 /
    (3 W H), with the flags of the oracle's forward image."""
    W, H = cam["width"], cam["height"]
    fwd = oracle.render(oracle.project(g, cam), W, H, bg=bg)
    mask = (fwd["flags"] & AMBIG) == 0
    g64 = {k: (np.asarray(v, np.float64) if k != "sh_degree" else v) for k, v in g.items()}
    up = 2.0 * (fwd["rgb"] - target) * mask[..., None] / fwd["rgb"].size
    return oracle.adjoint(g64, cam, bg=bg, d_img=up), mask, fwd


@pytest.mark.parametrize("case,_", PROJ_CASES)
def test_project_backward_matches_oracle(case, _):
    g, cam = scene_for(case)
    target = scenes.training_target(cam["width"], cam["height"])
    ref, _, _ = oracle_grads(g, cam, target)
    n = len(g["logits"])
    d = np.zeros((n, 12), np.float32)
    d[:, :9] = ref["d_proj"]
    gd = tg.to_device(g, dev())
    out = tg.project_backward(gd, cam, torch.as_tensor(d).to(dev()))
    torch.cuda.synchronize()
    # the oracle's parameter gradients from the binary32-rounded lines
    g64 = {k: (np.asarray(v, np.float64) if k != "sh_degree" else v) for k, v in g.items()}
    for k in KEYS:
        got = to_np(out[k])
        assert got.shape == np.asarray(g[k]).shape, k
        assert grad_err(got, ref[k]) <= 1e-4, (case, k, grad_err(got, ref[k]))
    assert g64["means"].shape[0] == n


@pytest.mark.parametrize("case", ["fd_subcase", "training_d3"])
def test_autograd_gradients_match_oracle(case):
    g, cam = scene_for(case)
    W, H = cam["width"], cam["height"]
    target = scenes.training_target(W, H)
    ref, mask, fwd = oracle_grads(g, cam, target)
    r = tg.Renderer(cam, device=dev())
    gd = tg.to_device(g, dev())
    params = {k: gd[k].clone().requires_grad_(True) for k in KEYS}
    params["sh_degree"] = gd["sh_degree"]
    for order in ("binned", "global"):
        for k in KEYS:
            params[k].grad = None
        rgb, alpha = tg.render_differentiable(r, params, order=order)
        tgt = torch.as_tensor(target).to(dev())
        m = torch.as_tensor(mask.astype(np.float32)).to(dev())[..., None]
        loss = (((rgb - tgt) ** 2) * m).sum() / rgb.numel()
        loss.backward()
        torch.cuda.synchronize()
        ref_loss = float((((fwd["rgb"] - target) ** 2) * mask[..., None]).sum() / fwd["rgb"].size)
        assert abs(float(loss.detach()) - ref_loss) <= 1e-4 * ref_loss
        errs = {k: grad_err(to_np(params[k].grad), ref[k]) for k in KEYS}
        assert max(errs.values()) <= GRAD_TOL, (order, errs)
