"""Pins of the oracle's adjoint (the gradient of a loss of the image).

The paper has no backward pass; the adjoint is the derivative of the forward
model, so it is pinned by binary64 central finite differences of the same
forward model (h = 1e-6 max(1, |theta|)) on the 200-Gaussian 64x64 sub-case
of the 500k training scene, with the loss mean((rgb - target)^2) against a
U[0, 1] target (seed 1). A parameter whose stencil crosses a discontinuity
(the 1/255 cut, the stopping rule, a rect edge) shows one-sided differences
that disagree; such parameters are excluded and counted. Separate cases give
the paths that the sub-case may not exercise: the 0.99 cap, colour clamped at
zero, the frustum guard of the Jacobian, a background colour and a loss term
on alpha. The compositing part alone (gradients with respect to the projected
quantities) is checked against finite differences of ``oracle.render``.
"""
import numpy as np

import oracle
import scenes

KEYS = ("means", "log_scales", "quats", "logits", "sh")


def as64(g):
    return {k: (np.array(v, np.float64) if k != "sh_degree" else v) for k, v in g.items()}


def loss_fn(g, cam, target, bg=(0.0, 0.0, 0.0), w_alpha=None):
    a = oracle.adjoint(g, cam, bg=bg)
    L, up = oracle.mse_upstream(a["rgb"], target)
    if w_alpha is not None:
        L += float(np.sum(w_alpha * a["alpha"]))
    return L, up


def fd_check(g, cam, target, keys=KEYS, per_key=200, seed=0, bg=(0.0, 0.0, 0.0), w_alpha=None,
             only=None, rel=1e-4):
    """Compares the adjoint with central differences on a random sample of
    each parameter array (or of the Gaussians listed in ``only``). Returns
    (number compared, number excluded)."""
    g = as64(g)
    L0, up = loss_fn(g, cam, target, bg, w_alpha)
    a = oracle.adjoint(g, cam, bg=bg, d_img=up, d_alpha=w_alpha)
    rng = np.random.default_rng(seed)
    compared = excluded = 0
    for key in keys:
        arr = g[key]
        per_g = arr.size // arr.shape[0]
        if only is None:
            idx = rng.choice(arr.size, size=min(per_key, arr.size), replace=False)
        else:
            idx = np.concatenate([np.arange(per_g) + per_g * i for i in only])
        gmax = np.abs(a[key]).max()
        for i in idx:
            th = float(arr.reshape(-1)[i])
            h = 1e-6 * max(1.0, abs(th))
            vals = []
            for s in (+1, -1):
                gg = dict(g)
                gg[key] = arr.copy()
                gg[key].reshape(-1)[i] = th + s * h
                vals.append(loss_fn(gg, cam, target, bg, w_alpha)[0])
            Lp, Lm = vals
            if abs((Lp - L0) / h - (L0 - Lm) / h) > 1e-4 * gmax + 1e-9:
                excluded += 1
                continue
            fd = (Lp - Lm) / (2 * h)
            ad = a[key].reshape(-1)[i]
            assert abs(ad - fd) <= rel * (abs(fd) + 1e-3 * gmax) + 1e-10, (key, int(i), ad, fd)
            compared += 1
    return compared, excluded


def test_adjoint_forward_is_the_tiled_image():
    for g, cam in (scenes.fd_subcase(), scenes.small_forward(n=500)):
        for bg in ((0.0, 0.0, 0.0), (0.3, 0.6, 0.9)):
            ref = oracle.render(oracle.project(g, cam), cam["width"], cam["height"], bg=bg)
            a = oracle.adjoint(g, cam, bg=bg)
            np.testing.assert_allclose(a["rgb"], ref["rgb"], rtol=0, atol=1e-12)
            np.testing.assert_allclose(a["alpha"], ref["alpha"], rtol=0, atol=1e-12)


def test_adjoint_matches_central_differences_on_fd_subcase():
    g, cam = scenes.fd_subcase()
    target = scenes.training_target(cam["width"], cam["height"])
    compared, excluded = fd_check(g, cam, target)
    assert compared >= 950 and excluded <= 0.02 * (compared + excluded), (compared, excluded)


def test_adjoint_with_background_and_alpha_term():
    g, cam = scenes.fd_subcase()
    target = scenes.training_target(cam["width"], cam["height"])
    w = np.random.default_rng(5).normal(0.0, 1e-4, size=(cam["height"], cam["width"]))
    compared, excluded = fd_check(g, cam, target, per_key=60, seed=1, bg=(0.2, 0.5, 0.8), w_alpha=w)
    assert compared >= 280 and excluded <= 6


def _one(mean, log_scale, logit, sh0, quat=(1.0, 0.0, 0.0, 0.0), degree=0):
    nsh = (degree + 1) ** 2
    sh = np.zeros((1, nsh, 3))
    sh[0, 0] = sh0
    return {"means": np.array([mean], np.float64), "log_scales": np.array([log_scale], np.float64),
            "quats": np.array([quat], np.float64), "logits": np.array([logit], np.float64), "sh": sh,
            "sh_degree": degree}


def _cat(*gs):
    return {k: (np.concatenate([x[k] for x in gs]) if k != "sh_degree" else gs[0][k]) for k in gs[0]}


def test_adjoint_capped_alpha_and_clamped_colour():
    cam = scenes.camera(np.eye(3), np.zeros(3), 40.0, 40.0, 20.0, 20.0, 40, 40)
    # o = sigmoid(7) ~ 0.9991: alpha is capped at 0.99 near the centre; the
    # red channel's raw colour is negative, so it is clamped to zero
    a = _one((0.05, -0.02, 3.0), (-1.6, -1.9, -1.7), 7.0, (-3.0, 0.8, 0.3), quat=(0.9, 0.2, -0.3, 0.1))
    b = _one((-0.1, 0.1, 4.0), (-1.3, -1.5, -1.4), 0.5, (0.4, -0.2, 0.9))
    g = _cat(a, b)
    target = np.full((40, 40, 3), 0.25)
    ga = as64(g)
    alone = oracle.adjoint(as64(a), cam)
    assert alone["alpha"].max() == 0.99 and alone["rgb"][..., 0].max() == 0.0
    out = oracle.adjoint(ga, cam)
    _, up = oracle.mse_upstream(out["rgb"], target)
    grads = oracle.adjoint(ga, cam, d_img=up)
    assert grads["sh"][0, 0, 0] == 0.0  # clamped channel
    compared, excluded = fd_check(g, cam, target, only=[0, 1])
    assert compared >= 20 and excluded == 0


def test_adjoint_frustum_guard():
    # mean far right of the image (x / z beyond the guard): the Jacobian uses
    # the guarded tx, which no longer depends on x
    cam = scenes.camera(np.eye(3), np.zeros(3), 30.0, 30.0, 16.0, 16.0, 32, 32)
    far = _one((3.0, 0.05, 2.0), (0.2, -0.4, 0.1), 2.0, (0.6, 0.2, 0.1), quat=(0.8, 0.1, 0.5, -0.2))
    near = _one((0.1, 0.0, 3.0), (-2.0, -2.1, -2.2), 1.0, (0.1, 0.3, 0.5))
    g = _cat(far, near)
    cam_d = dict(cam)
    lim = 1.3 * 32 / (2 * 30.0)  # the guard: 1.3 tan(half FOV), centred principal point
    assert 3.0 / 2.0 > lim
    target = np.full((32, 32, 3), 0.5)
    ga = as64(g)
    out = oracle.adjoint(ga, cam_d)
    assert out["alpha"][:, -4:].max() > 0.05  # the far Gaussian reaches the image
    compared, excluded = fd_check(g, cam_d, target, only=[0, 1])
    assert compared >= 20 and excluded == 0


def test_compositing_adjoint_matches_render_differences():
    # dL/d(mean2d, conic, opacity, rgb) against central differences of the
    # plain per-pixel compositing in oracle.render
    g, cam = scenes.fd_subcase()
    W, H = cam["width"], cam["height"]
    target = scenes.training_target(W, H)
    proj = oracle.project(g, cam)
    img = oracle.render(proj, W, H)
    L0, up = oracle.mse_upstream(img["rgb"], target)
    d = oracle.adjoint(as64(g), cam, d_img=up)["d_proj"]
    fields = [("mean2d", 0), ("mean2d", 1), ("conic", 0), ("conic", 1), ("conic", 2), ("opacity", None),
              ("rgb", 0), ("rgb", 1), ("rgb", 2)]
    rng = np.random.default_rng(3)
    vis = np.flatnonzero(proj["flags"] & oracle.VISIBLE)
    compared = 0
    for j, (name, comp) in enumerate(fields):
        gmax = np.abs(d[:, j]).max()
        for gi in rng.choice(vis, size=25, replace=False):
            base = proj[name][gi] if comp is None else proj[name][gi, comp]
            h = 1e-6 * max(1.0, abs(base))
            vals = []
            for s in (+1, -1):
                p = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in proj.items()}
                if comp is None:
                    p[name][gi] = base + s * h
                else:
                    p[name][gi, comp] = base + s * h
                vals.append(oracle.mse_upstream(oracle.render(p, W, H)["rgb"], target)[0])
            if abs((vals[0] - L0) - (L0 - vals[1])) / h > 1e-4 * gmax + 1e-9:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(d[gi, j] - fd) <= 1e-4 * (abs(fd) + 1e-3 * gmax) + 5e-10, (name, comp, gi, d[gi, j], fd)
            compared += 1
    assert compared >= 200


def test_invisible_gaussians_have_zero_gradient():
    g, cam = scenes.fd_subcase()
    g = as64(g)
    g["means"][:5, 2] = -1.0  # behind the camera
    g["logits"][5:8] = -8.0   # opacity below 1/255
    target = scenes.training_target(cam["width"], cam["height"])
    _, up = oracle.mse_upstream(oracle.adjoint(g, cam)["rgb"], target)
    a = oracle.adjoint(g, cam, d_img=up)
    for k in KEYS:
        assert not np.any(a[k][:8]), k
    assert np.abs(a["means"][8:]).max() > 0


def test_composite_adjoint_on_records_matches_full_adjoint():
    # the records-level entry (used with synthetic splats) on the projected
    # records of a scene gives the same image and dL/d(projected)
    g, cam = scenes.fd_subcase()
    W, H = cam["width"], cam["height"]
    target = scenes.training_target(W, H)
    proj = oracle.project(g, cam)
    full0 = oracle.adjoint(as64(g), cam, bg=(0.1, 0.2, 0.3))
    _, up = oracle.mse_upstream(full0["rgb"], target)
    w = np.random.default_rng(2).normal(0.0, 1e-4, size=(H, W))
    full = oracle.adjoint(as64(g), cam, bg=(0.1, 0.2, 0.3), d_img=up, d_alpha=w)
    rec = oracle.composite_adjoint(proj, W, H, bg=(0.1, 0.2, 0.3), d_img=up, d_alpha=w)
    np.testing.assert_allclose(rec["rgb"], full["rgb"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(rec["alpha"], full["alpha"], rtol=0, atol=1e-12)
    scale = np.abs(full["d_proj"]).max(axis=0)
    assert np.all(np.abs(rec["d_proj"] - full["d_proj"]) <= 1e-9 * scale + 1e-15)


def test_project_adjoint_against_differences_of_the_projection():
    # oracle.project_adjoint(d) is the gradient of the linear functional
    # F = sum_g d[g] . (mean2d, conic, opacity, rgb)(theta) of the binary64
    # projection. Central differences of oracle.project (which takes binary32
    # parameters: the stencil points are binary32 values and the step is
    # their exact difference) check it, with one Gaussian beyond the frustum
    # guard and one with a colour channel clamped at zero.
    cam = scenes.camera(np.eye(3), np.zeros(3), 90.0, 80.0, 33.0, 30.0, 64, 56)
    rng = np.random.default_rng(5)
    n = 6
    g = {
        "means": np.stack([rng.uniform(-0.4, 0.4, n), rng.uniform(-0.4, 0.4, n), rng.uniform(2, 4, n)], 1),
        "log_scales": rng.normal(-2.5, 0.4, (n, 3)), "quats": rng.normal(0, 1, (n, 4)),
        "logits": rng.normal(0.5, 1.0, n), "sh": rng.normal(0, 0.3, (n, 16, 3)), "sh_degree": 3,
    }
    g["means"][1] = (2.0, -0.1, 2.0)   # x/z = 1, beyond the guard (about 0.58 on the right)
    g["log_scales"][1] = (-0.5, -0.6, -0.4)  # large enough to reach the image
    g["sh"][2, 0, 0] = -3.0            # red channel clamped at zero
    g = {k: (np.asarray(v, np.float32) if k != "sh_degree" else v) for k, v in g.items()}
    d = rng.normal(0, 1, (n, 9))
    # balance the conic terms against the others (conics of large splats are
    # small), and let the guarded Gaussian's gradient come from its conic
    # alone, so that the guard's part of the Jacobian derivative dominates it
    d[:, 2:5] /= np.abs(oracle.project(g, cam)["conic"]).max(axis=1, keepdims=True)
    d[1, [0, 1, 5, 6, 7, 8]] = 0.0
    got = oracle.project_adjoint(g, cam, d)
    assert got["sh"][2, :, 0].max() == 0.0 and np.abs(got["sh"][2, :, 1]).max() > 0

    def F(gg):
        p = oracle.project(gg, cam)
        assert np.all(p["flags"] & oracle.VISIBLE)
        v = np.concatenate([p["mean2d"], p["conic"], p["opacity"][:, None], p["rgb"]], 1)
        return float(np.sum(d * v))

    checked = 0
    for key in KEYS:
        arr = g[key]
        for i in range(arr.size):
            th = arr.reshape(-1)[i]
            h = np.float32(2e-3 * max(0.05, abs(float(th))))
            vals, pts = [], []
            for s in (+1, -1):
                gg = dict(g)
                gg[key] = arr.copy()
                gg[key].reshape(-1)[i] = np.float32(th + s * h)
                pts.append(float(gg[key].reshape(-1)[i]))
                vals.append(F(gg))
            fd = (vals[0] - vals[1]) / (pts[0] - pts[1])
            an = float(got[key].reshape(-1)[i])
            scale = np.abs(got[key][i // (arr.size // n)]).max()
            assert abs(fd - an) <= 2e-4 * (abs(an) + 1e-2 * scale), (key, i, fd, an)
            checked += 1
    assert checked == n * (3 + 3 + 4 + 1 + 48)


def test_project_adjoint_is_the_last_step_of_the_full_adjoint():
    # On the finite-difference sub-case the projection adjoint fed the full
    # adjoint's d_proj returns the full adjoint's parameter gradients
    g, cam = scenes.fd_subcase()
    target = scenes.training_target(cam["width"], cam["height"])
    ga = as64(g)
    _, up = loss_fn(ga, cam, target)
    a = oracle.adjoint(ga, cam, d_img=up)
    p = oracle.project_adjoint(ga, cam, a["d_proj"])
    for k in KEYS:
        assert np.array_equal(p[k], a[k]), k
