"""Pins of the oracle's projection and colour (EWA splatting / 3DGS image model).

Each test checks the oracle against something other than its own formulas:
closed forms of special cases, a numerical Jacobian, scipy's spherical
harmonics, quadrature orthonormality and exact invariances.
"""
import math

import numpy as np
import pytest

import oracle
import scenes


def one_gaussian(mean, log_scales, quat=(1.0, 0.0, 0.0, 0.0), logit=0.0, sh=None, degree=0):
    if sh is None:
        sh = np.zeros(((degree + 1) ** 2, 3))
    return {
        "means": np.array([mean], np.float32), "log_scales": np.array([log_scales], np.float32),
        "quats": np.array([quat], np.float32), "logits": np.array([logit], np.float32),
        "sh": np.array([sh], np.float32), "sh_degree": degree,
    }


def ident_cam(f=100.0, w=64, h=64):
    return scenes.camera(np.eye(3), np.zeros(3), f, f, w / 2.0, h / 2.0, w, h)


def test_isotropic_on_axis_closed_form():
    # mu = (0, 0, z) on the optical axis: J has a zero third column on the
    # axis, so Sigma' = (f sigma / z)^2 I + 0.3 I exactly.
    s, z, f = 0.05, 3.0, 100.0
    g = one_gaussian((0.0, 0.0, z), [math.log(s)] * 3)
    p = oracle.project(g, ident_cam(f))
    s32 = float(np.float32(math.log(s)))
    sig = f * math.exp(s32) / z
    expect = sig * sig + 0.3
    np.testing.assert_allclose(p["cov2d"][0], [expect, 0.0, expect], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(p["conic"][0], [1 / expect, 0.0, 1 / expect], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(p["mean2d"][0], [32.0, 32.0], rtol=0, atol=1e-12)
    assert p["depth"][0] == pytest.approx(3.0)
    assert p["opacity"][0] == pytest.approx(0.5)


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.1, 2.5])
def test_anisotropic_rotation_about_optical_axis(theta):
    # A rotation by theta about the optical axis rotates the 2D covariance by
    # theta: Sigma' = (f/z)^2 R(theta) diag(s1^2, s2^2) R(theta)^T + 0.3 I.
    s1, s2, s3, z, f = 0.08, 0.02, 0.5, 4.0, 120.0
    q = (math.cos(theta / 2), 0.0, 0.0, math.sin(theta / 2))
    g = one_gaussian((0.0, 0.0, z), [math.log(s1), math.log(s2), math.log(s3)], quat=q)
    p = oracle.project(g, ident_cam(f))
    q32 = np.array(q, np.float32).astype(np.float64)
    th = 2.0 * math.atan2(q32[3], q32[0])
    ls = np.array([math.log(s1), math.log(s2)], np.float32).astype(np.float64)
    a1, a2 = np.exp(ls) * f / z
    c, sn = math.cos(th), math.sin(th)
    Rt = np.array([[c, -sn], [sn, c]])
    S = Rt @ np.diag([a1 * a1, a2 * a2]) @ Rt.T + 0.3 * np.eye(2)
    np.testing.assert_allclose(p["cov2d"][0], [S[0, 0], S[0, 1], S[1, 1]], rtol=1e-10, atol=1e-12)


def test_jacobian_against_numerical_derivative():
    # For an isotropic Gaussian Sigma_cam = s^2 I, so Sigma' - 0.3 I = s^2 J J^T
    # where J is the derivative of the pinhole map (fx x/z + cx, fy y/z + cy).
    rng = np.random.default_rng(3)
    fx, fy, W, H = 150.0, 130.0, 96, 80
    cam = scenes.camera(np.eye(3), np.zeros(3), fx, fy, 41.0, 37.0, W, H)
    for _ in range(10):
        mu = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), rng.uniform(1.5, 4)], np.float32)
        s = 0.03
        p = oracle.project(one_gaussian(mu, [math.log(s)] * 3), cam)
        m = mu.astype(np.float64)

        def pin(v):
            return np.array([fx * v[0] / v[2] + 41.0, fy * v[1] / v[2] + 37.0])
        h = 1e-6
        J = np.stack([(pin(m + h * e) - pin(m - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        s64 = math.exp(float(np.float32(math.log(s))))
        S = s64 * s64 * J @ J.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(p["cov2d"][0], [S[0, 0], S[0, 1], S[1, 1]], rtol=1e-7)
        np.testing.assert_allclose(p["mean2d"][0], pin(m), rtol=1e-12)


def test_world_scale_invariance():
    # Scaling the means, the scales and the camera translation by k leaves the
    # screen-space projection unchanged (and the depth scaled by k).
    g, cam = scenes.small_forward(seed=4, n=300)
    cam["t"] = np.array([0.1, -0.2, 0.5])
    k = 2.0  # a power of two keeps the fp32 inputs exact
    g2 = dict(g)
    g2["means"] = (g["means"] * k).astype(np.float32)
    g2["log_scales"] = (g["log_scales"] + np.float32(math.log(k))).astype(np.float32)
    cam2 = dict(cam)
    cam2["t"] = cam["t"] * k
    a, b = oracle.project(g, cam), oracle.project(g2, cam2)
    vis = (a["flags"] & 1) > 0
    np.testing.assert_array_equal(vis, (b["flags"] & 1) > 0)
    np.testing.assert_allclose(a["mean2d"][vis], b["mean2d"][vis], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(a["cov2d"][vis], b["cov2d"][vis], rtol=1e-5)
    np.testing.assert_allclose(a["depth"][vis] * k, b["depth"][vis], rtol=1e-14)


def test_rigid_motion_invariance():
    # Moving the world by a rotation Q and translation d and the camera with it
    # (R' = R Q^T, t' = t - R' d) leaves the projection unchanged (degree 0, so
    # the colour does not depend on the view direction).
    g, cam = scenes.small_forward(seed=5, n=200)
    rng = np.random.default_rng(0)
    A = rng.normal(size=(3, 3))
    Q, _ = np.linalg.qr(A)
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    d = np.array([0.25, -0.5, 1.0])
    g2 = dict(g)
    g2["means"] = (g["means"].astype(np.float64) @ Q.T + d).astype(np.float32)
    qw = g["quats"].astype(np.float64)
    # compose the rotation of each Gaussian with Q (quaternion of Q times q)
    from scipy.spatial.transform import Rotation
    rq = Rotation.from_quat(np.concatenate([qw[:, 1:], qw[:, :1]], 1))
    rq2 = Rotation.from_matrix(Q) * rq
    x = rq2.as_quat()
    g2["quats"] = np.concatenate([x[:, 3:], x[:, :3]], 1).astype(np.float32)
    R2 = cam["R"] @ Q.T
    cam2 = dict(cam)
    cam2["R"] = R2
    cam2["t"] = cam["t"] - R2 @ d
    a, b = oracle.project(g, cam), oracle.project(g2, cam2)
    vis = ((a["flags"] & 1) > 0) & ((b["flags"] & 1) > 0)
    assert vis.sum() > 150
    # fp32 rounding of the moved means limits the agreement
    np.testing.assert_allclose(a["mean2d"][vis], b["mean2d"][vis], rtol=0, atol=2e-4)
    np.testing.assert_allclose(a["cov2d"][vis], b["cov2d"][vis], rtol=2e-4, atol=1e-5)
    np.testing.assert_allclose(a["rgb"][vis], b["rgb"][vis], rtol=1e-12)


def test_sh_low_order_closed_forms():
    rng = np.random.default_rng(1)
    for _ in range(20):
        d = rng.normal(size=3)
        x, y, z = d / np.linalg.norm(d)
        Y = oracle.sh_basis(d, 1)
        c1 = math.sqrt(3 / (4 * math.pi))
        np.testing.assert_allclose(Y, [1 / (2 * math.sqrt(math.pi)), -c1 * y, c1 * z, -c1 * x], rtol=1e-13)


def test_sh_against_scipy():
    # Real harmonics from scipy's complex ones (which carry the Condon-Shortley
    # phase): sqrt(2) Re Y_l^m for m > 0, sqrt(2) Im Y_l^|m| for m < 0.
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(2)
    for _ in range(25):
        d = rng.normal(size=3)
        u = d / np.linalg.norm(d)
        polar, azim = math.acos(u[2]), math.atan2(u[1], u[0])
        Y = oracle.sh_basis(d, 3)
        for l in range(4):
            for m in range(-l, l + 1):
                c = sph_harm_y(l, abs(m), polar, azim)
                if m > 0:
                    ref = math.sqrt(2) * c.real
                elif m < 0:
                    ref = math.sqrt(2) * c.imag
                else:
                    ref = c.real
                assert Y[l * l + l + m] == pytest.approx(ref, abs=1e-12), (l, m)


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) times a uniform rule in phi integrates
    # products of degree <= 6 exactly: the Gram matrix must be the identity.
    nt, nphi = 12, 16
    xs, ws = np.polynomial.legendre.leggauss(nt)
    G = np.zeros((16, 16))
    for ct, w in zip(xs, ws):
        st = math.sqrt(1 - ct * ct)
        for k in range(nphi):
            ph = 2 * math.pi * k / nphi
            Y = oracle.sh_basis(np.array([st * math.cos(ph), st * math.sin(ph), ct]), 3)
            G += w * (2 * math.pi / nphi) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_degree0_colour_and_degree3_reduction():
    rng = np.random.default_rng(3)
    dc = rng.normal(size=3)
    g0 = one_gaussian((0.1, -0.2, 3.0), [-3.0] * 3, sh=[dc], degree=0)
    sh3 = np.zeros((16, 3))
    sh3[0] = dc
    g3 = one_gaussian((0.1, -0.2, 3.0), [-3.0] * 3, sh=sh3, degree=3)
    cam = ident_cam()
    a, b = oracle.project(g0, cam), oracle.project(g3, cam)
    dc32 = np.float32(dc).astype(np.float64)
    np.testing.assert_allclose(a["rgb"][0], np.maximum(0, 0.5 + dc32 / (2 * math.sqrt(math.pi))), rtol=1e-14)
    np.testing.assert_allclose(a["rgb"][0], b["rgb"][0], rtol=1e-14)


def test_sh_colour_uses_view_direction_and_clamps():
    # Degree 1 with only the z coefficient: colour = max(0, 0.5 + c * Y_10(d)).
    sh = np.zeros((4, 3))
    sh[2] = [1.0, -1.0, 3.0]
    g = one_gaussian((0.0, 0.0, 2.0), [-3.0] * 3, sh=sh, degree=1)
    p = oracle.project(g, ident_cam())
    c1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(p["rgb"][0], [0.5 + c1, max(0.0, 0.5 - c1), 0.5 + 3 * c1], rtol=1e-7)


def test_visibility_rules():
    cam = ident_cam()
    assert oracle.project(one_gaussian((0, 0, 0.005), [-3] * 3), cam)["flags"][0] & 1 == 0  # before znear
    assert oracle.project(one_gaussian((0, 0, -1.0), [-3] * 3), cam)["flags"][0] & 1 == 0   # behind
    assert oracle.project(one_gaussian((0, 0, 2), [-3] * 3, quat=(0, 0, 0, 0)), cam)["flags"][0] & 1 == 0
    assert oracle.project(one_gaussian((np.nan, 0, 2), [-3] * 3), cam)["flags"][0] & 1 == 0
    # opacity below 1/255 can never pass the alpha test
    assert oracle.project(one_gaussian((0, 0, 2), [-3] * 3, logit=-5.6), cam)["flags"][0] & 1 == 0
    assert oracle.project(one_gaussian((0, 0, 2), [-3] * 3, logit=-5.5), cam)["flags"][0] & 1 == 1
    # far outside the image
    assert oracle.project(one_gaussian((5.0, 0, 2), [-3] * 3), cam)["flags"][0] & 1 == 0


def test_footprint_covers_alpha_support():
    # The opacity-aware rect must contain every pixel where alpha >= 1/255:
    # for a large splat, check the tiles of all such pixels (evaluated from the
    # closed-form isotropic image) lie inside the rect.
    s, z, f = 0.2, 3.0, 100.0
    g = one_gaussian((0.11, -0.07, z), [math.log(s)] * 3, logit=2.0)
    p = oracle.project(g, ident_cam(f, 128, 128))
    sig2 = (f * math.exp(float(np.float32(math.log(s)))) / z) ** 2 + 0.3
    o = 1 / (1 + math.exp(-2.0))
    mx, my = p["mean2d"][0]
    x0, y0, x1, y1 = p["rect"][0]
    ys, xs = np.mgrid[0:128, 0:128] + 0.5
    a = o * np.exp(-0.5 * ((xs - mx) ** 2 + (ys - my) ** 2) / sig2)
    yy, xx = np.nonzero(a >= 1 / 255)
    assert len(xx) > 100
    assert (xx // 16).min() >= x0 and (xx // 16).max() < x1
    assert (yy // 16).min() >= y0 and (yy // 16).max() < y1


@pytest.mark.parametrize("side", [1.0, -1.0])
@pytest.mark.parametrize("axis", [0, 1])
def test_frustum_guard_closed_form(side, axis):
    # The 3DGS frustum guard clamps x/z (and y/z) of the Jacobian's centre to
    # 1.3 tan(half FOV) = 1.3 W / (2 f) with a centred principal point. For
    # an isotropic Gaussian (Sigma_cam = s^2 I) at (u z, 0, z):
    #   Sigma'_00 = s^2 (f/z)^2 (1 + c^2) + 0.3,  Sigma'_01 = 0,
    #   Sigma'_11 = s^2 (f/z)^2 + 0.3,
    # with c = u inside the guard and c = +-1.3 W / (2 f) beyond it (swap the
    # roles for the y axis). Gaussians 1.25x and 1.35x the half FOV off axis
    # sit on the two sides of the limit; a guard of another width (such as
    # the image edge plus 30 % of the whole width, 1.6 W / (2 f)) fails the
    # second case.
    f, W, H, z, s = 100.0, 64, 48, 3.0, 0.05
    cam = scenes.camera(np.eye(3), np.zeros(3), f, f, W / 2.0, H / 2.0, W, H)
    half = (W if axis == 0 else H) / (2.0 * f)
    s32 = math.exp(float(np.float32(math.log(s))))
    k = (f / z) ** 2 * s32 * s32
    for frac, clamped in ((1.25, False), (1.35, True), (3.0, True)):
        mean = [0.0, 0.0, z]
        mean[axis] = side * frac * half * z
        mu = np.array(mean, np.float32)
        p = oracle.project(one_gaussian(mu, [math.log(s)] * 3), cam)
        u = float(mu[axis]) / float(mu[2])
        c = side * 1.3 * half if clamped else u
        along, across = k * (1.0 + c * c) + 0.3, k + 0.3
        want = [along, 0.0, across] if axis == 0 else [across, 0.0, along]
        np.testing.assert_allclose(p["cov2d"][0], want, rtol=1e-12, atol=1e-12)
        # the screen position is never clamped
        np.testing.assert_allclose(p["mean2d"][0][axis], f * u + (W if axis == 0 else H) / 2.0, rtol=1e-12)


def test_frustum_guard_off_centre_principal_point():
    # With an off-centre principal point the guard is asymmetric: x/z is
    # clamped to (W - cx)/fx + 0.3 W/(2 fx) on the right and to
    # -(cx/fx + 0.3 W/(2 fx)) on the left (the gsplat form of the guard, equal
    # to +-1.3 W/(2 fx) when cx = W/2).
    fx, W, H, cx, z, s = 80.0, 64, 64, 20.0, 2.0, 0.04
    cam = scenes.camera(np.eye(3), np.zeros(3), fx, fx, cx, 32.0, W, H)
    s32 = math.exp(float(np.float32(math.log(s))))
    k = (fx / z) ** 2 * s32 * s32
    right = (W - cx) / fx + 0.3 * W / (2 * fx)   # 0.67
    left = cx / fx + 0.3 * W / (2 * fx)          # 0.37
    for u, clamped in ((0.6, False), (0.8, True), (-0.3, False), (-0.5, True)):
        mu = np.array([u * z, 0.0, z], np.float32)
        p = oracle.project(one_gaussian(mu, [math.log(s)] * 3), cam)
        c = (right if u > 0 else -left) if clamped else float(mu[0]) / float(mu[2])
        np.testing.assert_allclose(p["cov2d"][0], [k * (1 + c * c) + 0.3, 0.0, k + 0.3], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("ts", [8, 16, 32])
def test_three_sigma_footprint_closed_form(ts):
    # THREE_SIGMA: the tiles meeting the square of half side
    # r = ceil(3 sqrt(lambda_max)) around the mean. For an on-axis isotropic
    # Gaussian Sigma' = (f sigma / z)^2 I + 0.3 I, so lambda_max = the
    # diagonal value v when v^2 - det = 0 < 0.1, i.e. lambda_max = v +
    # sqrt(0.1): the 0.1 floor of the baseline's eigenvalue formula.
    # The principal point puts the mean half a pixel right of a tile
    # boundary plus r, so a radius one pixel smaller (no 0.1 floor, or a
    # 2.9-sigma rule) moves the rect's first column.
    f, W, H, z = 100.0, 96, 64, 3.0
    for s in (0.02, 0.05, 0.2):
        s32 = math.exp(float(np.float32(math.log(s))))
        v = (f * s32 / z) ** 2 + 0.3
        r = math.ceil(3.0 * math.sqrt(v + math.sqrt(0.1)))
        cx, cy = 32.0 + r - 0.5, H / 2.0
        cam = scenes.camera(np.eye(3), np.zeros(3), f, f, cx, cy, W, H)
        g = one_gaussian((0.0, 0.0, z), [math.log(s)] * 3)
        p = oracle.project(g, cam, tile_size=ts, footprint="three_sigma")
        tx, ty = (W + ts - 1) // ts, (H + ts - 1) // ts
        want = [max(0, math.floor((cx - r) / ts)), max(0, math.floor((cy - r) / ts)),
                min(tx, math.floor((cx + r) / ts) + 1), min(ty, math.floor((cy + r) / ts) + 1)]
        assert list(p["rect"][0]) == want, (s, r)
        assert p["flags"][0] & oracle.VISIBLE


def test_three_sigma_footprint_no_opacity_cut_and_truncation():
    # no opacity cut: o < 1/255 still gets its 3-sigma tiles (and never
    # passes the alpha test); an opaque Gaussian (o = 0.99: alpha support
    # out to sqrt(2 ln(255 o)) = 3.3 sigma) is cut at its 3-sigma tiles,
    # while the opacity-aware rect reaches every pixel of its support
    f, W, H, z, s = 100.0, 128, 128, 3.0, 0.2
    cam = ident_cam(f, W, H)
    faint = one_gaussian((0.0, 0.0, z), [math.log(s)] * 3, logit=-7.0)
    pf = oracle.project(faint, cam, footprint="three_sigma")
    assert pf["flags"][0] & oracle.VISIBLE and pf["opacity"][0] < 1 / 255
    assert not (oracle.project(faint, cam)["flags"][0] & oracle.VISIBLE)
    img = oracle.render(pf, W, H)
    assert img["alpha"].max() == 0.0 and img["nvisit"].max() == 1
    # mean at pixel (69.5, 69.5): the 3-sigma square (half side 21) starts
    # just inside tile 3, the alpha support (3.3 sigma = 22.2 px) in tile 2
    off = (69.5 - 64.0) * z / f
    opaque = one_gaussian((off, off, z), [math.log(s)] * 3, logit=math.log(0.99 / 0.01))
    p3 = oracle.project(opaque, cam, tile_size=16, footprint="three_sigma")
    po = oracle.project(opaque, cam, tile_size=16)
    x0, y0, x1, y1 = p3["rect"][0]
    ox0, oy0, ox1, oy1 = po["rect"][0]
    assert ox0 < x0 and oy0 < y0 and ox1 == x1  # the alpha support reaches tiles the square does not
    a3 = oracle.render(p3, W, H)["alpha"]
    ao = oracle.render(po, W, H)["alpha"]
    inside = np.zeros((H, W), bool)
    inside[y0 * 16:y1 * 16, x0 * 16:x1 * 16] = True
    assert np.array_equal(a3[inside], ao[inside])
    assert a3[~inside].max() == 0.0 and ao[~inside].max() > 1 / 255
