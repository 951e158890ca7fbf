"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms
on analytic scenes, finite differences of an independently written projection,
library routines (scipy rotations, numpy solve / lstsq, scipy digamma, numpy
float16), brute force on tiny images, and exact recovery of a known rigid
motion.  Nothing here needs a GPU.
"""
import math

import numpy as np
import pytest
from scipy.ndimage import gaussian_filter
from scipy.spatial.transform import Rotation
from scipy.special import digamma as sp_digamma

import oracle

CAM160 = (160, 120, 131.25, 131.25, 79.5, 59.5)
CAM640 = (640, 480, 525.0, 525.0, 319.5, 239.5)


def plane_field(cam, n, d):
    """Inverse depth of the plane n.X = d seen by a camera at the origin:
    W(p) = n.K^-1 p / d, which is linear in the pixel coordinates."""
    w, h, fx, fy, cx, cy = cam
    v, u = np.mgrid[0:h, 0:w].astype(np.float64)
    return (n[0] * (u - cx) / fx + n[1] * (v - cy) / fy + n[2]) / d


def smooth_texture(rng, h, w, sigma=2.0):
    return gaussian_filter(rng.uniform(0, 255, size=(h, w)), sigma) * 4.0 - 384.0


# ----------------------------------------------------------------- camera / pyramid


def test_level_camera_of_640_is_160_camera():
    # Level 2 of the 640x480 Kinect-like camera is the 160x120 camera.
    assert oracle.camera_level(CAM640, 2) == pytest.approx(CAM160, abs=0)


@pytest.mark.parametrize("levels", [4])
def test_pyramid_planar_closed_form(levels):
    # The 2x2 mean of a field linear in p is its value at the block centre, so
    # every level of a planar inverse-depth map equals n.K_l^-1 p / d.
    n = np.array([0.2, -0.1, 1.0]) / np.linalg.norm([0.2, -0.1, 1.0])
    d = 2.3
    W0 = plane_field(CAM640, n, d)
    I0 = np.full_like(W0, 77.0)
    pyr = oracle.pyramid(CAM640, levels, I0, W0, storage="f64")
    for l, (Il, Wl) in enumerate(pyr):
        cl = oracle.camera_level(CAM640, l)
        ref = plane_field(cl, n, d)
        assert Wl.shape == ref.shape == (480 >> l, 640 >> l)
        np.testing.assert_allclose(Wl, ref, rtol=1e-13, atol=0)
        assert np.all(Il == 77.0)


def test_downsample_brute_force_with_holes():
    rng = np.random.default_rng(3)
    I = rng.uniform(0, 255, size=(6, 9))
    W = rng.uniform(0.2, 2.0, size=(6, 9))
    W[rng.uniform(size=W.shape) < 0.4] = 0.0
    W[0, 0] = W[0, 1] = W[1, 0] = W[1, 1] = 0.0      # an all-hole block
    W[2, 2] = np.nan                                   # non-finite is a hole
    I2, W2 = oracle.downsample(I, W)
    assert I2.shape == (3, 4)
    for v in range(3):
        for u in range(4):
            blk_i = [I[2 * v, 2 * u], I[2 * v, 2 * u + 1], I[2 * v + 1, 2 * u], I[2 * v + 1, 2 * u + 1]]
            blk_w = [W[2 * v, 2 * u], W[2 * v, 2 * u + 1], W[2 * v + 1, 2 * u], W[2 * v + 1, 2 * u + 1]]
            good = [x for x in blk_w if np.isfinite(x) and x > 0]
            assert I2[v, u] == pytest.approx(sum(blk_i) / 4, rel=1e-15)
            assert W2[v, u] == (pytest.approx(sum(good) / len(good), rel=1e-15) if good else 0.0)
    assert W2[0, 0] == 0.0


def test_round_f16_matches_numpy():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(0, 3, 2000), rng.uniform(0, 255, 2000),
                        10.0 ** rng.uniform(-8, 4.8, 2000), [0.0, 65504.0, 65519.0, 65520.0]])
    ours = np.array([oracle.round_f16(v) for v in x])
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(ours, ref)


# ----------------------------------------------------------------- SO(3) / SE(3)


def test_exp_log_against_scipy():
    rng = np.random.default_rng(1)
    for _ in range(50):
        ax = rng.normal(size=3)
        th = ax / np.linalg.norm(ax) * rng.uniform(0, 3.0)     # |theta| < pi
        R = oracle.exp_so3(th)
        np.testing.assert_allclose(R, Rotation.from_rotvec(th).as_matrix(), atol=1e-14)
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-14)
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-14)
        np.testing.assert_allclose(oracle.log_so3(R), th, atol=1e-12)
    tiny = np.array([3e-10, -1e-9, 2e-9])
    np.testing.assert_allclose(oracle.exp_so3(tiny), Rotation.from_rotvec(tiny).as_matrix(),
                               atol=1e-17)


def test_update_is_inverse_exp_times_T():
    # T <- exp(xi)^-1 T with the decoupled exp(xi) = [Rot(theta), v].
    rng = np.random.default_rng(2)
    R = Rotation.from_rotvec(rng.normal(size=3) * 0.3).as_matrix()
    t = rng.normal(size=3)
    xi = rng.normal(size=6) * 0.1
    E = np.eye(4)
    E[:3, :3] = Rotation.from_rotvec(xi[3:]).as_matrix()
    E[:3, 3] = xi[:3]
    T = np.eye(4)
    T[:3, :3], T[:3, 3] = R, t
    ref = np.linalg.inv(E) @ T
    R2, t2 = oracle.update(R, t, xi)
    np.testing.assert_allclose(R2, ref[:3, :3], atol=1e-14)
    np.testing.assert_allclose(t2, ref[:3, 3], atol=1e-14)


def test_solve_against_numpy():
    rng = np.random.default_rng(4)
    A = rng.normal(size=(40, 6))
    H = A.T @ A
    g = rng.normal(size=6)
    np.testing.assert_allclose(oracle.solve(H, g), np.linalg.solve(H, -g), rtol=1e-12)
    Hs = H.copy()
    Hs[:, 5] = Hs[5, :] = 0.0          # singular direction
    assert oracle.solve(Hs, g) is None
    assert oracle.solve(np.zeros((6, 6)), g) is None


# ----------------------------------------------------------------- warp


def test_warp_identity_reproduces_A():
    rng = np.random.default_rng(5)
    w, h = 40, 30
    cam = (w, h, 50.0, 50.0, 19.5, 14.5)
    I = rng.uniform(0, 255, (h, w))
    W = rng.uniform(0.3, 1.5, (h, w))
    W[rng.uniform(size=W.shape) < 0.1] = 0.0
    Iw, Ww, V = oracle.warp(cam, W, I, W, np.eye(3), np.zeros(3))
    assert V.sum() > 0.6 * w * h
    np.testing.assert_allclose(Iw[V], I[V], rtol=1e-12)
    np.testing.assert_allclose(Ww[V], W[V], rtol=1e-12)
    # a pixel whose 3x3 neighbourhood is hole-free must be warp-valid
    ok = np.ones_like(V)
    for dv in (-1, 0, 1):
        for du in (-1, 0, 1):
            ok &= np.roll(np.roll(W > 0, dv, 0), du, 1)
    ok[0, :] = ok[-1, :] = ok[:, 0] = ok[:, -1] = False
    assert np.all(V[ok])
    assert not np.any(V[W == 0])


@pytest.mark.parametrize("shift", [-0.25, 0.25])
def test_warp_clamped_taps_at_the_image_edge(shift):
    # A fronto-parallel plane at depth 1 and a translation along x move every
    # projection by `shift` pixels along u.  I_B = a + b u + c v is linear, so
    # inside the image the bilinear sample is the line at u + shift; where
    # u + shift falls in [-0.5, 0) or [w - 1, w - 0.5) both taps are clamped
    # to the edge column and the sample is that column's value (sec. 5.3
    # bounds, clamped taps): no extrapolation and no zero padding.
    w, h = 16, 12
    fx = 20.0
    cam = (w, h, fx, fx, 7.5, 5.5)
    u, v = np.meshgrid(np.arange(w, dtype=float), np.arange(h, dtype=float))
    a, b, c = 40.0, 3.0, 1.5
    IB = a + b * u + c * v
    ones = np.ones((h, w))
    t = np.array([-shift / fx, 0.0, 0.0])
    Iw, Ww, V = oracle.warp(cam, ones, IB, ones, np.eye(3), t)
    ub = u + shift
    want = a + b * np.clip(ub, 0.0, w - 1.0) + c * v
    assert np.all(V)
    np.testing.assert_allclose(Iw, want, rtol=0, atol=1e-9)
    np.testing.assert_allclose(Ww, ones, rtol=0, atol=1e-12)
    edge = (ub < 0.0) | (ub > w - 1.0)
    assert edge.sum() == h    # one column at the edge the shift points to


def test_warp_pure_z_translation_closed_form():
    # W_B constant and I_B linear in u: W* = W_B / (1 + W_B t_z) and
    # I*(u) = I_B(u_B) with u_B = cx + (u - cx) Z0 / (Z0 - t_z).
    w, h = 64, 48
    cam = (w, h, 60.0, 60.0, 31.5, 23.5)
    Z0, tz, WBc = 2.0, 0.07, 0.61
    WA = np.full((h, w), 1.0 / Z0)
    WB = np.full((h, w), WBc)
    v, u = np.mgrid[0:h, 0:w].astype(float)
    IB = 3.0 * u + 10.0
    Iw, Ww, V = oracle.warp(cam, WA, IB, WB, np.eye(3), np.array([0.0, 0.0, tz]))
    ub = 31.5 + (u - 31.5) * Z0 / (Z0 - tz)
    vb = 23.5 + (v - 23.5) * Z0 / (Z0 - tz)
    inb = (ub >= -0.5) & (ub < w - 0.5) & (vb >= -0.5) & (vb < h - 0.5)
    np.testing.assert_array_equal(V, inb)
    np.testing.assert_allclose(Ww[V], WBc / (1 + WBc * tz), rtol=1e-14)
    # bilinear on a ramp is exact away from the clamped border taps
    core = V & (ub >= 0) & (ub <= w - 1)
    np.testing.assert_allclose(Iw[core], 3.0 * ub[core] + 10.0, rtol=1e-12)


def test_warp_planar_scene_true_pose_gives_WA():
    # For consistent planar geometry the printed W_B* formula is exact:
    # warping W_B at the true pose returns W_A (and W_B is linear in p, so the
    # bilinear sample is exact).
    rng = np.random.default_rng(6)
    cam = CAM160
    n = np.array([0.15, -0.2, 1.0])
    n /= np.linalg.norm(n)
    d = 1.7
    R = Rotation.from_rotvec(rng.normal(size=3) * 0.02).as_matrix()
    t = rng.normal(size=3) * 0.03
    WA = plane_field(cam, n, d)
    # X_A = R X_B + t: in B the plane is (R^T n).X_B = d - n.t
    WB = plane_field(cam, R.T @ n, d - n @ t)
    I = np.zeros_like(WA)
    Iw, Ww, V = oracle.warp(cam, WA, I, WB, R, t)
    assert V.sum() > 0.8 * WA.size
    # bilinear is exact on a linear field except where the taps are clamped
    w, h, fx, fy, cx, cy = cam
    v, u = np.mgrid[0:h, 0:w].astype(float)
    X = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], -1) / WA[..., None]
    Y = (X - t) @ R
    ub = fx * Y[..., 0] / Y[..., 2] + cx
    vb = fy * Y[..., 1] / Y[..., 2] + cy
    core = V & (ub >= 0) & (ub <= w - 1) & (vb >= 0) & (vb <= h - 1)
    assert core.sum() > 0.8 * WA.size
    np.testing.assert_allclose(Ww[core], WA[core], rtol=1e-12)


def test_warp_fullres_downsample_strict_rule():
    rng = np.random.default_rng(7)
    w, h = 32, 24
    cam = (w, h, 30.0, 30.0, 15.5, 11.5)
    IB = rng.uniform(0, 255, (h, w))
    WB = rng.uniform(0.4, 1.2, (h, w))
    WA = WB.copy()
    WA[5, 7] = 0.0
    I0, W0, V0 = oracle.warp(cam, WA, IB, WB, np.eye(3), np.zeros(3))
    for level in (1, 2):
        Il, Wl, Vl = oracle.warp_fullres(cam, level, WA, IB, WB, np.eye(3), np.zeros(3))
        b = 1 << level
        for v in range(h >> level):
            for u in range(w >> level):
                blk = (slice(v * b, (v + 1) * b), slice(u * b, (u + 1) * b))
                assert Vl[v, u] == V0[blk].all()
                if Vl[v, u]:
                    assert Il[v, u] == pytest.approx(I0[blk].mean(), rel=1e-13)
                    assert Wl[v, u] == pytest.approx(W0[blk].mean(), rel=1e-13)
    _, _, V1 = oracle.warp_fullres(cam, 1, WA, IB, WB, np.eye(3), np.zeros(3))
    assert not V1[5 // 2, 7 // 2]


# ----------------------------------------------------------------- Jacobians, lambda_n


def _project(cam, X):
    w, h, fx, fy, cx, cy = cam
    return np.array([fx * X[0] / X[2] + cx, fy * X[1] / X[2] + cy])


def _moved(X, xi):
    # exp(xi) X with the decoupled exponential (scipy rotation, own code path)
    return Rotation.from_rotvec(xi[3:]).as_matrix() @ X + xi[:3]


def test_intensity_jacobian_matches_finite_differences():
    # With a ramp image the gradient is exact, so J_I = grad I . d(p')/d(xi)
    # where p' = pi(exp(xi) X_A) is the flow of the linearised constraint.
    cam = CAM160
    w, h, fx, fy, cx, cy = cam
    v, u = np.mgrid[0:h, 0:w].astype(float)
    gu, gv = 1.7, -0.6
    IA = gu * u + gv * v + 30.0
    n = np.array([0.1, 0.3, 1.0])
    n /= np.linalg.norm(n)
    WA = plane_field(cam, n, 2.0)
    res = oracle.residuals(cam, IA, WA, IA, WA, np.ones_like(WA, dtype=bool))
    eps = 1e-6
    for (pu, pv) in [(10, 7), (80, 60), (150, 100), (33, 90)]:
        X = np.array([(pu - cx) / fx, (pv - cy) / fy, 1.0]) / WA[pv, pu]
        J = np.zeros(6)
        for k in range(6):
            e = np.zeros(6)
            e[k] = eps
            dp = (_project(cam, _moved(X, e)) - _project(cam, _moved(X, -e))) / (2 * eps)
            J[k] = gu * dp[0] + gv * dp[1]
        np.testing.assert_allclose(res["JI"][pv, pu], J, rtol=1e-7, atol=1e-7 * np.abs(J).max())


def test_depth_jacobian_matches_finite_differences():
    # Inverse-depth constraint W_B(p + dp)(1 + W_A e_z.dX) - W_A with W_B = W_A
    # a planar (linear) field: its xi-derivative at 0 is the printed J_W.
    cam = CAM160
    w, h, fx, fy, cx, cy = cam
    n = np.array([-0.2, 0.25, 1.0])
    n /= np.linalg.norm(n)
    d = 1.8
    WA = plane_field(cam, n, d)
    IA = np.zeros_like(WA)
    res = oracle.residuals(cam, IA, WA, IA, WA, np.ones_like(WA, dtype=bool))

    def field(q):
        return (n[0] * (q[0] - cx) / fx + n[1] * (q[1] - cy) / fy + n[2]) / d

    eps = 1e-6
    for (pu, pv) in [(12, 9), (80, 60), (140, 30), (40, 110)]:
        wa = WA[pv, pu]
        X = np.array([(pu - cx) / fx, (pv - cy) / fy, 1.0]) / wa

        def F(xi):
            Xm = _moved(X, xi)
            return field(_project(cam, Xm)) * (1.0 + wa * (Xm[2] - X[2])) - wa

        J = np.array([(F(np.eye(6)[k] * eps) - F(-np.eye(6)[k] * eps)) / (2 * eps)
                      for k in range(6)])
        np.testing.assert_allclose(res["JW"][pv, pu], J, rtol=1e-6, atol=1e-7 * np.abs(J).max())
        assert res["rW"][pv, pu] == 0.0 and res["vW"][pv, pu]


def test_lambda_n_is_cosine_of_incidence():
    # For a plane with unit normal n, lambda_n = |n.x| / |x|, the cosine of the
    # angle between the viewing ray and the surface normal; fronto-parallel at
    # the principal point gives exactly 1.
    cam = (41, 31, 40.0, 40.0, 20.0, 15.0)
    for nvec in ([0.0, 0.0, 1.0], [0.3, -0.4, 1.0], [0.9, 0.1, 0.5]):
        n = np.array(nvec) / np.linalg.norm(nvec)
        WA = plane_field(cam, n, 2.0)
        ok = WA > 0
        res = oracle.residuals(cam, np.zeros_like(WA), np.where(ok, WA, 0), np.zeros_like(WA),
                               np.where(ok, WA, 0), ok)
        v, u = np.mgrid[0:31, 0:41].astype(float)
        x = np.stack([(u - 20.0) / 40.0, (v - 15.0) / 40.0, np.ones_like(u)], -1)
        ref = np.abs(x @ n) / np.linalg.norm(x, axis=-1)
        m = res["vW"]
        assert m.sum() > 100
        np.testing.assert_allclose(res["lam"][m], ref[m], rtol=1e-12)
        if nvec == [0.0, 0.0, 1.0]:
            assert res["lam"][15, 20] == 1.0


def test_residual_validity_rules():
    rng = np.random.default_rng(8)
    cam = (20, 16, 20.0, 20.0, 9.5, 7.5)
    IA = rng.uniform(0, 255, (16, 20))
    WA = rng.uniform(0.5, 1.0, (16, 20))
    WA[8, 8] = 0.0
    wv = np.ones_like(WA, dtype=bool)
    wv[4, 4] = False
    res = oracle.residuals(cam, IA, WA, IA, WA, wv)
    assert not res["vI"][0].any() and not res["vI"][:, -1].any()      # borders
    assert not res["vI"][8, 8] and not res["vI"][4, 4]                 # hole / no warp
    assert res["vI"][8, 9] and not res["vW"][8, 9]                     # grad W needs neighbours
    assert res["vW"][3, 3]
    assert np.all(res["vW"] <= res["vI"])


# ----------------------------------------------------------------- robust statistics


def test_digamma_against_scipy():
    for x in [0.05, 0.5, 1.0, 1.5, 2.5, 3.0, 5.5, 6.0, 7.25, 20.0, 123.4]:
        assert oracle.digamma(x) == pytest.approx(sp_digamma(x), abs=1e-13, rel=1e-13)


def test_weights():
    assert oracle.omega("student_t", 0.0, 5.0) == pytest.approx(6.0 / 5.0)
    assert oracle.omega("student_t", 2.0, 3.0) == pytest.approx(4.0 / 7.0)
    assert oracle.omega("huber", 1.0) == 1.0
    assert oracle.omega("huber", -2.69, k=1.345) == pytest.approx(0.5)


@pytest.mark.parametrize("kind", ["huber", "student_t"])
def test_scale_satisfies_stationarity(kind):
    # sec. 6.3: sum w (r - mu) = 0 and sum (1 - w (r-mu)^2 / sigma^2) = 0 at
    # the solution (weights evaluated at the solution).
    rng = np.random.default_rng(9)
    r = rng.standard_t(4, size=5000) * 3.0 + 0.7
    mu, sg = oracle.scale(r, kind=kind, nu=5.0, iters=300, floor=1e-9)
    x = (r - mu) / sg
    wts = np.array([oracle.omega(kind, xi, 5.0) for xi in x])
    assert abs(np.sum(wts * (r - mu))) / len(r) < 1e-9
    assert abs(np.sum(1.0 - wts * x * x)) / len(r) < 1e-9


def test_scale_unit_weights_is_mean_and_variance():
    rng = np.random.default_rng(10)
    r = rng.normal(2.0, 3.0, size=1000)
    mu, sg = oracle.scale(r, kind="huber", k=1e9, iters=3, floor=0.0)
    assert mu == pytest.approx(r.mean(), rel=1e-13)
    assert sg == pytest.approx(r.std(), rel=1e-12)


@pytest.mark.parametrize("kind", ["huber", "student_t"])
def test_scale_convergence_stop_meets_stationarity(kind):
    # The convergence stop (the step that moves mu and sigma by at most
    # tol sigma is the last) leaves the two stationarity equations of sec. 6.3
    # satisfied to about tol: the next step would move mu by
    # sum w (r - mu) / sum w and sigma^2 by sigma^2 (sum w x^2 / n - 1).
    rng = np.random.default_rng(12)
    r = rng.standard_t(4, size=5000) * 3.0 + 0.7
    tol = oracle.SCALE_TOL
    for start in (None, (2.0, 9.0), (-1.0, 0.5)):
        mu, sg = oracle.scale(r, kind=kind, nu=5.0, iters=300, floor=1e-9, start=start, tol=tol)
        x = (r - mu) / sg
        wts = np.array([oracle.omega(kind, xi, 5.0) for xi in x])
        assert abs(np.sum(wts * (r - mu)) / np.sum(wts)) <= 2 * tol * sg
        assert abs(np.mean(wts * x * x) - 1.0) <= 4 * tol


@pytest.mark.parametrize("kind", ["huber", "student_t"])
def test_scale_warm_start_reaches_the_cold_fixed_point(kind):
    # The fixed point does not depend on where the iteration starts: warm
    # starts near and far from it end within a few tol of the cold start run
    # to exact convergence, and a start at the fixed point stops after one
    # step that leaves it there.
    rng = np.random.default_rng(13)
    r = np.concatenate([rng.normal(0.3, 2.0, size=4000), rng.normal(0.0, 25.0, size=600)])
    mu0, sg0 = oracle.scale(r, kind=kind, iters=1000, floor=1e-9)
    tol = oracle.SCALE_TOL
    for start in ((mu0, sg0), (mu0 + 0.5, 1.3 * sg0), (-3.0, 0.2 * sg0), (0.0, 40.0)):
        mu, sg = oracle.scale(r, kind=kind, iters=300, floor=1e-9, start=start, tol=tol)
        assert abs(mu - mu0) <= 4 * tol * sg0 and abs(sg - sg0) <= 4 * tol * sg0
    mu, sg = oracle.scale(r, kind=kind, iters=1, floor=1e-9, start=(mu0, sg0), tol=tol)
    assert abs(mu - mu0) <= 1e-12 * sg0 and abs(sg - sg0) <= 1e-12 * sg0
    # tol = 0 keeps the fixed number of steps: 3 steps from a far start are
    # still far from the fixed point
    mu, sg = oracle.scale(r, kind=kind, iters=3, floor=1e-9, start=(0.0, 40.0), tol=0.0)
    assert abs(sg - sg0) > 1e-3 * sg0


def test_align_scale_warm_start_same_optimum():
    # Warm-started scale (default) and the cold fixed schedule reach the same
    # Gauss-Newton optimum on a converging pair (weights agree to about 1e-6).
    import synth
    p = synth.pair_c1(0)
    kw = dict(levels=3, iters=[8, 8, 8], weight="huber")
    Rw, tw, sw_ = oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, oracle.Params(**kw))
    Rc, tc, sc = oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W,
                              oracle.Params(scale_warm=False, **kw))
    assert sw_["status"] == sc["status"] == 0
    assert np.linalg.norm(oracle.log_so3(Rw.T @ Rc)) < 1e-7
    assert np.linalg.norm(tw - tc) < 1e-7
    assert abs(sw_["sigma_I"] - sc["sigma_I"]) <= 1e-5 * sc["sigma_I"]
    assert abs(sw_["sigma_W"] - sc["sigma_W"]) <= 1e-5 * sc["sigma_W"]


def test_scale_floor_and_empty():
    mu, sg = oracle.scale(np.zeros(50), kind="huber", floor=1e-3)
    assert mu == 0.0 and sg == 1e-3
    assert oracle.scale(np.zeros(0), floor=1e-6) == (0.0, 1e-6)


def test_nu_estimate():
    rng = np.random.default_rng(11)
    # root of the nu equation when inside (2, 10); decreasing in nu
    r = rng.standard_t(4, size=20000)
    mu, sg = oracle.scale(r, kind="student_t", nu=5.0, iters=50, floor=1e-9)
    nu = oracle.estimate_nu(r, mu, sg)
    assert 2.0 < nu < 10.0
    assert abs(oracle.nu_equation(r, mu, sg, nu)) < 1e-3 * len(r) * 1e-3
    # bracketing: the likelihood rises at nu = 2 and falls at nu = 10, and the
    # bisection ends on the sign change
    assert oracle.nu_equation(r, mu, sg, 2.0) > 0 > oracle.nu_equation(r, mu, sg, 10.0)
    assert oracle.nu_equation(r, mu, sg, nu - 1e-6) > 0 > oracle.nu_equation(r, mu, sg, nu + 1e-6)
    # heavy tails -> small nu, Gaussian -> clamps at 10
    r3 = rng.standard_t(2.2, size=20000)
    m3, s3 = oracle.scale(r3, kind="student_t", iters=50, floor=1e-9)
    assert oracle.estimate_nu(r3, m3, s3) < nu
    rg = rng.normal(size=20000)
    mg, sgg = oracle.scale(rg, kind="student_t", iters=50, floor=1e-9)
    assert oracle.estimate_nu(rg, mg, sgg) == 10.0


@pytest.mark.parametrize("df", [3.0, 4.0, 6.0])
def test_nu_estimate_is_student_t_likelihood_argmax(df):
    # The nu equation of sec. 6.3 is twice the derivative in nu of the
    # Student-t log-likelihood with location and scale held at (mu, sigma).
    # Its bisection root must therefore be the argmax over [2, 10] of the
    # summed scipy.stats.t log-density, found here by bounded Brent search on
    # that library function (no digamma, no oracle arithmetic).  A wrong
    # factor on the data-free digamma/log term, or on the per-sample term,
    # moves the root by far more than 1e-6.
    from scipy.optimize import minimize_scalar
    from scipy.stats import t as student_t
    rng = np.random.default_rng(int(df * 10))
    r = 0.7 + 2.5 * rng.standard_t(df, size=20000)
    mu, sg = oracle.scale(r, kind="student_t", nu=5.0, iters=50, floor=1e-9)
    nu = oracle.estimate_nu(r, mu, sg)
    nll = lambda v: -float(np.sum(student_t.logpdf(r, df=v, loc=mu, scale=sg)))
    best = minimize_scalar(nll, bounds=(2.0, 10.0), method="bounded",
                           options={"xatol": 1e-10, "maxiter": 500})
    assert 2.0 < best.x < 10.0
    assert nu == pytest.approx(best.x, abs=1e-6)


def test_nu_estimate_clamps_where_likelihood_is_monotone():
    # Gaussian residuals: the likelihood still rises at nu = 10, so nu = 10;
    # very heavy tails (t with 1.2 degrees of freedom): it already falls at
    # nu = 2, so nu = 2.  Checked on the scipy log-density, not the oracle.
    from scipy.stats import t as student_t
    rng = np.random.default_rng(5)
    for r, want in ((rng.normal(size=20000), 10.0), (rng.standard_t(1.2, size=20000), 2.0)):
        mu, sg = oracle.scale(r, kind="student_t", nu=5.0, iters=50, floor=1e-9)
        ll = lambda v: float(np.sum(student_t.logpdf(r, df=v, loc=mu, scale=sg)))
        grid = [ll(v) for v in np.linspace(2.0, 10.0, 17)]
        if want == 10.0:
            assert all(b > a for a, b in zip(grid, grid[1:]))
        else:
            assert all(b < a for a, b in zip(grid, grid[1:]))
        assert oracle.estimate_nu(r, mu, sg) == want


def test_sample_strides():
    # N = 19200 gives integer strides over the 640x480 pyramid (sec. 6.3).
    assert [oracle.sample_stride(640 >> l, 480 >> l) for l in range(4)] == [4, 2, 1, 1]
    assert oracle.sample_stride(1280, 960) == 8
    assert oracle.sample_stride(320, 240) == 2
    assert oracle.sample_stride(160, 120) == 1
    # the sample never exceeds N, also for sizes that are not 640x480 multiples
    for w, h in [(300, 250), (641, 481), (139, 139), (1000, 20), (7, 5)]:
        s = oracle.sample_stride(w, h)
        assert -(-w // s) * -(-h // s) <= 19200
        assert s == 1 or -(-w // (s - 1)) * -(-h // (s - 1)) > 19200
    for l in range(3):
        s = oracle.sample_stride(640 >> l, 480 >> l)
        assert len(range(0, 640 >> l, s)) * len(range(0, 480 >> l, s)) == 19200


@pytest.mark.slow
def test_sample_precision_claim():
    # sec. 6.3 claims a 0.03 relative precision of the scale from the
    # systematic 19200-sample at 99.7% confidence.
    rng = np.random.default_rng(12)
    fails = 0
    for _ in range(40):
        r = rng.standard_t(5, size=(480, 640)) * 2.0
        mu_s, s_s = oracle.scale(r[::4, ::4], kind="huber", floor=0)
        mu_a, s_a = oracle.scale(r, kind="huber", floor=0)
        fails += abs(s_s / s_a - 1) > 0.03
    assert fails == 0


# ----------------------------------------------------------------- normal equations


def test_normal_equations_solution_is_weighted_least_squares():
    # xi = -H^-1 g equals lstsq(sqrt(w) J, -sqrt(w) r) on the same residuals.
    rng = np.random.default_rng(13)
    w, h = 24, 18
    cam = (w, h, 22.0, 22.0, 11.5, 8.5)
    IA = smooth_texture(rng, h, w, 1.5)
    WA = rng.uniform(0.5, 0.8, (h, w))
    Iw = IA + rng.normal(0, 3, (h, w))
    Ww = WA + rng.normal(0, 0.01, (h, w))
    V = rng.uniform(size=(h, w)) > 0.1
    P = oracle.Params(levels=1, iters=[1], weight="huber")
    st = oracle.normal_equations(cam, IA, WA, Iw, Ww, V, P)
    res = oracle.residuals(cam, IA, WA, Iw, Ww, V)
    vI, vW = res["vI"], res["vW"]
    wI = np.array([oracle.omega("huber", (r - st["mu_I"]) / st["sigma_I"]) for r in res["rI"][vI]])
    wI /= st["sigma_I"] ** 2
    wW = np.array([oracle.omega("huber", (r - st["mu_W"]) / st["sigma_W"]) for r in res["rW"][vW]])
    wW *= res["lam"][vW] / st["sigma_W"] ** 2
    A = np.concatenate([np.sqrt(wI)[:, None] * res["JI"][vI], np.sqrt(wW)[:, None] * res["JW"][vW]])
    b = np.concatenate([np.sqrt(wI) * res["rI"][vI], np.sqrt(wW) * res["rW"][vW]])
    xi_ls = np.linalg.lstsq(A, -b, rcond=None)[0]
    np.testing.assert_allclose(oracle.solve(st["H"], st["g"]), xi_ls, rtol=1e-9, atol=1e-12)
    assert st["cost"] == pytest.approx(b @ b, rel=1e-12)
    assert st["n_valid_I"] == vI.sum() and st["n_valid_W"] == vW.sum()
    np.testing.assert_allclose(st["H"], st["H"].T, rtol=1e-14)


def test_zero_residual_at_identity_gives_zero_step():
    rng = np.random.default_rng(14)
    w, h = 48, 36
    cam = (w, h, 45.0, 45.0, 23.5, 17.5)
    I = smooth_texture(rng, h, w)
    W = rng.uniform(0.4, 1.0, (h, w))
    P = oracle.Params(levels=1, iters=[1], weight="huber", storage="f64")
    st = oracle.normal_equations_at(cam, I, W, I, W, 0, np.eye(3), np.zeros(3), P)
    xi = oracle.solve(st["H"], st["g"])
    assert np.abs(xi).max() < 1e-10


# ----------------------------------------------------------------- whole iteration


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("weight", ["huber", "student_t"])
def test_exact_recovery_of_shifted_plane(k, weight):
    # Fronto-parallel textured plane, B = A shifted by k pixels (both cropped
    # from one texture).  The true motion t = (k / (fx W), 0, 0), R = I has
    # zero residual on every included pixel; GN from identity recovers it.
    w, h, fx = 160, 120, 131.25
    cam = (w, h, fx, fx, 79.5, 59.5)
    rng = np.random.default_rng(20 + k)
    T = smooth_texture(rng, h, w + k)
    Z0 = 2.0
    Wc = np.full((h, w), 1.0 / Z0)
    P = oracle.Params(levels=1, iters=[30], weight=weight, storage="f64")
    R, t, st = oracle.align(cam, T[:, :w], Wc, T[:, k:k + w], Wc, P)
    assert st["status"] == 0
    np.testing.assert_allclose(t, [k * Z0 / fx, 0, 0], atol=1e-9)
    assert np.linalg.norm(oracle.log_so3(R)) < 1e-9


def test_exact_recovery_multilevel_rendered_planes():
    # Noiseless rendered three-plane pair at the c1 camera, 3 levels: the
    # estimate converges to the truth up to the rendering's crease and
    # supersampling error (measured ~1e-5 here; stated bound 1e-4).
    import synth
    p = synth.pair_c1(0, noise=False)
    P = oracle.Params(levels=3, iters=[15, 15, 15], weight="huber", storage="f64")
    R, t, st = oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, P)
    assert st["status"] == 0
    assert np.linalg.norm(oracle.log_so3(R.T @ p.R)) < 1e-4
    assert np.linalg.norm(t - p.t) < 1e-4


def test_degenerate_all_holes():
    w, h = 32, 24
    cam = (w, h, 30.0, 30.0, 15.5, 11.5)
    I = np.random.default_rng(0).uniform(0, 255, (h, w))
    W = np.zeros((h, w))
    P = oracle.Params(levels=1, iters=[5])
    R, t, st = oracle.align(cam, I, W, I, W, P)
    assert st["status"] == -5
    np.testing.assert_array_equal(R, np.eye(3))
    np.testing.assert_array_equal(t, np.zeros(3))


def test_initial_guess_is_used():
    import synth
    p = synth.pair_c1(1)
    P = oracle.Params(levels=1, iters=[0])
    R, t, st = oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, P, R0=p.R, t0=p.t)
    np.testing.assert_array_equal(R, p.R)
    np.testing.assert_array_equal(t, p.t)


# ----------------------------------------------------------------- fusion


def test_fuse_identity_same_map():
    rng = np.random.default_rng(15)
    cam = (30, 20, 25.0, 25.0, 14.5, 9.5)
    W = rng.uniform(0.3, 1.0, (20, 30))
    W[3, 4] = 0.0
    C = np.ones_like(W)
    W2, C2, n = oracle.fuse(cam, W, C, W, np.eye(3), np.zeros(3), tol=0.01)
    np.testing.assert_allclose(W2, W, rtol=1e-14)
    m = W > 0
    assert n > 0
    assert np.all((C2[m] == 2.0) | (C2[m] == 1.0))
    assert W2[3, 4] == 0.0 and C2[3, 4] == 1.0


def test_fuse_z_translation_weighted_mean():
    # Fronto-parallel keyframe at Z0, frames translated by t_z along the axis
    # with constant W_k: W* = W_k / (1 + W_k t_z), C_k = (1 + W_k t_z)^4, and
    # the fused map is the C-weighted mean (brute force).
    w, h = 40, 30
    cam = (w, h, 40.0, 40.0, 19.5, 14.5)
    Z0 = 2.0
    Wkf = np.full((h, w), 1.0 / Z0)
    Ckf = np.ones((h, w))
    frames = [(0.05, 1 / (Z0 - 0.05) + 0.002), (-0.03, 1 / (Z0 + 0.03) - 0.001),
              (0.02, 1 / (Z0 - 0.02))]
    num, den = Wkf[0, 0] * 1.0, 1.0
    for tz, wk in frames:
        Wk = np.full((h, w), wk)
        Wkf, Ckf, n = oracle.fuse(cam, Wkf, Ckf, Wk, np.eye(3), np.array([0, 0, tz]), tol=0.01)
        ck = (1 + wk * tz) ** 4
        num += ck * wk / (1 + wk * tz)
        den += ck
        assert n > 0.5 * w * h
    centre = (slice(10, 20), slice(12, 28))
    np.testing.assert_allclose(Wkf[centre], num / den, rtol=1e-14)
    np.testing.assert_allclose(Ckf[centre], den, rtol=1e-14)


def test_fuse_occluder_rejected():
    w, h = 40, 30
    cam = (w, h, 40.0, 40.0, 19.5, 14.5)
    Wkf = np.full((h, w), 0.5)
    Wk = np.full((h, w), 0.5)
    Wk[:, :20] = 1.5                        # something much closer in the frame
    W2, C2, n = oracle.fuse(cam, Wkf, np.ones((h, w)), Wk, np.eye(3), np.zeros(3), tol=0.01)
    assert np.all(C2[:, :19] == 1.0) and np.all(W2[:, :19] == 0.5)
    assert np.all(C2[:, 21:] == 2.0)


# ----------------------------------------------------------------- covisibility


def test_covisibility_identity_and_shift():
    # identity, B = A: every pixel with a valid 2x2 tap neighbourhood is visible
    w, h = 60, 40
    cam = (w, h, 50.0, 50.0, 29.5, 19.5)
    Z0 = 2.0
    W = np.full((h, w), 1.0 / Z0)
    nH, nV = oracle.covisibility(cam, W, W, np.eye(3), np.zeros(3), 0.01)
    assert nH == w * h and nV == w * h
    # fronto-parallel plane, B translated by k pixels along x: columns whose
    # transfer leaves the image are not visible (closed form: k columns)
    for k in (1, 3, 7):
        t = np.array([k * Z0 / 50.0, 0.0, 0.0])
        nH, nV = oracle.covisibility(cam, W, W, np.eye(3), t, 0.01)
        assert nH == w * h and nV == (w - k) * h
        r, counts = oracle.covisibility_ratio(cam, W, W, np.eye(3), t, 0.01)
        assert r == pytest.approx((w - k) / w)


def test_covisibility_occluder_and_holes():
    w, h = 40, 30
    cam = (w, h, 40.0, 40.0, 19.5, 14.5)
    WA = np.full((h, w), 0.5)
    WA[:5, :] = 0.0                      # holes are not in S_H
    WB = np.full((h, w), 0.5)
    WB[:, 30:] = 1.5                     # an occluder in B
    nH, nV = oracle.covisibility(cam, WA, WB, np.eye(3), np.zeros(3), 0.01)
    assert nH == (h - 5) * w
    assert nV == (h - 5) * 30           # columns 30.. see the occluder


# A plane n.X = d seen from the keyframe / reference camera, and a second
# camera with pose (R, t) in it (X_ref = R X_2 + t).  Inverse depth is linear
# in the pixel coordinates in both views, so bilinear sampling is exact and
# the geometry is consistent: every transferred pixel meets the other view's
# surface.  The transfer below is written independently of the oracle with
# explicit matrix products.
_ROT_CAM = (64, 48, 60.0, 60.0, 31.5, 23.5)
_ROT_N = np.array([0.12, -0.08, 1.0]) / np.linalg.norm([0.12, -0.08, 1.0])
_ROT_D = 2.0
_ROT_R = Rotation.from_rotvec(np.deg2rad(4.0) * np.array([0.3, 0.8, 0.5]) /
                              np.linalg.norm([0.3, 0.8, 0.5])).as_matrix()
_ROT_T = np.array([0.06, -0.035, 0.045])


def _second_view_plane(cam, n, d, R, t):
    """Inverse depth of the plane in the second camera: (R^T n).X_2 = d - n.t."""
    return plane_field(cam, R.T @ n, d - n @ t)


def _transfer(cam, W, R, t):
    """Pixel positions and 1/Y_z of every pixel of W in the second camera:
    Y = R^T (K^-1 p / W - t)."""
    w, h, fx, fy, cx, cy = cam
    v, u = np.mgrid[0:h, 0:w].astype(np.float64)
    ray = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], axis=-1)
    X = ray / W[..., None] - t
    Y = X @ R            # row vector times R = (R^T X^T)^T
    Rray = ray @ R
    ub = fx * Y[..., 0] / Y[..., 2] + cx
    vb = fy * Y[..., 1] / Y[..., 2] + cy
    return ub, vb, Y[..., 2], Rray[..., 2]


def _inside(cam, ub, vb):
    w, h = cam[:2]
    ins = (ub >= -0.5) & (ub < w - 0.5) & (vb >= -0.5) & (vb < h - 0.5)
    # no transfer within rounding of the bounds, so the count is well posed
    edge = np.minimum.reduce([np.abs(ub + 0.5), np.abs(ub - (w - 0.5)),
                              np.abs(vb + 0.5), np.abs(vb - (h - 0.5))])
    assert edge.min() > 1e-6
    return ins


def _plane_sample(cam, n, d, ub, vb):
    """Bilinear sample of a linear inverse-depth field with the taps clamped
    to the image: inside [0, w-1] x [0, h-1] it is the field itself; in the
    outer half-pixel band both taps of an axis are the edge pixel, so the
    field is taken at the clamped coordinate."""
    w, h, fx, fy, cx, cy = cam
    uc, vc = np.clip(ub, 0.0, w - 1.0), np.clip(vb, 0.0, h - 1.0)
    return (n[0] * (uc - cx) / fx + n[1] * (vc - cy) / fy + n[2]) / d


def _fuse_expected(cam, Wkf, Ckf, R, t, tol):
    """One fusion step of a consistent plane frame, in closed form: the
    covisibility decision |w_b - 1/Y_z| < tol, W* = (R^T x)_z w_b /
    (1 + w_b (R^T t)_z), C_k = ((1 + w_b (R^T t)_z)^2 / (R^T x)_z)^2 and the
    weighted mean."""
    ub, vb, Yz, Rz = _transfer(cam, Wkf, R, t)
    ins = _inside(cam, ub, vb) & (Yz > 0)
    wb = _plane_sample(cam, R.T @ _ROT_N, _ROT_D - _ROT_N @ t, ub, vb)
    gap = np.abs(wb - 1.0 / Yz)
    assert np.all(np.abs(gap[ins] - tol) > 1e-9)
    fused = ins & (gap < tol)
    den = 1.0 + wb * (R.T @ t)[2]
    Ws = Rz * wb / den
    Ck = (den * den / Rz) ** 2
    Wn = np.where(fused, (Wkf * Ckf + Ck * Ws) / (Ckf + Ck), Wkf)
    Cn = np.where(fused, Ckf + Ck, Ckf)
    interior = fused & (ub >= 0) & (ub <= cam[0] - 1) & (vb >= 0) & (vb <= cam[1] - 1)
    return Wn, Cn, fused, interior, Rz, Yz


def test_fuse_rotated_consistent_plane_closed_form():
    # R != I.  Where the transfer lands between pixel centres the bilinear
    # sample is exact, the geometry is consistent, and the warped inverse depth
    # equals the keyframe's own (W* = W_kf): W stays as it was and C grows by
    # C_k = ((R^T x)_z / (W_kf Y_z)^2)^2 (the weight of sec. 7.2 with
    # 1 + w_b (R^T t)_z = (R^T x)_z / (W_kf Y_z)).  In the outer half-pixel band
    # the clamped taps give the field at the clamped coordinate; that is
    # closed form too.  Fails with a transposed rotation in the transfer, in
    # (R^T x)_z or in R^T t.
    cam, tol = _ROT_CAM, 1e-3
    Wkf = plane_field(cam, _ROT_N, _ROT_D)
    Wk = _second_view_plane(cam, _ROT_N, _ROT_D, _ROT_R, _ROT_T)
    assert Wkf.min() > 0 and Wk.min() > 0
    Wn, Cn, fused, interior, Rz, Yz = _fuse_expected(cam, Wkf, np.ones_like(Wkf), _ROT_R,
                                                     _ROT_T, tol)
    assert 0.5 * fused.size < interior.sum() < fused.sum() < fused.size
    W2, C2, n = oracle.fuse(cam, Wkf, np.ones_like(Wkf), Wk, _ROT_R, _ROT_T, tol=tol)
    assert n == fused.sum()
    np.testing.assert_allclose(W2[interior], Wkf[interior], rtol=1e-13)
    np.testing.assert_allclose(C2[interior], 1.0 + (Rz / (Wkf * Yz) ** 2)[interior] ** 2,
                               rtol=1e-12)
    np.testing.assert_allclose(W2, Wn, rtol=1e-12)
    np.testing.assert_allclose(C2, Cn, rtol=1e-12)
    assert np.all(C2[~fused] == 1.0)
    # a second, different frame of the same plane on the fused map
    R2 = Rotation.from_rotvec([-0.03, 0.02, 0.05]).as_matrix()
    t2 = np.array([-0.04, 0.05, -0.02])
    Wk2 = _second_view_plane(cam, _ROT_N, _ROT_D, R2, t2)
    Wn2, Cn2, fused2, interior2, _, _ = _fuse_expected(cam, W2, C2, R2, t2, tol)
    W3, C3, n2 = oracle.fuse(cam, W2, C2, Wk2, R2, t2, tol=tol)
    assert n2 == fused2.sum() and interior2.sum() > 0.5 * fused2.size
    np.testing.assert_allclose(W3, Wn2, rtol=1e-12)
    np.testing.assert_allclose(C3, Cn2, rtol=1e-12)


def test_covisibility_rotated_plane_closed_form():
    # R != I on a consistent plane: a pixel is visible iff its transfer lands
    # inside the other image with the sampled inverse depth within tol of
    # 1/Y_z, which holds everywhere except possibly in the outer half-pixel
    # band (clamped taps).  Counted in each direction (B -> A with the inverse
    # pose).  A transposed rotation lands elsewhere and leaves the plane,
    # which fails these counts.
    cam, tol = _ROT_CAM, 1e-3
    WA = plane_field(cam, _ROT_N, _ROT_D)
    WB = _second_view_plane(cam, _ROT_N, _ROT_D, _ROT_R, _ROT_T)

    def visible(W, n, d, R, t):
        ub, vb, Yz, _ = _transfer(cam, W, R, t)
        ins = _inside(cam, ub, vb) & (Yz > 0)
        gap = np.abs(_plane_sample(cam, R.T @ n, d - n @ t, ub, vb) - 1.0 / Yz)
        assert np.all(np.abs(gap[ins] - tol) > 1e-9)
        return int((ins & (gap < tol)).sum())

    want_ab = visible(WA, _ROT_N, _ROT_D, _ROT_R, _ROT_T)
    # B's plane is (R^T n).X_B = d - n.t; A in B is (R^T, -R^T t)
    nB, dB = _ROT_R.T @ _ROT_N, _ROT_D - _ROT_N @ _ROT_T
    want_ba = visible(WB, nB, dB, _ROT_R.T, -_ROT_R.T @ _ROT_T)
    n = cam[0] * cam[1]
    assert 0.5 * n < want_ab < n and 0.5 * n < want_ba < n
    assert oracle.covisibility(cam, WA, WB, _ROT_R, _ROT_T, tol) == (n, want_ab)
    r, counts = oracle.covisibility_ratio(cam, WA, WB, _ROT_R, _ROT_T, tol)
    assert counts == (n, want_ab, n, want_ba)
    assert r == min(want_ab, want_ba) / n


# ----------------------------------------------------------------- covariance


def test_bilateral_reduces_to_gaussian_blur_and_keeps_edges():
    from scipy.ndimage import correlate
    rng = np.random.default_rng(30)
    I = rng.uniform(0, 255, (20, 24))
    W = rng.uniform(0.5, 0.6, (20, 24))
    # huge range sigmas: a normalised 5x5 Gaussian (library correlation, with
    # the weights renormalised over the in-image part of the window)
    Io, Wo = oracle.bilateral(I, W, 2, 1.5, 1e12, 1e12)
    d = np.arange(-2, 3)
    g = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2 * 1.5 ** 2))
    num = correlate(I, g, mode="constant")
    den = correlate(np.ones_like(I), g, mode="constant")
    np.testing.assert_allclose(Io, num / den, rtol=1e-12)
    # constant image stays constant; a step edge is kept with a small sigma
    C = np.full((10, 10), 7.0)
    np.testing.assert_allclose(oracle.bilateral(C, C * 0 + 0.5)[0], C, rtol=1e-14)
    S = np.where(np.arange(10)[None, :] < 5, 0.0, 200.0) * np.ones((10, 1))
    Wd = np.where(np.arange(10)[None, :] < 5, 0.5, 1.0) * np.ones((10, 1))
    So, Wdo = oracle.bilateral(S, Wd, 2, 1.5, 1.0, 0.01)
    np.testing.assert_allclose(So, S, atol=1e-9)
    np.testing.assert_allclose(Wdo, Wd, rtol=1e-9)
    # holes stay holes and are skipped
    Wh = W.copy()
    Wh[5, 5] = 0.0
    _, Who = oracle.bilateral(I, Wh)
    assert Who[5, 5] == 0.0 and np.all(Who[Wh > 0] > 0)


def test_covariance_is_inverse_of_filtered_hessian():
    import synth
    p = synth.pair_c1(2)
    P = oracle.Params(levels=1, iters=[1], storage="f64")
    S, st = oracle.covariance(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, p.R, p.t, P)
    np.testing.assert_allclose(S @ st["H"], np.eye(6), atol=1e-9)
    np.testing.assert_allclose(S, S.T, rtol=1e-9, atol=1e-20)
    assert np.all(np.linalg.eigvalsh(S) > 0)
    # the Hessian is that of the filtered reference at the given pose
    If, Wf = oracle.bilateral(p.A.I, p.A.W)
    st2 = oracle.normal_equations_at(p.cam, If, Wf, p.B.I, p.B.W, 0, p.R, p.t, P)
    np.testing.assert_allclose(st2["H"], st["H"], rtol=1e-12)
