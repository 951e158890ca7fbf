"""Pins of the sensor input path of the oracle (sec. 4.1, 4.2, 5.1, 5.2),
CPU only: hand-derived values of the Brown distortion, exact copies under
the identity, bilinear exactness on linear images, the depth-correction terms
one by one, the closed form of a registered fronto-parallel plane under a
general motion, occlusion by the greatest inverse depth, a brute-force
gather for the translation splat, and a two-camera rendering of one scene."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth


def _cam(w=40, h=30, f=35.0):
    return (w, h, f, f, (w - 1) / 2.0, (h - 1) / 2.0)


# ---------------------------------------------------------------- distortion


def test_distortion_radial_terms_on_an_axis():
    # on the x axis r = x, so each radial term adds k x^(2j+1) to x only
    x = 0.4
    for idx, power in ((0, 3), (1, 5), (4, 7)):
        k = [0.0] * 5
        k[idx] = 0.3
        xd, yd = oracle.distort(k, x, 0.0)
        assert xd == pytest.approx(x + 0.3 * x ** power, abs=1e-15) and yd == 0.0


def test_distortion_tangential_terms_on_the_axes():
    # k3 / k4 follow the decentring form: on (x, 0) k3 moves y by k3 x^2 and
    # k4 moves x by 3 k4 x^2; on (0, y) k3 moves y by 3 k3 y^2, k4 moves x by k4 y^2
    a = 0.05
    assert oracle.distort([0, 0, a, 0, 0], 0.5, 0.0) == pytest.approx((0.5, a * 0.25), abs=1e-15)
    assert oracle.distort([0, 0, 0, a, 0], 0.5, 0.0) == pytest.approx((0.5 + 3 * a * 0.25, 0.0), abs=1e-15)
    assert oracle.distort([0, 0, a, 0, 0], 0.0, 0.5) == pytest.approx((0.0, 0.5 + 3 * a * 0.25), abs=1e-15)
    assert oracle.distort([0, 0, 0, a, 0], 0.0, 0.5) == pytest.approx((a * 0.25, 0.5), abs=1e-15)


def test_radial_distortion_commutes_with_rotation_about_the_axis():
    rng = np.random.default_rng(1)
    k = [0.2, -0.05, 0.0, 0.0, 0.01]
    for _ in range(20):
        x, y = rng.uniform(-0.6, 0.6, size=2)
        ang = rng.uniform(0, 2 * np.pi)
        c, s = np.cos(ang), np.sin(ang)
        xd, yd = oracle.distort(k, x, y)
        xr, yr = oracle.distort(k, c * x - s * y, s * x + c * y)
        assert (xr, yr) == pytest.approx((c * xd - s * yd, s * xd + c * yd), abs=1e-14)


def test_undistort_identity_and_linear_image():
    cam = _cam()
    w, h = cam[:2]
    rng = np.random.default_rng(2)
    img = rng.uniform(0, 255, size=(h, w))
    assert np.array_equal(oracle.undistort(cam, [0.0] * 5, img, False), img)
    # bilinear interpolation of a linear image is exact wherever the sample
    # point is inside the image
    k = [0.08, -0.01, 0.004, -0.003, 0.0]
    vv, uu = np.mgrid[0:h, 0:w].astype(float)
    lin = 3.0 + 0.7 * uu - 1.3 * vv
    out = oracle.undistort(cam, k, lin, False)
    for v in range(h):
        for u in range(w):
            xd, yd = oracle.distort(k, (u - cam[4]) / cam[2], (v - cam[5]) / cam[3])
            x, y = cam[2] * xd + cam[4], cam[3] * yd + cam[5]
            if 1e-9 <= x <= w - 1 - 1e-9 and 0 <= y <= h - 1:
                assert out[v, u] == pytest.approx(3.0 + 0.7 * x - 1.3 * y, abs=1e-10)
            elif not (-0.5 <= x < w - 0.5 and -0.5 <= y < h - 0.5):
                assert out[v, u] == 0.0


def test_undistort_depth_needs_four_valid_taps():
    cam = _cam()
    w, h = cam[:2]
    W = np.full((h, w), 0.5)
    W[10, 12] = 0.0
    k = [0.05, 0.0, 0.0, 0.0, 0.0]
    out = oracle.undistort(cam, k, W, True)
    for v in range(h):
        for u in range(w):
            xd, yd = oracle.distort(k, (u - cam[4]) / cam[2], (v - cam[5]) / cam[3])
            x, y = cam[2] * xd + cam[4], cam[3] * yd + cam[5]
            if not (-0.5 <= x < w - 0.5 and -0.5 <= y < h - 0.5):
                assert out[v, u] == 0.0
                continue
            x0, y0 = int(np.floor(x)), int(np.floor(y))
            taps = {(min(max(x0 + i, 0), w - 1), min(max(y0 + j, 0), h - 1))
                    for i in (0, 1) for j in (0, 1)}
            if (12, 10) in taps:
                assert out[v, u] == 0.0
            else:
                assert out[v, u] == pytest.approx(0.5, abs=1e-15)


# ---------------------------------------------------------------- depth correction


def test_depth_correction_linear_and_shift():
    cam = _cam()
    w, h = cam[:2]
    rng = np.random.default_rng(3)
    Z = rng.uniform(0.5, 5.0, size=(h, w))
    Z[5, 7] = 0.0
    out = oracle.depth_correct(cam, Z, beta0=0.1, beta1=2.0, p0=(4, 4))
    assert np.all(out[:4, :] == 0) and np.all(out[:, :4] == 0)
    with np.errstate(divide="ignore"):
        want = 2.0 / Z[:-4, :-4] + 0.1
    want[5, 7] = 0.0
    np.testing.assert_allclose(out[4:, 4:], want, rtol=1e-15)
    # no shift, identity
    np.testing.assert_allclose(oracle.depth_correct(cam, Z, p0=(0, 0))[Z > 0], 1.0 / Z[Z > 0],
                               rtol=1e-15)


@pytest.mark.parametrize("j", range(9))
def test_depth_spatial_polynomial_terms(j):
    cam = _cam()
    Z = np.full((cam[1], cam[0]), 2.0)
    u, v = 31, 6
    mx, my = (u - cam[4]) / cam[2], (v - cam[5]) / cam[3]
    r2 = mx * mx + my * my
    terms = [1.0, r2, r2 ** 2, r2 ** 3, mx, my, mx * my, mx * mx * my, mx * my * my]
    q0 = [0.0] * 9
    q0[j] = 0.2
    out = oracle.depth_correct(cam, Z, p0=(0, 0), spatial=True, q0=q0)
    assert out[v, u] == pytest.approx(0.5 + 0.2 * terms[j], abs=1e-15)
    q1 = [0.0] * 9
    q1[j] = 1.5
    q1z = q1.copy()
    out = oracle.depth_correct(cam, Z, p0=(0, 0), spatial=True, q1=q1z)
    want = 1.5 * terms[j] * 0.5
    assert out[v, u] == pytest.approx(want if want > 0 else 0.0, abs=1e-15)


# ---------------------------------------------------------------- registration


def test_register_identity_is_exact():
    cam = _cam()
    rng = np.random.default_rng(4)
    W = rng.uniform(0.2, 2.0, size=(cam[1], cam[0]))
    W[rng.random(W.shape) < 0.1] = 0.0
    assert np.array_equal(oracle.register(cam, W, cam, np.eye(3), np.zeros(3)), W)


@pytest.mark.parametrize("tz", [0.0, 0.15, -0.2])
def test_register_fronto_parallel_plane_closed_form(tz):
    # plane Z_A = d: W_B(p) = e_z^T R K_B^-1 p / (d - t_z) exactly wherever the
    # nearest B_t pixel was covered
    camA = _cam(60, 45, 50.0)
    camB = (50, 40, 45.0, 46.0, 24.0, 20.5)
    d = 2.0
    WA = np.full((camA[1], camA[0]), 1.0 / d)
    R = Rotation.from_rotvec([0.02, -0.03, 0.01]).as_matrix()
    t = np.array([0.05, -0.03, tz])
    Wt = oracle.register_translate(camA, WA, t)
    inner = Wt[8:-8, 8:-8]      # moving back shrinks the image towards the centre
    assert np.all(inner == pytest.approx(1.0 / (d - tz), rel=1e-15))   # no holes (relief texture)
    WB = oracle.register_rotate(camA, Wt, camB, R)
    vv, uu = np.mgrid[0:camB[1], 0:camB[0]].astype(float)
    m = np.stack([(uu - camB[4]) / camB[2], (vv - camB[5]) / camB[3], np.ones_like(uu)])
    want = np.einsum("j,jhw->hw", R[2], m) / (d - tz)
    ok = WB > 0
    assert ok.mean() > 0.8
    np.testing.assert_allclose(WB[ok], want[ok], rtol=1e-13)


def test_register_occlusion_keeps_the_nearest_surface():
    cam = _cam(40, 30, 35.0)
    WA = np.full((30, 40), 0.25)          # wall at 4 m
    WA[:, 18:22] = 1.0                    # pole at 1 m
    t = np.array([0.3, 0.0, 0.0])         # sideways: the pole sweeps over the wall
    Wt = oracle.register_translate(cam, WA, t)
    # wall points move by -fx t_x W = -2.625 px, pole points by -10.5 px
    cols_pole = np.arange(18, 22) - 10.5
    for c in range(40):
        if cols_pole[0] - 0.5 <= c < cols_pole[-1] + 0.5:
            assert np.all(Wt[:, c] == 1.0)


def test_register_translate_brute_force_gather():
    cam = (12, 9, 10.0, 11.0, 5.3, 4.1)
    rng = np.random.default_rng(6)
    WA = rng.uniform(0.3, 1.5, size=(9, 12))
    WA[rng.random(WA.shape) < 0.15] = 0.0
    t = np.array([0.12, -0.08, 0.3])
    got = oracle.register_translate(cam, WA, t)
    tx = cam[2] * t[0] + cam[4] * t[2]
    ty = cam[3] * t[1] + cam[5] * t[2]
    want = np.zeros_like(WA)
    for qy in range(9):
        for qx in range(12):
            best = 0.0
            for v in range(9):
                for u in range(12):
                    W = WA[v, u]
                    if W <= 0:
                        continue
                    den = 1 - W * t[2]
                    if den <= 0:
                        continue
                    x, y, half = (u - W * tx) / den, (v - W * ty) / den, 0.5 / den
                    if x - half <= qx < x + half and y - half <= qy < y + half:
                        best = max(best, W / den)
            want[qy, qx] = best
    np.testing.assert_array_equal(got, want)


def test_preprocess_two_camera_rendering():
    # depth and colour cameras 2.5 cm apart looking at one room scene: the
    # registered corrected depth agrees with the colour camera's own render
    # except within a pixel of depth discontinuities
    scene = synth.room_scene(11)
    depth = synth.Camera(160, 120, 130.0, 130.0, 79.5, 59.5)
    color = synth.Camera(160, 120, 131.25, 131.25, 80.0, 60.0)
    R_dc = Rotation.from_rotvec([0.0, 0.004, 0.0]).as_matrix()
    t_dc = np.array([0.025, 0.0, 0.0])
    pose_d = (Rotation.from_euler("x", -10, degrees=True).as_matrix(), np.zeros(3))
    pose_c = synth.compose(pose_d, (R_dc, t_dc))
    Zd, _ = synth.render(scene, depth, pose_d, ss=1)
    Zc, Ic = synth.render(scene, color, pose_c, ss=1)
    Zd = np.where(np.isfinite(Zd), Zd, 0.0)
    s = oracle.Sensor(color=color.as_tuple(), depth=depth.as_tuple(), p0=(0, 0),
                      R_dc=R_dc, t_dc=t_dc)
    Io, Wo = oracle.preprocess(s, Ic, Zd)
    assert np.array_equal(Io, Ic)
    Wc = np.where(np.isfinite(Zc) & (Zc > 0), 1.0 / np.where(Zc > 0, Zc, 1.0), 0.0)
    both = (Wo > 0) & (Wc > 0)
    assert both.mean() > 0.9
    rel = np.abs(Wo[both] - Wc[both]) / Wc[both]
    assert np.median(rel) < 2e-3 and np.mean(rel < 0.02) > 0.97
