"""Pins of the front-end oracle (sec. 7.1, sec. 7.2, appendix on covariance
propagation), CPU only.

The covariance maps are checked against finite differences of the pose
compositions themselves (rotation exponential and logarithm from scipy), so a
wrong sign, a transposed rotation or a missing skew term fails; the tracking
policy is checked on short rendered sequences whose switch points follow from
the geometry."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth
from oracle import frontend as fe


def _rand_pose(rng, ang=0.6, tr=1.0):
    R = Rotation.from_rotvec(rng.normal(size=3) * ang).as_matrix()
    return R, rng.normal(size=3) * tr


def _left(T, d):
    """Left perturbation of the appendix: t + dt, exp(dtheta) R."""
    R, t = T
    return Rotation.from_rotvec(d[3:]).as_matrix() @ R, t + d[:3]


def _left_delta(T0, T1):
    """(dt, dtheta) with T1 = left perturbation of T0."""
    dth = Rotation.from_matrix(T1[0] @ T0[0].T).as_rotvec()
    return np.concatenate([T1[1] - T0[1], dth])


def _fd_jacobian(f, T, eps=1e-6):
    base = f(T)
    J = np.zeros((6, 6))
    for i in range(6):
        d = np.zeros(6)
        d[i] = eps
        dp = _left_delta(base, f(_left(T, d)))
        d[i] = -eps
        dm = _left_delta(base, f(_left(T, d)))
        J[:, i] = (dp - dm) / (2 * eps)
    return J


def test_compose_inverse_against_4x4():
    rng = np.random.default_rng(3)
    a, b = _rand_pose(rng), _rand_pose(rng)

    def m(T):
        M = np.eye(4)
        M[:3, :3], M[:3, 3] = T
        return M

    c = fe.compose(a, b)
    assert np.allclose(m(c), m(a) @ m(b), atol=1e-14)
    assert np.allclose(m(fe.inverse(a)), np.linalg.inv(m(a)), atol=1e-13)


def test_relative_covariance_jacobians_by_finite_differences():
    rng = np.random.default_rng(11)
    Twa, Twb = _rand_pose(rng), _rand_pose(rng)
    # Jacobians of T_A^B = (T_W^A)^-1 T_W^B w.r.t. left perturbations of each
    Ja = _fd_jacobian(lambda T: fe.compose(fe.inverse(T), Twb), Twa)
    Jb = _fd_jacobian(lambda T: fe.compose(fe.inverse(Twa), T), Twb)
    Sa = rng.normal(size=(6, 6))
    Sa = Sa @ Sa.T
    Sb = rng.normal(size=(6, 6))
    Sb = Sb @ Sb.T
    want = Ja @ Sa @ Ja.T + Jb @ Sb @ Jb.T
    got = fe.relative_covariance(Twa, Sa, Twb, Sb)
    assert np.allclose(got, want, rtol=1e-6, atol=1e-6 * np.abs(want).max())


def test_relative_covariance_monte_carlo():
    """Sampled left perturbations of both poses, composed exactly: the sample
    covariance of the composed perturbation matches to first order."""
    rng = np.random.default_rng(5)
    Twa, Twb = _rand_pose(rng), _rand_pose(rng)
    L = np.diag([2e-3, 1e-3, 3e-3, 1e-3, 2e-3, 1.5e-3])
    Sa = L @ L.T
    Sb = 0.5 * Sa
    base = fe.compose(fe.inverse(Twa), Twb)
    n = 40000
    da = rng.normal(size=(n, 6)) @ L.T
    db = rng.normal(size=(n, 6)) @ (L.T * math.sqrt(0.5))
    out = np.array([_left_delta(base, fe.compose(fe.inverse(_left(Twa, da[i])), _left(Twb, db[i])))
                    for i in range(n)])
    emp = np.cov(out.T)
    want = fe.relative_covariance(Twa, Sa, Twb, Sb)
    scale = np.sqrt(np.outer(np.diag(want), np.diag(want)))
    assert np.all(np.abs(emp - want) <= 0.05 * scale)


def test_xi_to_left_against_update():
    """The alignment's update T <- exp(xi)^-1 T (sec. 6.2) is, to first
    order, the left perturbation M xi."""
    rng = np.random.default_rng(8)
    R, t = _rand_pose(rng)
    M = fe.xi_to_left((R, t))
    eps = 1e-6
    for i in range(6):
        xi = np.zeros(6)
        xi[i] = eps
        Rp, tp = oracle.update(R, t, xi)
        xi[i] = -eps
        Rm, tm = oracle.update(R, t, xi)
        col = (_left_delta((R, t), (Rp, tp)) - _left_delta((R, t), (Rm, tm))) / (2 * eps)
        assert np.allclose(col, M[:, i], atol=1e-8)


def _walk(n, step_deg, step_m, seed):
    return synth.track_sequence(n, step_deg, step_m, seed=seed)


def test_tracker_recovers_constant_velocity_walk_and_switches():
    cam, poses, frames = _walk(9, 3.0, 0.04, seed=4)
    p = fe.TrackerParams(align=oracle.Params(levels=3, iters=[8, 8, 8]), rf_threshold=0.85,
                         kf_threshold=0.7, covis_level=1, buffer=4, covariance=True)
    trk = fe.Tracker(cam, p)
    outs = [trk.track(f.I, f.W) for f in frames]
    P0 = poses[0]
    for k, o in enumerate(outs):
        truth = fe.compose(fe.inverse(P0), poses[k])
        R, t = o["T_w_k"]
        rot = np.linalg.norm(Rotation.from_matrix(R.T @ truth[0]).as_rotvec())
        assert rot < 2e-3 and np.linalg.norm(t - truth[1]) < 5e-3, (k, rot)
        if k:
            # the odometry constraint is consistent with the absolute poses
            prev = outs[k - 1]["T_w_k"]
            od = fe.compose(fe.inverse(prev), o["T_w_k"])
            assert np.allclose(od[0], o["T_prev_k"][0], atol=1e-12)
            assert np.allclose(od[1], o["T_prev_k"][1], atol=1e-12)
            assert np.all(np.linalg.eigvalsh(o["S_odo"]) > 0)
    # covisibility falls monotonically with the distance to the reference
    # until a switch; 3 deg + 4 cm per frame makes at least one of each
    assert any(o["rf_switched"] for o in outs)
    assert any(o["kf_switched"] for o in outs)
    for o in outs[1:]:
        assert o["rf_switched"] == (o["covis_rf"] < p.rf_threshold)
        assert o["kf_switched"] == (o["covis_kf"] < p.kf_threshold)
    # after a keyframe switch the buffered frames are fused one per frame
    ks = [k for k, o in enumerate(outs) if o["kf_switched"]]
    if ks and ks[0] + 1 < len(outs) and not outs[ks[0] + 1]["kf_switched"]:
        assert outs[ks[0] + 1]["n_fused_buffer"] > 0


def test_tracker_static_camera_never_switches():
    cam, poses, frames = _walk(4, 0.0, 0.0, seed=2)
    trk = fe.Tracker(cam, fe.TrackerParams(align=oracle.Params(levels=2, iters=[5, 5]),
                                           covis_level=1, covariance=False))
    outs = [trk.track(f.I, f.W) for f in frames]
    for o in outs[1:]:
        assert not o["rf_switched"] and not o["kf_switched"]
        assert o["covis_rf"] > 0.95
        assert np.linalg.norm(o["T_w_k"][1]) < 1e-3
    # every frame after the first is fused into the keyframe: C grows by one
    # per frame on pixels seen in all frames
    assert np.median(trk.Ckf[trk.Wkf > 0]) > len(frames) - 0.5
