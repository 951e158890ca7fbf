"""FP64 oracle of the tracking front-end (sec. 7.1, sec. 7.2, sec. 6.4,
appendix on covariance propagation).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Composes the oracle's
alignment, covisibility ratio, fusion and covariance in the order the paper's
front-end runs them; everything here is plain numpy on 4x4 / 6x6 matrices.

Poses are (R, t) with X_A = R X_B + t for the pose T_A^B of B in A.
Covariances are over the left perturbation (dt, dtheta) of the appendix:
t -> t + dt, R -> exp(dtheta) R, translation first.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import Params, align, covariance, covisibility_ratio, fuse, pyramid, camera_level


def compose(a, b):
    """T_A^C = T_A^B T_B^C."""
    Ra, ta = a
    Rb, tb = b
    return Ra @ Rb, Ra @ tb + ta


def inverse(a):
    R, t = a
    return R.T, -R.T @ t


def identity():
    return np.eye(3), np.zeros(3)


def skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def xi_to_left(T):
    """Map M from the alignment's twist xi = (v, theta), whose update is
    T <- exp(xi)^-1 T (sec. 6.2), to the appendix's left perturbation of T:
    to first order dtheta = -theta and dt = -v + [t]x theta."""
    _, t = T
    M = np.zeros((6, 6))
    M[:3, :3] = -np.eye(3)
    M[:3, 3:] = skew(t)
    M[3:, 3:] = -np.eye(3)
    return M


def relative_covariance(T_wa, S_wa, T_wb, S_wb):
    """Covariance of T_A^B = (T_W^A)^-1 T_W^B from those of T_W^A and T_W^B
    (appendix on covariance propagation): the two first-order Jacobians with
    respect to left perturbations of each factor, applied as J S J^T."""
    Ra, ta = T_wa
    _, tb = T_wb
    Ja = np.zeros((6, 6))
    Ja[:3, :3] = Ra.T
    Ja[:3, 3:] = Ra.T @ skew(ta - tb)
    Ja[3:, 3:] = Ra.T
    Ja = -Ja
    Jb = np.zeros((6, 6))
    Jb[:3, :3] = Ra.T
    Jb[3:, 3:] = Ra.T
    return Ja @ S_wa @ Ja.T + Jb @ S_wb @ Jb.T


@dataclass
class TrackerParams:
    align: Params = field(default_factory=lambda: Params(levels=4, iters=[10] * 4))
    rf_threshold: float = 0.8     # reference-frame switch (above the keyframe one)
    kf_threshold: float = 0.7     # keyframe switch (sec. 7.2)
    covis_level: int = 2
    tol_sigmas: float = 3.0       # occlusion test of sec. 6.4
    buffer: int = 8               # pre-keyframe frame buffer
    covariance: bool = True


class Tracker:
    """Frame-to-reference tracking with a constant-velocity initial guess,
    covisibility-driven reference and keyframe switching, keyframe fusion of
    every frame and of the buffered frames recorded before the keyframe
    (sec. 7.1, sec. 7.2)."""

    def __init__(self, cam, params: TrackerParams = None):
        self.cam = cam
        self.p = params or TrackerParams()
        self.k = -1

    def _frame(self, I, W):
        return dict(I=np.asarray(I, np.float64), W=np.asarray(W, np.float64))

    def _ratio(self, A, B, T, tol):
        l = self.p.covis_level
        cl = camera_level(self.cam, l)
        st = self.p.align.storage
        pa = pyramid(self.cam, l + 1, A["I"], A["W"], storage=st)
        pb = pyramid(self.cam, l + 1, B["I"], B["W"], storage=st)
        r, _ = covisibility_ratio(cl, pa[l][1], pb[l][1], T[0], T[1], tol)
        return r

    def track(self, I, W):
        p = self.p
        self.k += 1
        F = self._frame(I, W)
        out = dict(k=self.k, rf_switched=False, kf_switched=False, n_fused=0, n_fused_buffer=0)
        if self.k == 0:
            self.rf, self.T_w_rf = F, identity()
            self.kf_frame, self.T_w_kf = F, identity()
            self.Wkf, self.Ckf = F["W"].copy(), np.ones_like(F["W"])
            self.T_rf_prev, self.S_rf_prev = identity(), np.zeros((6, 6))
            self.T_prev2_prev = identity()
            self.pending, self.recorded = [], []
            out.update(T_w_k=identity(), T_rf_k=identity(), T_prev_k=identity(),
                       S_rf_k=np.zeros((6, 6)), S_odo=np.zeros((6, 6)), covis_rf=1.0,
                       covis_kf=1.0, status=0)
            return out
        # constant-velocity initial guess (sec. 7.1)
        init = compose(self.T_rf_prev, self.T_prev2_prev)
        R, t, st = align(self.cam, self.rf["I"], self.rf["W"], F["I"], F["W"], p.align,
                         R0=init[0], t0=init[1])
        T_rf_k = (R, t)
        tol = p.tol_sigmas * st["sigma_W"]
        S_rf_k = np.zeros((6, 6))
        S_odo = np.zeros((6, 6))
        if p.covariance:
            S, _ = covariance(self.cam, self.rf["I"], self.rf["W"], F["I"], F["W"], R, t, p.align)
            M = xi_to_left(T_rf_k)
            S_rf_k = M @ S @ M.T
            S_odo = relative_covariance(self.T_rf_prev, self.S_rf_prev, T_rf_k, S_rf_k)
        T_prev_k = compose(inverse(self.T_rf_prev), T_rf_k)
        T_w_k = compose(self.T_w_rf, T_rf_k)
        # keyframe: switch or fuse (sec. 7.2)
        T_kf_k = compose(inverse(self.T_w_kf), T_w_k)
        c_kf = self._ratio(self.kf_frame, F, T_kf_k, tol)
        if c_kf < p.kf_threshold:
            out["kf_switched"] = True
            self.kf_frame, self.T_w_kf = F, T_w_k
            self.Wkf, self.Ckf = F["W"].copy(), np.ones_like(F["W"])
            # frames recorded with the previous keyframe, most recent first
            self.pending = list(reversed(self.recorded[-p.buffer:])) if p.buffer else []
            self.recorded = []
        else:
            self.Wkf, self.Ckf, n = fuse(self.cam, self.Wkf, self.Ckf, F["W"], *T_kf_k, tol)
            out["n_fused"] = n
            if self.pending:
                Wj, T_w_j, tol_j = self.pending.pop(0)
                T_kf_j = compose(inverse(self.T_w_kf), T_w_j)
                self.Wkf, self.Ckf, n = fuse(self.cam, self.Wkf, self.Ckf, Wj, *T_kf_j, tol_j)
                out["n_fused_buffer"] = n
        self.recorded.append((F["W"], T_w_k, tol))
        # reference frame (sec. 7.1 with the criterion of sec. 7.2)
        c_rf = self._ratio(self.rf, F, T_rf_k, tol)
        out.update(T_w_k=T_w_k, T_rf_k=T_rf_k, T_prev_k=T_prev_k, S_rf_k=S_rf_k, S_odo=S_odo,
                   covis_rf=c_rf, covis_kf=c_kf, status=st["status"], stats=st)
        self.T_prev2_prev = T_prev_k
        if c_rf < p.rf_threshold:
            out["rf_switched"] = True
            self.rf, self.T_w_rf = F, T_w_k
            self.T_rf_prev, self.S_rf_prev = identity(), np.zeros((6, 6))
        else:
            self.T_rf_prev, self.S_rf_prev = T_rf_k, S_rf_k
        return out
