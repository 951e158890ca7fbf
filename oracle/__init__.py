"""FP64 CPU oracle for RGBiD dense alignment and keyframe fusion.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  The HIP
library never loads it, and the two share no code: the oracle is plain C in
double precision (``rgbid_oracle.c``), compiled with gcc, wrapped here with
ctypes.  The convolutional warm-start network has its own FP64 numpy oracle
in ``cnn.py``.

Conventions: images are (h, w) row-major arrays; a hole in inverse depth is a
value <= 0 or non-finite; the pose (R, t) is the pose of B in A
(X_A = R X_B + t); twists are xi = (v, theta), translation first.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rgbid_oracle.c")
_LIB = os.path.join(_HERE, "_rgbid_oracle.so")

WEIGHTS = {"student_t": 0, "huber": 1}
WARPS = {"fullres": 0, "per_level": 1}
STORAGE = {"f64": 0, "f32": 1, "f16": 2}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cam(C.Structure):
    _fields_ = [("w", C.c_int), ("h", C.c_int), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("levels", C.c_int), ("iters", C.c_int * 8), ("weight", C.c_int),
                ("huber_k", C.c_double), ("estimate_nu", C.c_int),
                ("sample_max", C.c_int), ("scale_iters", C.c_int), ("warp", C.c_int),
                ("stop_eps_t", C.c_double), ("stop_eps_r", C.c_double),
                ("storage", C.c_int), ("scale_warm", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("H", C.c_double * 36), ("g", C.c_double * 6), ("mu_I", C.c_double),
                ("sigma_I", C.c_double), ("nu_I", C.c_double), ("mu_W", C.c_double),
                ("sigma_W", C.c_double), ("nu_W", C.c_double), ("cost", C.c_double),
                ("n_valid_I", C.c_longlong), ("n_valid_W", C.c_longlong),
                ("iters_done", C.c_int * 8), ("status", C.c_int)]


@dataclass
class Params:
    levels: int = 4
    iters: list = field(default_factory=lambda: [10] * 4)
    weight: str = "huber"
    huber_k: float = 1.345
    estimate_nu: bool = True
    sample_max: int = 19200
    scale_iters: int = 20
    warp: str = "fullres"
    stop_eps_t: float = 0.0
    stop_eps_r: float = 0.0
    storage: str = "f32"
    scale_warm: bool = True

    def _c(self) -> _Params:
        p = _Params()
        p.levels = self.levels
        its = list(self.iters) + [0] * (8 - len(self.iters))
        for i in range(8):
            p.iters[i] = its[i]
        p.weight = WEIGHTS[self.weight]
        p.huber_k = self.huber_k
        p.estimate_nu = int(self.estimate_nu)
        p.sample_max = self.sample_max
        p.scale_iters = self.scale_iters
        p.warp = WARPS[self.warp]
        p.stop_eps_t = self.stop_eps_t
        p.stop_eps_r = self.stop_eps_r
        p.storage = STORAGE[self.storage]
        p.scale_warm = int(self.scale_warm)
        return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        u8p = C.POINTER(C.c_uint8)
        cp = C.POINTER(_Cam)
        L.or_round_f16.restype = C.c_double
        L.or_round_f16.argtypes = [C.c_double]
        L.or_camera_level.argtypes = [cp, C.c_int, cp]
        L.or_downsample.argtypes = [dp, dp, C.c_int, C.c_int, dp, dp, C.c_int]
        L.or_exp_so3.argtypes = [dp, dp]
        L.or_log_so3.argtypes = [dp, dp]
        L.or_update.argtypes = [dp, dp, dp]
        L.or_warp.argtypes = [cp, dp, dp, dp, dp, dp, dp, dp, u8p]
        L.or_warp_fullres.argtypes = [cp, C.c_int, dp, dp, dp, dp, dp, dp, dp, u8p]
        L.or_residuals.argtypes = [cp, dp, dp, dp, dp, u8p, dp, dp, dp, dp, dp, u8p, u8p]
        L.or_omega.restype = C.c_double
        L.or_omega.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
        L.or_digamma.restype = C.c_double
        L.or_digamma.argtypes = [C.c_double]
        L.or_scale.argtypes = [dp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int,
                               C.c_double, dp, C.c_double, dp, dp]
        L.or_nu_equation.restype = C.c_double
        L.or_nu_equation.argtypes = [dp, C.c_int, C.c_double, C.c_double, C.c_double]
        L.or_estimate_nu.restype = C.c_double
        L.or_estimate_nu.argtypes = [dp, C.c_int, C.c_double, C.c_double]
        L.or_sample_stride.restype = C.c_int
        L.or_sample_stride.argtypes = [C.c_int, C.c_int, C.c_int]
        L.or_solve.restype = C.c_int
        L.or_solve.argtypes = [dp, dp, dp]
        L.or_normal_equations.argtypes = [cp, dp, dp, dp, dp, u8p, C.POINTER(_Params),
                                          C.c_void_p, C.POINTER(_Stats)]
        L.or_pyramid.argtypes = [cp, C.c_int, dp, dp, C.c_int, dp, dp]
        L.or_normal_equations_at.argtypes = [cp, C.c_int, dp, dp, dp, dp, C.c_int, dp, dp,
                                             C.POINTER(_Params), C.POINTER(_Stats)]
        L.or_align.restype = C.c_int
        L.or_align.argtypes = [cp, dp, dp, dp, dp, dp, dp, C.POINTER(_Params), dp, dp,
                               C.POINTER(_Stats)]
        L.or_covisibility.argtypes = [cp, dp, dp, dp, dp, C.c_double, C.POINTER(C.c_longlong),
                                      C.POINTER(C.c_longlong)]
        L.or_bilateral.argtypes = [dp, dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                   C.c_double, dp, dp]
        L.or_covariance.restype = C.c_int
        L.or_covariance.argtypes = [cp, C.c_int, dp, dp, dp, dp, dp, dp, C.POINTER(_Params),
                                    C.c_int, C.c_double, C.c_double, C.c_double, dp,
                                    C.POINTER(_Stats)]
        L.or_fuse.restype = C.c_longlong
        L.or_fuse.argtypes = [cp, dp, dp, dp, dp, dp, C.c_double]
        L.or_distort.argtypes = [dp, C.c_double, C.c_double, dp, dp]
        L.or_undistort.argtypes = [cp, dp, dp, C.c_int, dp]
        L.or_depth_correct.argtypes = [cp, dp, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                       dp, dp, dp]
        L.or_register_translate.argtypes = [cp, dp, dp, dp]
        L.or_register_rotate.argtypes = [cp, dp, cp, dp, dp]
        L.or_preprocess.argtypes = [cp, dp, cp, dp, C.c_double, C.c_double, C.c_int, C.c_int,
                                    C.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# helpers


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _pu8(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _cam(cam) -> _Cam:
    if isinstance(cam, _Cam):
        return cam
    w, h, fx, fy, cx, cy = cam.as_tuple() if hasattr(cam, "as_tuple") else cam
    return _Cam(int(w), int(h), float(fx), float(fy), float(cx), float(cy))


def _stats(st: _Stats) -> dict:
    return dict(H=np.array(st.H[:]).reshape(6, 6), g=np.array(st.g[:]),
                mu_I=st.mu_I, sigma_I=st.sigma_I, nu_I=st.nu_I, mu_W=st.mu_W,
                sigma_W=st.sigma_W, nu_W=st.nu_W, cost=st.cost,
                n_valid_I=st.n_valid_I, n_valid_W=st.n_valid_W,
                iters_done=list(st.iters_done[:]), status=st.status)


# --------------------------------------------------------------------------
# API


def round_f16(x: float) -> float:
    return lib().or_round_f16(float(x))


def camera_level(cam, l: int):
    out = _Cam()
    lib().or_camera_level(C.byref(_cam(cam)), int(l), C.byref(out))
    return (out.w, out.h, out.fx, out.fy, out.cx, out.cy)


def downsample(I, W, storage="f64"):
    I, W = _d(I), _d(W)
    h, w = I.shape
    I2 = np.zeros((h // 2, w // 2))
    W2 = np.zeros((h // 2, w // 2))
    lib().or_downsample(_p(I), _p(W), w, h, _p(I2), _p(W2), STORAGE[storage])
    return I2, W2


def pyramid(cam, levels: int, I0, W0, storage="f64"):
    I0, W0 = _d(I0), _d(W0)
    sizes = [camera_level(cam, l)[:2] for l in range(levels)]
    tot = sum(w * h for w, h in sizes)
    Io, Wo = np.zeros(tot), np.zeros(tot)
    lib().or_pyramid(C.byref(_cam(cam)), levels, _p(I0), _p(W0), STORAGE[storage],
                     _p(Io), _p(Wo))
    out, off = [], 0
    for w, h in sizes:
        out.append((Io[off:off + w * h].reshape(h, w), Wo[off:off + w * h].reshape(h, w)))
        off += w * h
    return out


def exp_so3(theta) -> np.ndarray:
    th = _d(theta)
    R = np.zeros(9)
    lib().or_exp_so3(_p(th), _p(R))
    return R.reshape(3, 3)


def log_so3(R) -> np.ndarray:
    R = _d(R).reshape(9)
    th = np.zeros(3)
    lib().or_log_so3(_p(R), _p(th))
    return th


def update(R, t, xi):
    R = _d(R).reshape(9).copy()
    t = _d(t).copy()
    lib().or_update(_p(R), _p(t), _p(_d(xi)))
    return R.reshape(3, 3), t


def warp(cam, WA, IB, WB, R, t):
    c = _cam(cam)
    WA, IB, WB = _d(WA), _d(IB), _d(WB)
    Iw, Ww = np.zeros_like(WA), np.zeros_like(WA)
    V = np.zeros(WA.shape, dtype=np.uint8)
    lib().or_warp(C.byref(c), _p(WA), _p(IB), _p(WB), _p(_d(R).reshape(9)), _p(_d(t)),
                  _p(Iw), _p(Ww), _pu8(V))
    return Iw, Ww, V.astype(bool)


def warp_fullres(cam0, level: int, WA0, IB0, WB0, R, t):
    c = _cam(cam0)
    w, h = camera_level(cam0, level)[:2]
    WA0, IB0, WB0 = _d(WA0), _d(IB0), _d(WB0)
    Iw, Ww = np.zeros((h, w)), np.zeros((h, w))
    V = np.zeros((h, w), dtype=np.uint8)
    lib().or_warp_fullres(C.byref(c), level, _p(WA0), _p(IB0), _p(WB0),
                          _p(_d(R).reshape(9)), _p(_d(t)), _p(Iw), _p(Ww), _pu8(V))
    return Iw, Ww, V.astype(bool)


def residuals(cam, IA, WA, Iw, Ww, valid):
    c = _cam(cam)
    IA, WA, Iw, Ww = _d(IA), _d(WA), _d(Iw), _d(Ww)
    V = np.ascontiguousarray(valid, dtype=np.uint8)
    h, w = IA.shape
    rI, rW, lam = np.zeros((h, w)), np.zeros((h, w)), np.zeros((h, w))
    JI, JW = np.zeros((h, w, 6)), np.zeros((h, w, 6))
    vI = np.zeros((h, w), dtype=np.uint8)
    vW = np.zeros((h, w), dtype=np.uint8)
    lib().or_residuals(C.byref(c), _p(IA), _p(WA), _p(Iw), _p(Ww), _pu8(V), _p(rI), _p(rW),
                       _p(JI), _p(JW), _p(lam), _pu8(vI), _pu8(vW))
    return dict(rI=rI, rW=rW, JI=JI, JW=JW, lam=lam, vI=vI.astype(bool), vW=vW.astype(bool))


def omega(kind: str, x: float, nu: float = 5.0, k: float = 1.345) -> float:
    return lib().or_omega(WEIGHTS[kind], float(x), float(nu), float(k))


def digamma(x: float) -> float:
    return lib().or_digamma(float(x))


# The convergence stop of the warm-started fixed point (fraction of sigma).
SCALE_TOL = 2.0 ** -16


def scale(r, kind="huber", nu=5.0, k=1.345, iters=20, floor=1e-3, start=None, tol=0.0):
    """mu, sigma by the fixed point of sec. 6.3: from start = (mu0, sigma0),
    else mu = 0, sigma^2 = mean r^2; at most `iters` steps, the step that moves
    both by at most tol * sigma the last."""
    r = _d(r).reshape(-1)
    mu, sg = C.c_double(), C.c_double()
    s0 = None if start is None else _d(start)
    st = None if s0 is None else _p(s0)
    lib().or_scale(_p(r), len(r), WEIGHTS[kind], nu, k, iters, floor, st, tol, C.byref(mu),
                   C.byref(sg))
    return mu.value, sg.value


def nu_equation(r, mu, sigma, nu):
    r = _d(r).reshape(-1)
    return lib().or_nu_equation(_p(r), len(r), mu, sigma, nu)


def estimate_nu(r, mu, sigma):
    r = _d(r).reshape(-1)
    return lib().or_estimate_nu(_p(r), len(r), mu, sigma)


def sample_stride(w: int, h: int, nmax: int = 19200) -> int:
    return lib().or_sample_stride(w, h, nmax)


def solve(H, g):
    H = _d(H).reshape(36)
    g = _d(g)
    xi = np.zeros(6)
    rc = lib().or_solve(_p(H), _p(g), _p(xi))
    return xi if rc == 0 else None


def normal_equations(cam, IA, WA, Iw, Ww, valid, params: Params = None):
    params = params or Params()
    c = _cam(cam)
    IA, WA, Iw, Ww = _d(IA), _d(WA), _d(Iw), _d(Ww)
    V = np.ascontiguousarray(valid, dtype=np.uint8)
    st = _Stats()
    pc = params._c()
    lib().or_normal_equations(C.byref(c), _p(IA), _p(WA), _p(Iw), _p(Ww), _pu8(V),
                              C.byref(pc), None, C.byref(st))
    return _stats(st)


def normal_equations_at(cam0, IA0, WA0, IB0, WB0, level, R, t, params: Params = None):
    params = params or Params()
    c = _cam(cam0)
    arrs = [_d(a) for a in (IA0, WA0, IB0, WB0)]
    st = _Stats()
    pc = params._c()
    lib().or_normal_equations_at(C.byref(c), params.levels, *[_p(a) for a in arrs], level,
                                 _p(_d(R).reshape(9)), _p(_d(t)), C.byref(pc), C.byref(st))
    return _stats(st)


def align(cam0, IA0, WA0, IB0, WB0, params: Params = None, R0=None, t0=None):
    """Coarse-to-fine alignment; returns (R, t, stats)."""
    params = params or Params()
    c = _cam(cam0)
    arrs = [_d(a) for a in (IA0, WA0, IB0, WB0)]
    R, t = np.zeros(9), np.zeros(3)
    st = _Stats()
    pc = params._c()
    Rp = _p(_d(R0).reshape(9)) if R0 is not None else None
    tp = _p(_d(t0)) if t0 is not None else None
    R0k = _d(R0).reshape(9) if R0 is not None else None   # keep alive
    t0k = _d(t0) if t0 is not None else None
    if R0k is not None:
        Rp = _p(R0k)
    if t0k is not None:
        tp = _p(t0k)
    lib().or_align(C.byref(c), *[_p(a) for a in arrs], Rp, tp, C.byref(pc), _p(R), _p(t),
                   C.byref(st))
    return R.reshape(3, 3), t, _stats(st)


def fuse(cam, Wkf, Ckf, Wk, R, t, tol):
    """Returns (W_kf', C_kf', n_fused); inputs are not modified."""
    c = _cam(cam)
    Wkf = _d(Wkf).copy()
    Ckf = _d(Ckf).copy()
    Wk = _d(Wk)
    n = lib().or_fuse(C.byref(c), _p(Wkf), _p(Ckf), _p(Wk), _p(_d(R).reshape(9)), _p(_d(t)),
                      float(tol))
    return Wkf, Ckf, int(n)


def covisibility(cam, WA, WB, R, t, tol):
    """(|S_H|, |S_V|) of A transferred into B (sec. 6.4)."""
    c = _cam(cam)
    nH, nV = C.c_longlong(), C.c_longlong()
    lib().or_covisibility(C.byref(c), _p(_d(WA)), _p(_d(WB)), _p(_d(R).reshape(9)), _p(_d(t)),
                          float(tol), C.byref(nH), C.byref(nV))
    return nH.value, nV.value


def covisibility_ratio(cam, WA, WB, R, t, tol):
    """min(vr_AB, vr_BA) with vr = |S_V| / |S_H| (sec. 6.4); B -> A uses the
    inverse pose."""
    hA, vA = covisibility(cam, WA, WB, R, t, tol)
    R = np.asarray(R, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    hB, vB = covisibility(cam, WB, WA, R.T, -R.T @ t, tol)
    ra = vA / hA if hA else 0.0
    rb = vB / hB if hB else 0.0
    return min(ra, rb), (hA, vA, hB, vB)


# default bilateral filter of the covariance iteration (a reading: the paper
# gives no parameters)
BILATERAL = dict(radius=2, sigma_s=1.5, sigma_I=10.0, rel_W=0.05)


def bilateral(I, W, radius=2, sigma_s=1.5, sigma_I=10.0, rel_W=0.05):
    I, W = _d(I), _d(W)
    h, w = I.shape
    Io, Wo = np.zeros((h, w)), np.zeros((h, w))
    lib().or_bilateral(_p(I), _p(W), w, h, radius, sigma_s, sigma_I, rel_W, _p(Io), _p(Wo))
    return Io, Wo


def covariance(cam0, IA0, WA0, IB0, WB0, R, t, params: Params = None, **bf):
    """(Sigma 6x6, stats) of the filtered extra linearisation at level 0."""
    params = params or Params()
    b = dict(BILATERAL, **bf)
    c = _cam(cam0)
    arrs = [_d(a) for a in (IA0, WA0, IB0, WB0)]
    S = np.zeros(36)
    st = _Stats()
    pc = params._c()
    rc = lib().or_covariance(C.byref(c), params.levels, *[_p(a) for a in arrs],
                             _p(_d(R).reshape(9)), _p(_d(t)), C.byref(pc), int(b["radius"]),
                             float(b["sigma_s"]), float(b["sigma_I"]), float(b["rel_W"]), _p(S),
                             C.byref(st))
    return (S.reshape(6, 6) if rc == 0 else None), _stats(st)


# --------------------------------------------------------------------------
# sensor input path (sec. 4.1, 4.2, 5.1, 5.2)


@dataclass
class Sensor:
    """Calibration of an RGB-D sensor: colour and depth pinhole cameras with
    Brown distortion k = (k1..k5), depth correction (beta0, beta1, p0 and the
    nine-term polynomials q0, q1 of D0, D1), and T_D^C, the pose of the colour
    camera in the depth camera."""
    color: tuple
    depth: tuple
    k_color: tuple = (0.0,) * 5
    k_depth: tuple = (0.0,) * 5
    beta0: float = 0.0
    beta1: float = 1.0
    p0: tuple = (4, 4)
    spatial: bool = False
    q0: tuple = (0.0,) * 9
    q1: tuple = (1.0,) + (0.0,) * 8
    R_dc: np.ndarray = field(default_factory=lambda: np.eye(3))
    t_dc: np.ndarray = field(default_factory=lambda: np.zeros(3))


def distort(k, x, y):
    xd, yd = C.c_double(), C.c_double()
    lib().or_distort(_p(_d(k)), float(x), float(y), C.byref(xd), C.byref(yd))
    return xd.value, yd.value


def undistort(cam, k, src, is_depth):
    c = _cam(cam)
    out = np.zeros((c.h, c.w))
    lib().or_undistort(C.byref(c), _p(_d(k)), _p(_d(src)), int(is_depth), _p(out))
    return out


def depth_correct(cam, Z, beta0=0.0, beta1=1.0, p0=(4, 4), spatial=False, q0=(0.0,) * 9,
                  q1=(1.0,) + (0.0,) * 8):
    c = _cam(cam)
    out = np.zeros((c.h, c.w))
    lib().or_depth_correct(C.byref(c), _p(_d(Z)), float(beta0), float(beta1), int(p0[0]),
                           int(p0[1]), int(spatial), _p(_d(q0)), _p(_d(q1)), _p(out))
    return out


def register_translate(camA, WA, t):
    c = _cam(camA)
    out = np.zeros((c.h, c.w))
    lib().or_register_translate(C.byref(c), _p(_d(WA)), _p(_d(t)), _p(out))
    return out


def register_rotate(camA, WBt, camB, R):
    ca, cb = _cam(camA), _cam(camB)
    out = np.zeros((cb.h, cb.w))
    lib().or_register_rotate(C.byref(ca), _p(_d(WBt)), C.byref(cb), _p(_d(R).reshape(9)), _p(out))
    return out


def register(camA, WA, camB, R, t):
    """Forward registration of W_A into camera B with T_A^B = (R, t)."""
    return register_rotate(camA, register_translate(camA, WA, t), camB, R)


def preprocess(s: Sensor, I_raw, Z_raw):
    cc, cd = _cam(s.color), _cam(s.depth)
    Io = np.zeros((cc.h, cc.w))
    Wo = np.zeros((cc.h, cc.w))
    lib().or_preprocess(C.byref(cc), _p(_d(s.k_color)), C.byref(cd), _p(_d(s.k_depth)),
                        float(s.beta0), float(s.beta1), int(s.p0[0]), int(s.p0[1]),
                        int(s.spatial), _p(_d(s.q0)), _p(_d(s.q1)), _p(_d(s.R_dc).reshape(9)),
                        _p(_d(s.t_dc)), _p(_d(I_raw)), _p(_d(Z_raw)), _p(Io), _p(Wo))
    return Io, Wo
