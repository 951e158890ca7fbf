"""ctypes binding of librgbid.so, the gfx950 dense RGB-D alignment library.

Names mirror the C ABI in include/rgbid.h.  The binding only marshals
arguments: torch tensors supply device memory (``data_ptr()``) and the HIP
stream; every step of the method runs in the library's HIP kernels.  If the
library is not built, loading raises immediately (there is no fallback).

Poses are ``(R, t)`` numpy tuples, the pose of B in A (X_A = R X_B + t).
Cameras are ``(width, height, fx, fy, cx, cy)`` tuples or objects with
``as_tuple()``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librgbid.so")

RGBID_OK, RGBID_E_ARG, RGBID_E_SHAPE, RGBID_E_DEVICE, RGBID_E_NOMEM, RGBID_E_DEGENERATE = (
    0, -1, -2, -3, -4, -5)
RGBID_F32, RGBID_F16 = 0, 1
RGBID_W_STUDENT_T, RGBID_W_HUBER = 0, 1
RGBID_WARP_FULLRES, RGBID_WARP_PER_LEVEL = 0, 1

_STATUS_NAMES = {0: "OK", -1: "E_ARG", -2: "E_SHAPE", -3: "E_DEVICE", -4: "E_NOMEM",
                 -5: "E_DEGENERATE"}


class RgbidError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(code, code), msg))
        self.code = code


class rgbid_camera(C.Structure):
    _fields_ = [("width", C.c_int), ("height", C.c_int), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double)]


class rgbid_pose(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3)]


class rgbid_align_params(C.Structure):
    _fields_ = [("levels", C.c_int), ("iters", C.c_int * 8), ("weight", C.c_int),
                ("huber_k", C.c_double), ("estimate_nu", C.c_int), ("sample_max", C.c_int),
                ("scale_iters", C.c_int), ("warp", C.c_int), ("stop_eps_t", C.c_double),
                ("stop_eps_r", C.c_double), ("scale_warm", C.c_int)]


class rgbid_bilateral(C.Structure):
    _fields_ = [("radius", C.c_int), ("sigma_s", C.c_double), ("sigma_I", C.c_double),
                ("rel_W", C.c_double)]


class rgbid_align_stats(C.Structure):
    _fields_ = [("H", C.c_double * 21), ("g", C.c_double * 6), ("mu_I", C.c_double),
                ("sigma_I", C.c_double), ("nu_I", C.c_double), ("mu_W", C.c_double),
                ("sigma_W", C.c_double), ("nu_W", C.c_double), ("cost", C.c_double),
                ("n_valid_I", C.c_longlong), ("n_valid_W", C.c_longlong),
                ("iters_done", C.c_int * 8), ("status", C.c_int)]

    def as_dict(self):
        H = np.zeros((6, 6))
        k = 0
        for a in range(6):
            for b in range(a, 6):
                H[a, b] = H[b, a] = self.H[k]
                k += 1
        return dict(H=H, g=np.array(self.g[:]), mu_I=self.mu_I, sigma_I=self.sigma_I,
                    nu_I=self.nu_I, mu_W=self.mu_W, sigma_W=self.sigma_W, nu_W=self.nu_W,
                    cost=self.cost, n_valid_I=self.n_valid_I, n_valid_W=self.n_valid_W,
                    iters_done=list(self.iters_done[:]), status=self.status)


class rgbid_lens(C.Structure):
    _fields_ = [("cam", rgbid_camera), ("k", C.c_double * 5)]


class rgbid_sensor(C.Structure):
    _fields_ = [("color", rgbid_lens), ("depth", rgbid_lens), ("beta0", C.c_double),
                ("beta1", C.c_double), ("p0x", C.c_int), ("p0y", C.c_int), ("spatial", C.c_int),
                ("q0", C.c_double * 9), ("q1", C.c_double * 9), ("T_dc", rgbid_pose)]


class rgbid_tracker_params(C.Structure):
    _fields_ = [("align", rgbid_align_params), ("rf_threshold", C.c_double),
                ("kf_threshold", C.c_double), ("covis_level", C.c_int),
                ("tol_sigmas", C.c_double), ("buffer", C.c_int), ("covariance", C.c_int)]


class rgbid_track_result(C.Structure):
    _fields_ = [("frame", C.c_longlong), ("T_w_k", rgbid_pose), ("T_rf_k", rgbid_pose),
                ("T_prev_k", rgbid_pose), ("Sigma_rf_k", C.c_double * 36),
                ("Sigma_odo", C.c_double * 36), ("covis_rf", C.c_double),
                ("covis_kf", C.c_double), ("rf_switched", C.c_int), ("kf_switched", C.c_int),
                ("cov_status", C.c_int), ("n_fused", C.c_longlong),
                ("n_fused_buffer", C.c_longlong), ("stats", rgbid_align_stats)]

    def as_dict(self):
        return dict(k=self.frame, T_w_k=pose_tuple(self.T_w_k), T_rf_k=pose_tuple(self.T_rf_k),
                    T_prev_k=pose_tuple(self.T_prev_k),
                    S_rf_k=np.array(self.Sigma_rf_k[:]).reshape(6, 6),
                    S_odo=np.array(self.Sigma_odo[:]).reshape(6, 6), covis_rf=self.covis_rf,
                    covis_kf=self.covis_kf, rf_switched=bool(self.rf_switched),
                    kf_switched=bool(self.kf_switched), cov_status=self.cov_status,
                    n_fused=self.n_fused, n_fused_buffer=self.n_fused_buffer,
                    stats=self.stats.as_dict())


_lib = None

# Every exported entry point with (restype, argtypes).
_P = C.c_void_p
_SIGS = {
    "rgbid_default_params": (None, [C.POINTER(rgbid_align_params)]),
    "rgbid_create": (C.c_int, [C.POINTER(_P), C.c_int, _P]),
    "rgbid_destroy": (None, [_P]),
    "rgbid_last_error": (C.c_char_p, [_P]),
    "rgbid_pyramid": (C.c_int, [_P, C.POINTER(rgbid_camera), C.c_int, C.c_int, _P, _P, C.c_size_t,
                                C.POINTER(_P)]),
    "rgbid_pyramid_update": (C.c_int, [_P, _P, _P, _P, C.c_size_t]),
    "rgbid_pyramid_update_batch": (C.c_int, [_P, C.c_int, C.POINTER(_P), C.POINTER(_P),
                                             C.POINTER(_P), C.POINTER(C.c_size_t)]),
    "rgbid_pyramid_read": (C.c_int, [_P, _P, C.c_int, _P, _P]),
    "rgbid_pyramid_level_size": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "rgbid_pyramid_free": (None, [_P]),
    "rgbid_align": (C.c_int, [_P, _P, _P, C.POINTER(rgbid_pose), C.POINTER(rgbid_align_params),
                              C.POINTER(rgbid_pose), C.POINTER(rgbid_align_stats)]),
    "rgbid_align_noalloc": (C.c_int, [_P, _P, _P, C.POINTER(rgbid_pose),
                                      C.POINTER(rgbid_align_params), C.POINTER(rgbid_pose),
                                      C.POINTER(rgbid_align_stats)]),
    "rgbid_align_batch": (C.c_int, [_P, C.c_int, C.POINTER(_P), C.POINTER(_P),
                                    C.POINTER(rgbid_pose), C.POINTER(rgbid_align_params),
                                    C.POINTER(rgbid_pose), C.POINTER(rgbid_align_stats)]),
    "rgbid_align_batch_async": (C.c_int, [_P, C.c_int, C.POINTER(_P), C.POINTER(_P),
                                          C.POINTER(rgbid_pose), C.POINTER(rgbid_align_params),
                                          _P, _P]),
    "rgbid_normal_equations": (C.c_int, [_P, _P, _P, C.c_int, C.POINTER(rgbid_pose),
                                         C.POINTER(rgbid_align_params),
                                         C.POINTER(rgbid_align_stats)]),
    "rgbid_keyframe_init": (C.c_int, [_P, C.POINTER(rgbid_camera), _P, C.c_size_t, C.POINTER(_P)]),
    "rgbid_fuse": (C.c_int, [_P, _P, _P, C.c_size_t, C.POINTER(rgbid_pose), C.c_double,
                             C.POINTER(C.c_longlong)]),
    "rgbid_keyframe_read": (C.c_int, [_P, _P, _P, _P]),
    "rgbid_keyframe_reset": (C.c_int, [_P, _P, _P, C.c_size_t]),
    "rgbid_keyframe_free": (None, [_P]),
    "rgbid_pose_exp": (None, [C.POINTER(C.c_double), C.POINTER(rgbid_pose)]),
    "rgbid_pose_log": (None, [C.POINTER(rgbid_pose), C.POINTER(C.c_double)]),
    "rgbid_warmstart_param_count": (C.c_size_t, []),
    "rgbid_warmstart_create": (C.c_int, [_P, C.POINTER(C.c_float), C.POINTER(_P)]),
    "rgbid_warmstart_free": (None, [_P]),
    "rgbid_warmstart_get_params": (C.c_int, [_P, _P, C.POINTER(C.c_float)]),
    "rgbid_warmstart_input": (C.c_int, [_P, C.c_int, C.POINTER(_P), C.POINTER(_P), _P]),
    "rgbid_warmstart_forward": (C.c_int, [_P, _P, C.c_int, _P, C.POINTER(C.c_double)]),
    "rgbid_warmstart_predict": (C.c_int, [_P, _P, C.c_int, C.POINTER(_P), C.POINTER(_P), _P,
                                          C.POINTER(rgbid_pose)]),
    "rgbid_warmstart_forward_pyr": (C.c_int, [_P, _P, C.c_int, C.POINTER(_P), C.POINTER(_P),
                                              C.POINTER(C.c_double)]),
    "rgbid_align_batch_warm": (C.c_int, [_P, _P, C.c_int, C.POINTER(_P), C.POINTER(_P),
                                         C.POINTER(rgbid_align_params), C.POINTER(rgbid_pose),
                                         C.POINTER(rgbid_align_stats)]),
    "rgbid_warmstart_gradient": (C.c_int, [_P, _P, C.c_int, _P, C.POINTER(C.c_double),
                                           C.POINTER(C.c_double), C.POINTER(C.c_float)]),
    "rgbid_warmstart_train_step": (C.c_int, [_P, _P, C.c_int, _P, C.POINTER(C.c_double), C.c_double,
                                             C.c_double, C.POINTER(C.c_double)]),
    "rgbid_autotune": (C.c_int, [_P, C.c_int, C.POINTER(_P), C.POINTER(_P),
                                 C.POINTER(rgbid_align_params), C.c_int, C.POINTER(C.c_double)]),
    "rgbid_fuse_batch": (C.c_int, [_P, _P, C.c_int, _P, C.c_size_t, _P, C.c_double, _P]),
    "rgbid_tune_save": (C.c_int, [_P, C.c_char_p]),
    "rgbid_tune_load": (C.c_int, [_P, C.c_char_p]),
    "rgbid_covisibility": (C.c_int, [_P, _P, _P, C.c_int, C.POINTER(rgbid_pose), C.c_double,
                                     C.POINTER(C.c_double), C.POINTER(C.c_longlong)]),
    "rgbid_covariance": (C.c_int, [_P, _P, _P, C.POINTER(rgbid_pose), C.POINTER(rgbid_align_params),
                                   C.POINTER(rgbid_bilateral), C.POINTER(C.c_double),
                                   C.POINTER(rgbid_align_stats)]),
    "rgbid_undistort": (C.c_int, [_P, C.POINTER(rgbid_lens), _P, C.c_size_t, C.c_int, _P]),
    "rgbid_register": (C.c_int, [_P, C.POINTER(rgbid_camera), _P, C.c_size_t,
                                 C.POINTER(rgbid_camera), C.POINTER(rgbid_pose), _P]),
    "rgbid_preprocess": (C.c_int, [_P, C.POINTER(rgbid_sensor), _P, C.c_size_t, _P, C.c_size_t,
                                   _P, _P]),
    "rgbid_tracker_default_params": (None, [C.POINTER(rgbid_tracker_params)]),
    "rgbid_tracker_create": (C.c_int, [_P, C.POINTER(rgbid_camera), C.c_int, C.c_int,
                                       C.POINTER(rgbid_tracker_params), C.POINTER(_P)]),
    "rgbid_track": (C.c_int, [_P, _P, _P, _P, C.c_size_t, C.POINTER(rgbid_track_result)]),
    "rgbid_tracker_keyframe": (_P, [_P]),
    "rgbid_tracker_free": (None, [_P]),
    "rgbid_set_profiling": (C.c_int, [_P, C.c_int]),
    "rgbid_kernel_times": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]),
}


def lib():
    """Loads librgbid.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librgbid.so is not built: run `python -m paper_1807_08271_amd.build`"
                               " (or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


# ----------------------------------------------------------------- helpers


def _cam(cam) -> rgbid_camera:
    if isinstance(cam, rgbid_camera):
        return cam
    w, h, fx, fy, cx, cy = cam.as_tuple() if hasattr(cam, "as_tuple") else cam
    return rgbid_camera(int(w), int(h), float(fx), float(fy), float(cx), float(cy))


def make_pose(R=None, t=None) -> rgbid_pose:
    p = rgbid_pose()
    R = np.eye(3) if R is None else np.asarray(R, dtype=np.float64).reshape(9)
    t = np.zeros(3) if t is None else np.asarray(t, dtype=np.float64).reshape(3)
    for i in range(9):
        p.R[i] = float(np.ravel(R)[i])
    for i in range(3):
        p.t[i] = float(t[i])
    return p


def pose_tuple(p: rgbid_pose):
    return np.array(p.R[:]).reshape(3, 3), np.array(p.t[:])


def _check(ctx, rc, allow=()):
    if rc != RGBID_OK and rc not in allow:
        raise RgbidError(rc, rgbid_last_error(ctx))
    return rc


def _img(t):
    """(pointer, pitch in elements) of a 2-D float32 device tensor."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dim() != 2 or t.dtype != torch.float32:
        raise TypeError("expected a 2-D float32 torch tensor")
    if not t.is_cuda:
        raise TypeError("expected a device tensor")
    if t.stride(1) != 1:
        raise ValueError("rows must be contiguous")
    return C.c_void_p(t.data_ptr()), int(t.stride(0))


# ----------------------------------------------------------------- ABI


def rgbid_default_params(**overrides) -> rgbid_align_params:
    p = rgbid_align_params()
    lib().rgbid_default_params(C.byref(p))
    for k, v in overrides.items():
        if k == "iters":
            its = list(v) + [0] * (8 - len(v))
            for i in range(8):
                p.iters[i] = int(its[i])
        elif k in dict(rgbid_align_params._fields_):
            setattr(p, k, v)
        else:
            raise TypeError("rgbid_align_params has no field %r" % k)
    return p


def rgbid_create(device: int = 0, stream=None):
    """stream: a torch stream, a raw hipStream_t int, or None for torch's
    current stream on `device`."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    ctx = C.c_void_p()
    rc = lib().rgbid_create(C.byref(ctx), int(device), C.c_void_p(handle))
    if rc != RGBID_OK:
        raise RgbidError(rc, "rgbid_create failed")
    return ctx


def rgbid_destroy(ctx):
    lib().rgbid_destroy(ctx)


def rgbid_last_error(ctx) -> str:
    s = lib().rgbid_last_error(ctx)
    return s.decode() if s else ""


def rgbid_pyramid(ctx, cam, levels: int, storage: int, I, W):
    pI, pitch = _img(I)
    pW, pitchW = _img(W)
    if pitch != pitchW:
        raise ValueError("I and W need the same row pitch")
    out = C.c_void_p()
    c = _cam(cam)
    _check(ctx, lib().rgbid_pyramid(ctx, C.byref(c), int(levels), int(storage), pI, pW, pitch,
                                    C.byref(out)))
    return out


def rgbid_pyramid_update(ctx, pyr, I, W):
    pI, pitch = _img(I)
    pW, _ = _img(W)
    _check(ctx, lib().rgbid_pyramid_update(ctx, pyr, pI, pW, pitch))


def rgbid_pyramid_update_batch(ctx, pyrs, Is, Ws):
    n = len(pyrs)
    arr = (C.c_void_p * n)(*[p.value for p in pyrs])
    pis, pws, pts = [], [], []
    for I, W in zip(Is, Ws):
        a, pitch = _img(I)
        b, _ = _img(W)
        pis.append(a.value)
        pws.append(b.value)
        pts.append(pitch)
    _check(ctx, lib().rgbid_pyramid_update_batch(ctx, n, arr, (C.c_void_p * n)(*pis),
                                                 (C.c_void_p * n)(*pws),
                                                 (C.c_size_t * n)(*pts)))


def rgbid_pyramid_level_size(pyr, level: int):
    w, h = C.c_int(), C.c_int()
    rc = lib().rgbid_pyramid_level_size(pyr, int(level), C.byref(w), C.byref(h))
    if rc != RGBID_OK:
        raise RgbidError(rc, "bad pyramid or level")
    return w.value, h.value


def rgbid_pyramid_read(ctx, pyr, level: int, device=None):
    import torch
    w, h = rgbid_pyramid_level_size(pyr, level)
    I = torch.empty((h, w), dtype=torch.float32, device=device or "cuda")
    W = torch.empty((h, w), dtype=torch.float32, device=device or "cuda")
    _check(ctx, lib().rgbid_pyramid_read(ctx, pyr, int(level), C.c_void_p(I.data_ptr()),
                                         C.c_void_p(W.data_ptr())))
    return I, W


def rgbid_pyramid_free(pyr):
    lib().rgbid_pyramid_free(pyr)


def rgbid_align(ctx, A, B, params: rgbid_align_params, init=None):
    """Returns (R, t, stats dict, status); E_DEGENERATE is reported in status."""
    out = rgbid_pose()
    st = rgbid_align_stats()
    ini = make_pose(*init) if init is not None else None
    rc = lib().rgbid_align(ctx, A, B, C.byref(ini) if ini is not None else None, C.byref(params),
                           C.byref(out), C.byref(st))
    _check(ctx, rc, allow=(RGBID_E_DEGENERATE,))
    R, t = pose_tuple(out)
    return R, t, st.as_dict(), rc


def rgbid_align_noalloc(ctx, A, B, params: rgbid_align_params, init=None):
    """rgbid_align without any allocation (scratch in the library's static
    device array); returns (R, t, stats dict, status)."""
    out = rgbid_pose()
    st = rgbid_align_stats()
    ini = make_pose(*init) if init is not None else None
    rc = lib().rgbid_align_noalloc(ctx, A, B, C.byref(ini) if ini is not None else None,
                                   C.byref(params), C.byref(out), C.byref(st))
    _check(ctx, rc, allow=(RGBID_E_DEGENERATE,))
    R, t = pose_tuple(out)
    return R, t, st.as_dict(), rc


def rgbid_align_batch(ctx, As, Bs, params: rgbid_align_params, inits=None):
    """Returns (list of (R, t), list of stats dicts)."""
    n = len(As)
    a = (C.c_void_p * n)(*[p.value for p in As])
    b = (C.c_void_p * n)(*[p.value for p in Bs])
    ini = None
    if inits is not None:
        ini = (rgbid_pose * n)(*[make_pose(*x) for x in inits])
    out = (rgbid_pose * n)()
    st = (rgbid_align_stats * n)()
    _check(ctx, lib().rgbid_align_batch(ctx, n, a, b, ini, C.byref(params), out, st))
    return [pose_tuple(out[i]) for i in range(n)], [st[i].as_dict() for i in range(n)]


POSE_BYTES = C.sizeof(rgbid_pose)
STATS_BYTES = C.sizeof(rgbid_align_stats)


def rgbid_align_batch_async(ctx, As, Bs, params: rgbid_align_params, out, stats=None, inits=None):
    """Enqueues the batch; poses (and stats) land in the device tensors out
    (>= n * POSE_BYTES bytes) and stats (>= n * STATS_BYTES bytes).  Nothing
    waits; read them with unpack_poses / unpack_stats after synchronising."""
    n = len(As)
    for t, need in ((out, n * POSE_BYTES), (stats, n * STATS_BYTES)):
        if t is not None and (not t.is_cuda or t.numel() * t.element_size() < need):
            raise ValueError("output buffers must be device tensors of the required size")
    a = (C.c_void_p * n)(*[p.value for p in As])
    b = (C.c_void_p * n)(*[p.value for p in Bs])
    ini = None
    if inits is not None:
        ini = (rgbid_pose * n)(*[make_pose(*x) for x in inits])
    _check(ctx, lib().rgbid_align_batch_async(
        ctx, n, a, b, ini, C.byref(params), C.c_void_p(out.data_ptr()),
        C.c_void_p(stats.data_ptr()) if stats is not None else None))


def unpack_poses(buf, n):
    """(R, t) list from a host copy of rgbid_align_batch_async's output."""
    raw = bytes(buf.cpu().numpy().tobytes()[:n * POSE_BYTES])
    arr = (rgbid_pose * n).from_buffer_copy(raw)
    return [pose_tuple(arr[i]) for i in range(n)]


def unpack_stats(buf, n):
    raw = bytes(buf.cpu().numpy().tobytes()[:n * STATS_BYTES])
    arr = (rgbid_align_stats * n).from_buffer_copy(raw)
    return [arr[i].as_dict() for i in range(n)]


def rgbid_normal_equations(ctx, A, B, level: int, T, params: rgbid_align_params):
    st = rgbid_align_stats()
    pose = make_pose(*T)
    _check(ctx, lib().rgbid_normal_equations(ctx, A, B, int(level), C.byref(pose), C.byref(params),
                                             C.byref(st)))
    return st.as_dict()


def rgbid_keyframe_init(ctx, cam, W):
    pW, pitch = _img(W)
    out = C.c_void_p()
    c = _cam(cam)
    _check(ctx, lib().rgbid_keyframe_init(ctx, C.byref(c), pW, pitch, C.byref(out)))
    return out


def rgbid_fuse(ctx, kf, Wk, T, tol: float, count: bool = True):
    pW, pitch = _img(Wk)
    pose = make_pose(*T)
    n = C.c_longlong(0)
    _check(ctx, lib().rgbid_fuse(ctx, kf, pW, pitch, C.byref(pose), float(tol),
                                 C.byref(n) if count else None))
    return n.value if count else None


def rgbid_fuse_batch(ctx, kf, Wks, Ts, tol: float, count: bool = False):
    """Fuses the maps Wks (FP32 device tensors of one pitch) with poses Ts
    ((R, t) each) in order in one launch; returns the per-frame counts when
    count is set."""
    n = len(Wks)
    if n != len(Ts):
        raise ValueError("one pose per map")
    ptrs = (C.c_void_p * n)()
    pitch = None
    for i, w in enumerate(Wks):
        p, pt = _img(w)
        if pitch is not None and pt != pitch:
            raise ValueError("all maps need the same row pitch")
        pitch = pt
        ptrs[i] = p.value
    poses = (rgbid_pose * n)(*[make_pose(*T) for T in Ts])
    cnt = (C.c_longlong * n)()
    _check(ctx, lib().rgbid_fuse_batch(ctx, kf, n, ptrs, pitch or 0, poses, float(tol),
                                       cnt if count else None))
    return list(cnt) if count else None


def rgbid_keyframe_read(ctx, kf, shape, device=None):
    import torch
    h, w = shape
    W = torch.empty((h, w), dtype=torch.float32, device=device or "cuda")
    Cm = torch.empty((h, w), dtype=torch.float32, device=device or "cuda")
    _check(ctx, lib().rgbid_keyframe_read(ctx, kf, C.c_void_p(W.data_ptr()), C.c_void_p(Cm.data_ptr())))
    return W, Cm


def rgbid_keyframe_reset(ctx, kf, W):
    pW, pitch = _img(W)
    _check(ctx, lib().rgbid_keyframe_reset(ctx, kf, pW, pitch))


RGBID_K_WARP, RGBID_K_SCALE, RGBID_K_REDUCE, RGBID_K_SOLVE = 0, 1, 2, 3
KERNEL_NAMES = ("warp", "scale", "reduce", "solve")


def rgbid_set_profiling(ctx, on: bool):
    _check(ctx, lib().rgbid_set_profiling(ctx, int(bool(on))))


def rgbid_kernel_times(ctx):
    """{(level, kernel name): (total ms, launches)} for entries with launches."""
    ms = (C.c_double * 32)()
    n = (C.c_longlong * 32)()
    _check(ctx, lib().rgbid_kernel_times(ctx, ms, n))
    out = {}
    for l in range(8):
        for k in range(4):
            if n[l * 4 + k]:
                out[(l, KERNEL_NAMES[k])] = (ms[l * 4 + k], n[l * 4 + k])
    return out


def rgbid_keyframe_free(kf):
    lib().rgbid_keyframe_free(kf)


# ----------------------------------------------------------------- pose maps


def rgbid_pose_exp(xi):
    x = (C.c_double * 6)(*[float(v) for v in np.ravel(xi)])
    p = rgbid_pose()
    lib().rgbid_pose_exp(x, C.byref(p))
    return pose_tuple(p)


def rgbid_pose_log(R, t):
    p = make_pose(R, t)
    x = (C.c_double * 6)()
    lib().rgbid_pose_log(C.byref(p), x)
    return np.array(x[:])


# ----------------------------------------------------------------- warm start


def rgbid_warmstart_param_count() -> int:
    return int(lib().rgbid_warmstart_param_count())


def rgbid_warmstart_create(ctx, params):
    a = np.ascontiguousarray(params, dtype=np.float32)
    if a.size != rgbid_warmstart_param_count():
        raise ValueError("expected %d parameters" % rgbid_warmstart_param_count())
    out = C.c_void_p()
    _check(ctx, lib().rgbid_warmstart_create(ctx, a.ctypes.data_as(C.POINTER(C.c_float)),
                                             C.byref(out)))
    return out


def rgbid_warmstart_free(net):
    lib().rgbid_warmstart_free(net)


def rgbid_warmstart_get_params(ctx, net):
    a = np.zeros(rgbid_warmstart_param_count(), dtype=np.float32)
    _check(ctx, lib().rgbid_warmstart_get_params(ctx, net, a.ctypes.data_as(C.POINTER(C.c_float))))
    return a


def _dev(t, n):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 \
            or not t.is_contiguous() or t.numel() < n * 4 * 60 * 80:
        raise TypeError("expected a contiguous float32 device tensor of n x 4 x 60 x 80")
    return C.c_void_p(t.data_ptr())


def rgbid_warmstart_input(ctx, As, Bs, x):
    n = len(As)
    a = (C.c_void_p * n)(*[p.value for p in As])
    b = (C.c_void_p * n)(*[p.value for p in Bs])
    _check(ctx, lib().rgbid_warmstart_input(ctx, n, a, b, _dev(x, n)))


def rgbid_warmstart_forward(ctx, net, x, n):
    xi = np.zeros(n * 6)
    _check(ctx, lib().rgbid_warmstart_forward(ctx, net, int(n), _dev(x, n),
                                              xi.ctypes.data_as(C.POINTER(C.c_double))))
    return xi.reshape(n, 6)


def rgbid_warmstart_forward_pyr(ctx, net, As, Bs):
    """Matrix-core forward from the pyramids' 80x60 level: xi0 (n x 6)."""
    n = len(As)
    a = (C.c_void_p * n)(*[p.value for p in As])
    b = (C.c_void_p * n)(*[p.value for p in Bs])
    xi = np.zeros(n * 6)
    _check(ctx, lib().rgbid_warmstart_forward_pyr(ctx, net, n, a, b,
                                                  xi.ctypes.data_as(C.POINTER(C.c_double))))
    return xi.reshape(n, 6)


def rgbid_align_batch_warm(ctx, net, As, Bs, params: rgbid_align_params):
    """Warm-started batch alignment, initial poses formed on the device;
    returns (list of (R, t), list of stats dicts)."""
    n = len(As)
    a = (C.c_void_p * n)(*[p.value for p in As])
    b = (C.c_void_p * n)(*[p.value for p in Bs])
    out = (rgbid_pose * n)()
    st = (rgbid_align_stats * n)()
    _check(ctx, lib().rgbid_align_batch_warm(ctx, net, n, a, b, C.byref(params), out, st))
    return [pose_tuple(out[i]) for i in range(n)], [st[i].as_dict() for i in range(n)]


def rgbid_warmstart_predict(ctx, net, As, Bs, x_scratch):
    n = len(As)
    a = (C.c_void_p * n)(*[p.value for p in As])
    b = (C.c_void_p * n)(*[p.value for p in Bs])
    out = (rgbid_pose * n)()
    _check(ctx, lib().rgbid_warmstart_predict(ctx, net, n, a, b, _dev(x_scratch, n), out))
    return [pose_tuple(out[i]) for i in range(n)]


def rgbid_warmstart_gradient(ctx, net, x, xi):
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    n = xi.shape[0]
    loss = C.c_double()
    g = np.zeros(rgbid_warmstart_param_count(), dtype=np.float32)
    _check(ctx, lib().rgbid_warmstart_gradient(ctx, net, n, _dev(x, n),
                                               xi.ctypes.data_as(C.POINTER(C.c_double)),
                                               C.byref(loss), g.ctypes.data_as(C.POINTER(C.c_float))))
    return loss.value, g


def rgbid_warmstart_train_step(ctx, net, x, xi, lr, wd=1e-4, want_loss=False):
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    n = xi.shape[0]
    loss = C.c_double()
    _check(ctx, lib().rgbid_warmstart_train_step(ctx, net, n, _dev(x, n),
                                                 xi.ctypes.data_as(C.POINTER(C.c_double)),
                                                 float(lr), float(wd),
                                                 C.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


# ----------------------------------------------------------------- autotuner


def rgbid_autotune(ctx, As, Bs, params, reps=3):
    n = len(As)
    a = (C.c_void_p * n)(*[p.value for p in As])
    b = (C.c_void_p * n)(*[p.value for p in Bs])
    best = (C.c_double * 8)()
    _check(ctx, lib().rgbid_autotune(ctx, n, a, b, C.byref(params), int(reps), best))
    return list(best[:params.levels])


def rgbid_tune_save(ctx, path):
    _check(ctx, lib().rgbid_tune_save(ctx, path.encode()))


def rgbid_tune_load(ctx, path):
    _check(ctx, lib().rgbid_tune_load(ctx, path.encode()))


# ----------------------------------------------------------------- covisibility


def rgbid_covisibility(ctx, A, B, level, T, tol):
    """Returns (ratio, (|S_H(A)|, |S_V(A->B)|, |S_H(B)|, |S_V(B->A)|))."""
    r = C.c_double()
    cnt = (C.c_longlong * 4)()
    pose = make_pose(*T)
    _check(ctx, lib().rgbid_covisibility(ctx, A, B, int(level), C.byref(pose), float(tol),
                                         C.byref(r), cnt))
    return r.value, tuple(cnt[:])


# ----------------------------------------------------------------- covariance


def rgbid_covariance(ctx, A, B, T, params, radius=2, sigma_s=1.5, sigma_I=10.0, rel_W=0.05):
    """Returns (Sigma 6x6, stats dict of the filtered linearisation)."""
    bf = rgbid_bilateral(int(radius), float(sigma_s), float(sigma_I), float(rel_W))
    S = (C.c_double * 36)()
    st = rgbid_align_stats()
    pose = make_pose(*T)
    _check(ctx, lib().rgbid_covariance(ctx, A, B, C.byref(pose), C.byref(params), C.byref(bf), S,
                                       C.byref(st)))
    return np.array(S[:]).reshape(6, 6), st.as_dict()


# ----------------------------------------------------------------- tracking front-end


def rgbid_tracker_default_params(align=None, **overrides) -> rgbid_tracker_params:
    p = rgbid_tracker_params()
    lib().rgbid_tracker_default_params(C.byref(p))
    if align is not None:
        p.align = align
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def rgbid_tracker_create(ctx, cam, levels: int, storage: int, params: rgbid_tracker_params):
    out = C.c_void_p()
    c = _cam(cam)
    _check(ctx, lib().rgbid_tracker_create(ctx, C.byref(c), int(levels), int(storage),
                                           C.byref(params), C.byref(out)))
    return out


def rgbid_track(ctx, trk, I, W):
    """Tracks the next frame; returns the result as a dict (poses as (R, t))."""
    pI, pitch = _img(I)
    pW, pitchW = _img(W)
    if pitch != pitchW:
        raise ValueError("I and W need the same row pitch")
    res = rgbid_track_result()
    _check(ctx, lib().rgbid_track(ctx, trk, pI, pW, pitch, C.byref(res)))
    return res.as_dict()


def rgbid_tracker_keyframe(trk):
    return C.c_void_p(lib().rgbid_tracker_keyframe(trk))


def rgbid_tracker_free(trk):
    lib().rgbid_tracker_free(trk)


# ----------------------------------------------------------------- sensor input path


def make_lens(cam, k=None) -> rgbid_lens:
    L = rgbid_lens()
    L.cam = _cam(cam)
    for i, v in enumerate(k if k is not None else [0.0] * 5):
        L.k[i] = float(v)
    return L


def make_sensor(color, depth, k_color=None, k_depth=None, beta0=0.0, beta1=1.0, p0=(4, 4),
                spatial=False, q0=None, q1=None, R_dc=None, t_dc=None) -> rgbid_sensor:
    S = rgbid_sensor()
    S.color = make_lens(color, k_color)
    S.depth = make_lens(depth, k_depth)
    S.beta0, S.beta1 = float(beta0), float(beta1)
    S.p0x, S.p0y = int(p0[0]), int(p0[1])
    S.spatial = int(bool(spatial))
    q0 = q0 if q0 is not None else [0.0] * 9
    q1 = q1 if q1 is not None else [1.0] + [0.0] * 8
    for i in range(9):
        S.q0[i], S.q1[i] = float(q0[i]), float(q1[i])
    S.T_dc = make_pose(R_dc, t_dc)
    return S


def _out(h, w, device=None):
    import torch
    return torch.empty((h, w), dtype=torch.float32, device=device or "cuda")


def rgbid_undistort(ctx, lens: rgbid_lens, src, is_depth: bool, out=None):
    p, pitch = _img(src)
    out = out if out is not None else _out(lens.cam.height, lens.cam.width, src.device)
    _check(ctx, lib().rgbid_undistort(ctx, C.byref(lens), p, pitch, int(is_depth),
                                      C.c_void_p(out.data_ptr())))
    return out


def rgbid_register(ctx, camA, WA, camB, T, out=None):
    p, pitch = _img(WA)
    ca, cb = _cam(camA), _cam(camB)
    out = out if out is not None else _out(cb.height, cb.width, WA.device)
    pose = make_pose(*T)
    _check(ctx, lib().rgbid_register(ctx, C.byref(ca), p, pitch, C.byref(cb), C.byref(pose),
                                     C.c_void_p(out.data_ptr())))
    return out


def rgbid_preprocess(ctx, sensor: rgbid_sensor, I_raw, Z_raw, I_out=None, W_out=None):
    pI, pitchI = _img(I_raw)
    pZ, pitchZ = _img(Z_raw)
    h, w = sensor.color.cam.height, sensor.color.cam.width
    I_out = I_out if I_out is not None else _out(h, w, I_raw.device)
    W_out = W_out if W_out is not None else _out(h, w, I_raw.device)
    _check(ctx, lib().rgbid_preprocess(ctx, C.byref(sensor), pI, pitchI, pZ, pitchZ,
                                       C.c_void_p(I_out.data_ptr()), C.c_void_p(W_out.data_ptr())))
    return I_out, W_out
