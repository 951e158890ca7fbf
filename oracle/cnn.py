"""FP64 oracle of the learned warm-start network (test infrastructure only).

The network predicts the initial twist xi0 = (v, theta) of an alignment from
the coarsest pyramid level (80 x 60) of both frames; Gauss-Newton always runs
after it.  It is not part of the paper: the paper's own initial guess is the
identity or a constant-velocity prediction (sec. 6.2, sec. 7.1).

Architecture (input N x 4 x 60 x 80: I_A/255, W_A/2, I_B/255, W_B/2):
  4 x [3x3 convolution, stride 2, zero padding 1, + bias, ReLU]
      channels 4 -> 32 -> 64 -> 128 -> 128, maps 30x40, 15x20, 8x10, 4x5
  global average pool -> fully connected 128 -> 6 (+ bias)
  xi0 = out * SCALE, SCALE = (0.15 m) x 3, (0.1745 rad) x 3
Loss: mean over the batch of sum_k (out_k - xi_k / SCALE_k)^2.
Convolution and fully-connected weights are used in bfloat16 (rounded to
nearest even from the FP32 master copy); biases stay FP32.  This oracle
promotes those values to float64 and does everything else in float64.
"""
from __future__ import annotations

import numpy as np

CHANNELS = [4, 32, 64, 128, 128]
H0, W0 = 60, 80
SCALE = np.array([0.15, 0.15, 0.15, 0.1745, 0.1745, 0.1745])


def param_shapes():
    shapes = []
    for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]):
        shapes += [(co, ci, 3, 3), (co,)]
    shapes += [(6, CHANNELS[-1]), (6,)]
    return shapes


def n_params():
    return int(sum(np.prod(s) for s in param_shapes()))


def unpack(flat):
    out, off = [], 0
    for s in param_shapes():
        n = int(np.prod(s))
        out.append(np.asarray(flat[off:off + n], dtype=np.float64).reshape(s))
        off += n
    return out


def is_weight(i):
    """Parameter i is a convolution / FC weight (bf16) rather than a bias."""
    return i % 2 == 0


def round_bf16(x):
    """Round float32 values to the nearest bfloat16 (ties to even)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def effective_params(flat_fp32):
    """The values the forward pass uses: bf16-rounded weights, FP32 biases."""
    ps = unpack(np.asarray(flat_fp32, dtype=np.float32))
    return [round_bf16(p).astype(np.float64) if is_weight(i) else p.astype(np.float64)
            for i, p in enumerate(ps)]


def init_params(seed: int = 0):
    """He-normal weights, zero biases (FP32 master copy)."""
    rng = np.random.default_rng(seed)
    out = []
    for s in param_shapes():
        if len(s) == 1:
            out.append(np.zeros(s))
        else:
            fan_in = int(np.prod(s[1:]))
            gain = np.sqrt(2.0 / fan_in) if len(s) == 4 else np.sqrt(1.0 / fan_in)
            out.append(rng.normal(0.0, gain, size=s))
    return np.concatenate([p.reshape(-1) for p in out]).astype(np.float32)


def conv_out(h):
    return (h + 2 - 3) // 2 + 1


def conv_fwd(x, w, b):
    """z[n,co,y,x] = b[co] + sum_{ci,ky,kx} w[co,ci,ky,kx] xp[n,ci,2y+ky,2x+kx]
    with xp the input zero-padded by one pixel."""
    N, C, H, W = x.shape
    Ho, Wo = conv_out(H), conv_out(W)
    xp = np.zeros((N, C, H + 2 + 1, W + 2 + 1))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    z = np.zeros((N, w.shape[0], Ho, Wo)) + b[None, :, None, None]
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2]
            z += np.einsum("nchw,oc->nohw", patch, w[:, :, ky, kx])
    return z


def conv_bwd(x, w, dz):
    """Gradients of conv_fwd w.r.t. x, w and b."""
    N, C, H, W = x.shape
    Ho, Wo = dz.shape[2], dz.shape[3]
    xp = np.zeros((N, C, H + 3, W + 3))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2]
            dw[:, :, ky, kx] = np.einsum("nohw,nchw->oc", dz, patch)
            dxp[:, :, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2] += np.einsum("nohw,oc->nchw", dz,
                                                                     w[:, :, ky, kx])
    return dxp[:, :, 1:H + 1, 1:W + 1], dw, dz.sum(axis=(0, 2, 3))


def forward(params, x):
    """params: list from effective_params; x: (N, 4, 60, 80).  Returns the
    normalised output (N, 6) and the activations for backward."""
    acts = [np.asarray(x, dtype=np.float64)]
    a = acts[0]
    for l in range(4):
        z = conv_fwd(a, params[2 * l], params[2 * l + 1])
        a = np.maximum(z, 0.0)
        acts.append(a)
    pooled = a.mean(axis=(2, 3))
    out = pooled @ params[8].T + params[9]
    return out, (acts, pooled)


def loss(out, xi):
    t = np.asarray(xi, dtype=np.float64) / SCALE
    return float(np.mean(np.sum((out - t) ** 2, axis=1)))


def backward(params, cache, out, xi):
    """Gradient of loss(out, xi) w.r.t. every parameter (flat, float64) and
    w.r.t. the input."""
    acts, pooled = cache
    N = out.shape[0]
    dout = 2.0 * (out - np.asarray(xi) / SCALE) / N
    grads = [None] * 10
    grads[8] = dout.T @ pooled
    grads[9] = dout.sum(axis=0)
    dp = dout @ params[8]
    a = acts[4]
    da = np.broadcast_to(dp[:, :, None, None] / (a.shape[2] * a.shape[3]), a.shape).copy()
    for l in range(3, -1, -1):
        dz = da * (acts[l + 1] > 0)
        dx, dw, db = conv_bwd(acts[l], params[2 * l], dz)
        grads[2 * l], grads[2 * l + 1] = dw, db
        da = dx
    return np.concatenate([g.reshape(-1) for g in grads]), da


def adamw_step(w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=1e-4,
               decay_mask=None):
    """One AdamW update (decoupled weight decay on the weights only):
    m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
    w -= lr (m / (1-b1^t) / (sqrt(v / (1-b2^t)) + eps) + wd w)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    dec = wd * w if decay_mask is None else wd * w * decay_mask
    w = w - lr * (mh / (np.sqrt(vh) + eps) + dec)
    return w, m, v


def weight_mask():
    """1 for bf16 weights (decayed), 0 for biases."""
    parts = [np.full(int(np.prod(s)), 1.0 if is_weight(i) else 0.0)
             for i, s in enumerate(param_shapes())]
    return np.concatenate(parts)
