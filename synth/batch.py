"""Batched GPU rendering of large-motion frame pairs (training and evaluation
data of the learned warm start).

Same scene family, texture and noise model as synth.scene, but vectorised over
many frames of one scene at once in float32 on the device, with one ray per
pixel, and noise / disc holes drawn from a seeded torch generator on the
device.  It holds no alignment arithmetic.  Frames come back as device
tensors; nothing here is used by the oracle parity tests.
"""
from __future__ import annotations

import math

import numpy as np
import torch
from scipy.spatial.transform import Rotation

from .scene import (Camera, camera_640, compose, random_motion, room_scene, _perlin,
                    _pitch_down)


def _cast_many(scene, origins, dirs):
    """origins (F, 3), dirs (F, P, 3) -> nearest positive hit parameter (F, P)."""
    dev, dt = dirs.device, dirs.dtype
    best = torch.full(dirs.shape[:2], math.inf, dtype=dt, device=dev)
    for n, d in scene.planes:
        nt = torch.as_tensor(n, dtype=dt, device=dev)
        den = dirs @ nt
        num = d - origins @ nt
        s = num[:, None] / den
        ok = (den != 0) & (s > 1e-6)
        best = torch.where(ok & (s < best), s, best)
    for lo, hi in scene.boxes:
        lo_t = torch.as_tensor(lo, dtype=dt, device=dev)
        hi_t = torch.as_tensor(hi, dtype=dt, device=dev)
        inv = 1.0 / dirs
        t1 = (lo_t - origins[:, None, :]) * inv
        t2 = (hi_t - origins[:, None, :]) * inv
        tmin = torch.minimum(t1, t2).nan_to_num(nan=-math.inf).amax(dim=2)
        tmax = torch.maximum(t1, t2).nan_to_num(nan=math.inf).amin(dim=2)
        ok = (tmax >= tmin) & (tmin > 1e-6)
        best = torch.where(ok & (tmin < best), tmin, best)
    return best


def _texture_many(scene, P):
    perm = torch.as_tensor(scene.perm, device=P.device)
    offs = torch.as_tensor(scene.octave_offsets, dtype=P.dtype, device=P.device)
    acc = torch.zeros(P.shape[:-1], dtype=P.dtype, device=P.device)
    freq, amp = scene.base_freq, 1.0
    for o in range(4):
        Q = P * freq + offs[o]
        acc = acc + amp * _perlin(perm, Q[..., 0], Q[..., 1], Q[..., 2])
        freq *= 2.0
        amp *= 0.5
    return 128.0 + 100.0 * acc


def render_frames(scene, cam: Camera, poses, gen: torch.Generator, device="cuda",
                  hole_frac=0.10, sigma_I=2.0, sigma_W_coef=1.5e-3, zmin=0.5, zmax=5.0):
    """Renders len(poses) frames of one scene; returns I, W as (F, h, w)
    float32 device tensors (holes W = 0)."""
    F = len(poses)
    dt = torch.float32
    v, u = torch.meshgrid(torch.arange(cam.h, device=device, dtype=dt),
                          torch.arange(cam.w, device=device, dtype=dt), indexing="ij")
    d = torch.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, torch.ones_like(u)],
                    dim=-1).reshape(-1, 3)
    R = torch.as_tensor(np.stack([p[0] for p in poses]), dtype=dt, device=device)
    o = torch.as_tensor(np.stack([p[1] for p in poses]), dtype=dt, device=device)
    dirs = torch.einsum("fij,pj->fpi", R, d)
    Z = _cast_many(scene, o, dirs)
    hit = torch.isfinite(Z)
    Pw = o[:, None, :] + dirs * torch.where(hit, Z, torch.zeros_like(Z))[..., None]
    tex = torch.where(hit, _texture_many(scene, Pw), torch.full_like(Z, 128.0))
    I = torch.clamp(torch.round(tex + sigma_I * torch.randn(tex.shape, generator=gen, device=device,
                                                            dtype=dt)), 0, 255)
    hole = ~hit | (Z < zmin) | (Z > zmax)
    W = torch.where(hole, torch.zeros_like(Z), 1.0 / torch.where(hole, torch.ones_like(Z), Z))
    W = W + torch.randn(W.shape, generator=gen, device=device, dtype=dt) * sigma_W_coef * W * W
    hole |= ~(W > 0)
    if hole_frac > 0:
        # discs of radius U[2, 8] px at uniform centres, about hole_frac of the image
        K = int(round(hole_frac * cam.w * cam.h / 75.0))
        cu = torch.rand((F, K), generator=gen, device=device) * cam.w
        cv = torch.rand((F, K), generator=gen, device=device) * cam.h
        r = 2.0 + 6.0 * torch.rand((F, K), generator=gen, device=device)
        off = torch.arange(-8, 9, device=device, dtype=dt)
        oy, ox = torch.meshgrid(off, off, indexing="ij")
        oy, ox = oy.reshape(-1), ox.reshape(-1)
        py = torch.floor(cv)[..., None] + oy
        px = torch.floor(cu)[..., None] + ox
        inside = ((px + 0.5 - cu[..., None]) ** 2 + (py + 0.5 - cv[..., None]) ** 2 <= (r ** 2)[..., None])
        inside &= (px >= 0) & (px < cam.w) & (py >= 0) & (py < cam.h)
        fi = torch.arange(F, device=device)[:, None, None].expand_as(px)
        flat = (fi * (cam.w * cam.h) + py.long() * cam.w + px.long())[inside]
        hm = hole.reshape(-1)
        hm[flat] = True
        hole = hm.reshape(F, -1)
    W = torch.where(hole, torch.zeros_like(W), W)
    return I.reshape(F, cam.h, cam.w).contiguous(), W.reshape(F, cam.h, cam.w).contiguous()


def warm_pairs(first: int, count: int, split: str = "train", cam: Camera = None,
               pairs_per_scene: int = 32, device="cuda", theta_max=10.0, t_max=0.15):
    """Pairs first .. first+count-1 of the large-motion stream (motion <= 10 deg
    / 15 cm; train and eval use disjoint seeds and scenes).  Returns
    (IA, WA, IB, WB) device tensors (count, h, w) and the true poses of B in A
    as a list of (R, t)."""
    cam = cam or camera_640()
    sid = 15 if split == "train" else 16
    base_scene = 40000 if split == "train" else 70000
    IA, WA, IB, WB, truth = [], [], [], [], []
    i = first
    end = first + count
    while i < end:
        g = i // pairs_per_scene
        j1 = min(end, (g + 1) * pairs_per_scene)
        scene = room_scene(base_scene + g)
        rng = np.random.default_rng(np.random.SeedSequence([1807, sid, g]))
        gen = torch.Generator(device=device)
        gen.manual_seed(int(np.random.SeedSequence([1807, sid, g, 1]).generate_state(1)[0]))
        poses = []
        for k in range(g * pairs_per_scene, (g + 1) * pairs_per_scene):
            yaw = Rotation.from_euler("y", rng.uniform(-15, 15), degrees=True).as_matrix()
            pA = (yaw @ _pitch_down(10.0), np.array([rng.uniform(-0.3, 0.3), 0.0,
                                                      rng.uniform(-0.3, 0.3)]))
            R, t = random_motion(rng, theta_max, t_max)
            if i <= k < j1:
                poses.append((pA, compose(pA, (R, t)), (R, t)))
        frames = [p[0] for p in poses] + [p[1] for p in poses]
        I, W = render_frames(scene, cam, frames, gen, device=device)
        m = len(poses)
        IA.append(I[:m])
        WA.append(W[:m])
        IB.append(I[m:])
        WB.append(W[m:])
        truth += [p[2] for p in poses]
        i = j1
    return torch.cat(IA), torch.cat(WA), torch.cat(IB), torch.cat(WB), truth
