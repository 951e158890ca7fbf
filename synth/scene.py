"""Procedural RGB-D scenes: planes + boxes with a solid Perlin texture.

Conventions
-----------
* Camera pose ``(R_wc, t_wc)`` maps camera to world: ``X_w = R_wc X_c + t_wc``.
  The camera looks along +Z, image-down is +Y, pixel centres are at integer
  (u, v), 0-based, and the pinhole is ``K = [[fx,0,cx],[0,fy,cy],[0,0,1]]``.
* A pair carries the relative pose of B in A, ``(R, t)`` with
  ``X_A = R X_B + t`` (the paper's T_A^B, section 5.2).
* Intensity is in grey levels [0, 255] (integers, exact in FP16); inverse
  depth ``W = 1/Z`` is in 1/m; a hole is stored as 0.

The renderer casts one ray per pixel centre for depth and ``ss x ss``
sub-pixel rays (box filter) for intensity.  The texture is Perlin's improved
gradient noise (Perlin 2002) summed over four octaves, evaluated on world
coordinates so every view of a surface sees the same pattern.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch
from scipy.spatial.transform import Rotation

# --------------------------------------------------------------------------
# cameras


@dataclass(frozen=True)
class Camera:
    w: int
    h: int
    fx: float
    fy: float
    cx: float
    cy: float

    def as_tuple(self):
        return (self.w, self.h, self.fx, self.fy, self.cx, self.cy)


def camera_160() -> Camera:
    return Camera(160, 120, 131.25, 131.25, 79.5, 59.5)


def camera_320() -> Camera:
    return Camera(320, 240, 262.5, 262.5, 159.5, 119.5)


def camera_640() -> Camera:
    return Camera(640, 480, 525.0, 525.0, 319.5, 239.5)


def camera_1280() -> Camera:
    return Camera(1280, 960, 1050.0, 1050.0, 639.5, 479.5)


# --------------------------------------------------------------------------
# rigid poses (scene placement only)


def compose(a, b):
    """(R_a, t_a) o (R_b, t_b)."""
    Ra, ta = a
    Rb, tb = b
    return (Ra @ Rb, Ra @ tb + ta)


def invert(a):
    R, t = a
    return (R.T, -R.T @ t)


def relative(pose_wA, pose_wB):
    """Pose of B in A: X_A = R X_B + t."""
    return compose(invert(pose_wA), pose_wB)


def random_motion(rng: np.random.Generator, theta_max_deg: float, t_max: float):
    """Rotation about a uniform axis by U[0, theta_max], translation along a
    uniform direction by U[0, t_max]."""
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    angle = math.radians(theta_max_deg) * rng.uniform()
    R = Rotation.from_rotvec(axis * angle).as_matrix()
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    t = d * (t_max * rng.uniform())
    return (R, t)


# --------------------------------------------------------------------------
# scenes


@dataclass
class Scene:
    planes: list = field(default_factory=list)   # (n unit (3,), d): n.X = d
    boxes: list = field(default_factory=list)    # (lo (3,), hi (3,))
    perm: np.ndarray = None                      # Perlin permutation (512,)
    octave_offsets: np.ndarray = None            # (4, 3)
    base_freq: float = 4.0                       # cycles per metre


def _texture_params(rng):
    p = rng.permutation(256).astype(np.int64)
    perm = np.concatenate([p, p])
    offs = rng.uniform(0.0, 256.0, size=(4, 3))
    return perm, offs


def planes3_scene(seed: int = 1807) -> Scene:
    """Three planes with linearly independent normals seen by a camera at the
    origin looking down +Z: a tilted back wall, a floor and a left wall."""
    rng = np.random.default_rng(seed)
    perm, offs = _texture_params(rng)
    n_back = np.array([0.1, 0.05, 1.0])
    n_side = np.array([1.0, 0.0, 0.3])
    planes = [
        (n_back / np.linalg.norm(n_back), 2.5),
        (np.array([0.0, 1.0, 0.0]), 0.6),
        (n_side / np.linalg.norm(n_side), -0.3),
    ]
    return Scene(planes=planes, boxes=[], perm=perm, octave_offsets=offs)


def room_scene(seed: int) -> Scene:
    """Floor (Y = 1.2), back wall (Z = 4.5), left wall (X = -2) and 3-5
    axis-aligned boxes of 0.3-1 m standing on the floor 1.5-4 m ahead."""
    rng = np.random.default_rng(seed)
    perm, offs = _texture_params(rng)
    planes = [
        (np.array([0.0, 1.0, 0.0]), 1.2),
        (np.array([0.0, 0.0, 1.0]), 4.5),
        (np.array([1.0, 0.0, 0.0]), -2.0),
    ]
    boxes = []
    for _ in range(int(rng.integers(3, 6))):
        size = rng.uniform(0.3, 1.0, size=3)
        cx = rng.uniform(-1.5, 1.5)
        cz = rng.uniform(1.5, 4.0)
        lo = np.array([cx - size[0] / 2, 1.2 - size[1], cz - size[2] / 2])
        hi = np.array([cx + size[0] / 2, 1.2, cz + size[2] / 2])
        boxes.append((lo, hi))
    return Scene(planes=planes, boxes=boxes, perm=perm, octave_offsets=offs)


def closed_room_scene(seed: int) -> Scene:
    """Closed 8 x 6 x 3 m room (X in [-4,4], Z in [-3,3], Y in [-1.8,1.2])
    with 4 boxes on the floor near the walls."""
    rng = np.random.default_rng(seed)
    perm, offs = _texture_params(rng)
    planes = [
        (np.array([0.0, 1.0, 0.0]), 1.2),     # floor
        (np.array([0.0, 1.0, 0.0]), -1.8),    # ceiling
        (np.array([1.0, 0.0, 0.0]), -4.0),
        (np.array([1.0, 0.0, 0.0]), 4.0),
        (np.array([0.0, 0.0, 1.0]), -3.0),
        (np.array([0.0, 0.0, 1.0]), 3.0),
    ]
    boxes = []
    for (bx, bz) in [(-3.2, 2.2), (3.1, -2.0), (2.8, 2.3), (-2.9, -2.2)]:
        size = rng.uniform(0.4, 1.0, size=3)
        lo = np.array([bx - size[0] / 2, 1.2 - size[1], bz - size[2] / 2])
        hi = np.array([bx + size[0] / 2, 1.2, bz + size[2] / 2])
        boxes.append((lo, hi))
    return Scene(planes=planes, boxes=boxes, perm=perm, octave_offsets=offs)


# --------------------------------------------------------------------------
# ray casting


def _cast(scene: Scene, origin, dirs):
    """Nearest positive hit parameter along origin + s * dirs (dirs (N,3))."""
    dev = dirs.device
    best = torch.full(dirs.shape[:1], math.inf, dtype=torch.float64, device=dev)
    o = torch.as_tensor(origin, dtype=torch.float64, device=dev)
    for n, d in scene.planes:
        nt = torch.as_tensor(n, dtype=torch.float64, device=dev)
        den = dirs @ nt
        num = d - float(np.dot(n, origin))
        s = num / den
        ok = (den != 0) & (s > 1e-9)
        best = torch.where(ok & (s < best), s, best)
    for lo, hi in scene.boxes:
        lo_t = torch.as_tensor(lo, dtype=torch.float64, device=dev)
        hi_t = torch.as_tensor(hi, dtype=torch.float64, device=dev)
        inv = 1.0 / dirs            # +-inf for zero components: slab rule holds
        t1 = (lo_t - o) * inv
        t2 = (hi_t - o) * inv
        tmin = torch.minimum(t1, t2).nan_to_num(nan=-math.inf).amax(dim=1)
        tmax = torch.maximum(t1, t2).nan_to_num(nan=math.inf).amin(dim=1)
        ok = (tmax >= tmin) & (tmin > 1e-9)
        best = torch.where(ok & (tmin < best), tmin, best)
    return best


def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def _grad(h, x, y, z):
    h = h & 15
    u = torch.where(h < 8, x, y)
    v = torch.where(h < 4, y, torch.where((h == 12) | (h == 14), x, z))
    return torch.where((h & 1) == 0, u, -u) + torch.where((h & 2) == 0, v, -v)


def _lerp(t, a, b):
    return a + t * (b - a)


def _perlin(perm, x, y, z):
    fx, fy, fz = torch.floor(x), torch.floor(y), torch.floor(z)
    X = fx.long() & 255
    Y = fy.long() & 255
    Z = fz.long() & 255
    x, y, z = x - fx, y - fy, z - fz
    u, v, w = _fade(x), _fade(y), _fade(z)
    A = perm[X] + Y
    AA = perm[A] + Z
    AB = perm[A + 1] + Z
    B = perm[X + 1] + Y
    BA = perm[B] + Z
    BB = perm[B + 1] + Z
    x1, y1, z1 = x - 1.0, y - 1.0, z - 1.0
    return _lerp(
        w,
        _lerp(v, _lerp(u, _grad(perm[AA], x, y, z), _grad(perm[BA], x1, y, z)),
              _lerp(u, _grad(perm[AB], x, y1, z), _grad(perm[BB], x1, y1, z))),
        _lerp(v, _lerp(u, _grad(perm[AA + 1], x, y, z1), _grad(perm[BA + 1], x1, y, z1)),
              _lerp(u, _grad(perm[AB + 1], x, y1, z1), _grad(perm[BB + 1], x1, y1, z1))))


def _texture(scene: Scene, P):
    """Grey level of the solid texture at world points P (N,3)."""
    perm = torch.as_tensor(scene.perm, device=P.device)
    offs = torch.as_tensor(scene.octave_offsets, dtype=torch.float64, device=P.device)
    acc = torch.zeros(P.shape[0], dtype=torch.float64, device=P.device)
    freq, amp = scene.base_freq, 1.0
    for o in range(4):
        Q = P * freq + offs[o]
        acc = acc + amp * _perlin(perm, Q[:, 0], Q[:, 1], Q[:, 2])
        freq *= 2.0
        amp *= 0.5
    return 128.0 + 100.0 * acc


def render(scene: Scene, cam: Camera, pose_wc, ss: int = 4, device="cpu",
           max_rays: int = 1 << 21):
    """Depth Z along the optical axis (pixel-centre ray; inf on a miss) and the
    box-filtered texture value over ss x ss sub-pixel rays, both float64."""
    R, t = pose_wc
    Rt = torch.as_tensor(R, dtype=torch.float64, device=device)
    o = np.asarray(t, dtype=np.float64)
    ot = torch.as_tensor(o, dtype=torch.float64, device=device)
    Z = np.empty((cam.h, cam.w))
    I = np.empty((cam.h, cam.w))
    sub = (torch.arange(ss, dtype=torch.float64, device=device) + 0.5) / ss - 0.5
    rows = max(1, max_rays // (cam.w * ss * ss))
    u = torch.arange(cam.w, dtype=torch.float64, device=device)
    for r0 in range(0, cam.h, rows):
        r1 = min(cam.h, r0 + rows)
        v = torch.arange(r0, r1, dtype=torch.float64, device=device)
        # centre rays
        vv, uu = torch.meshgrid(v, u, indexing="ij")
        d = torch.stack([(uu - cam.cx) / cam.fx, (vv - cam.cy) / cam.fy,
                         torch.ones_like(uu)], dim=-1).reshape(-1, 3)
        s = _cast(scene, o, d @ Rt.T)
        Z[r0:r1] = s.reshape(r1 - r0, cam.w).cpu().numpy()
        # sub-pixel rays for intensity
        vs = (v[:, None] + sub[None, :]).reshape(-1)
        us = (u[:, None] + sub[None, :]).reshape(-1)
        vv, uu = torch.meshgrid(vs, us, indexing="ij")
        d = torch.stack([(uu - cam.cx) / cam.fx, (vv - cam.cy) / cam.fy,
                         torch.ones_like(uu)], dim=-1).reshape(-1, 3)
        dw = d @ Rt.T
        s = _cast(scene, o, dw)
        hit = torch.isfinite(s)
        P = ot + dw * torch.where(hit, s, torch.zeros_like(s))[:, None]
        tex = torch.where(hit, _texture(scene, P), torch.full_like(s, 128.0))
        tex = tex.reshape(r1 - r0, ss, cam.w, ss).mean(dim=(1, 3))
        I[r0:r1] = tex.cpu().numpy()
    return Z, I


# --------------------------------------------------------------------------
# sensor model


@dataclass
class Frame:
    I: np.ndarray      # float32 (h, w), grey levels
    W: np.ndarray      # float32 (h, w), 1/m, 0 = hole
    pose_wc: tuple     # (R, t) camera-to-world


def _blob_holes(rng, mask, target_frac, rmin=2.0, rmax=8.0):
    h, w = mask.shape
    vv, uu = np.mgrid[0:h, 0:w]
    while mask.mean() < target_frac:
        cu, cv = rng.uniform(0, w), rng.uniform(0, h)
        r = rng.uniform(rmin, rmax)
        u0, u1 = int(max(0, cu - r - 1)), int(min(w, cu + r + 2))
        v0, v1 = int(max(0, cv - r - 1)), int(min(h, cv + r + 2))
        sub = (uu[v0:v1, u0:u1] - cu) ** 2 + (vv[v0:v1, u0:u1] - cv) ** 2 <= r * r
        mask[v0:v1, u0:u1] |= sub
    return mask


def make_frame(scene: Scene, cam: Camera, pose_wc, rng: np.random.Generator,
               sigma_I: float = 2.0, sigma_W="quadratic", sigma_W_coef: float = 1.5e-3,
               zmin: float = 0.5, zmax: float = 5.0, hole_frac: float = 0.0,
               ss: int = 4, device="cpu") -> Frame:
    """Render and corrupt one frame.

    sigma_W: "quadratic" gives sigma_W = coef * W^2 (a constant depth sigma
    propagated to inverse depth), "constant" gives sigma_W = coef.
    """
    Z, tex = render(scene, cam, pose_wc, ss=ss, device=device)
    I = np.clip(np.round(tex + rng.normal(0.0, sigma_I, size=tex.shape)), 0, 255)
    hole = ~np.isfinite(Z) | (Z < zmin) | (Z > zmax)
    with np.errstate(divide="ignore"):
        W = np.where(hole, 0.0, 1.0 / np.where(hole, 1.0, Z))
    if sigma_W == "quadratic":
        sW = sigma_W_coef * W * W
    else:
        sW = np.full_like(W, sigma_W_coef)
    W = W + rng.normal(0.0, 1.0, size=W.shape) * sW
    hole |= ~(W > 0)
    if hole_frac > 0:
        hole = _blob_holes(rng, hole, hole_frac)
    W = np.where(hole, 0.0, W)
    return Frame(I.astype(np.float32), W.astype(np.float32), pose_wc)


def to_fp16_grid(x: np.ndarray) -> np.ndarray:
    """Round to the nearest binary16 value and return it as float32."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


# --------------------------------------------------------------------------
# workloads


@dataclass
class Pair:
    cam: Camera
    A: Frame
    B: Frame
    R: np.ndarray      # true pose of B in A
    t: np.ndarray


def _seed(*parts) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([1807, *parts]))


def _pitch_down(deg):
    return Rotation.from_euler("x", -deg, degrees=True).as_matrix()


def pair_c1(i: int, ss: int = 4, noise: bool = True, device="cpu") -> Pair:
    """160x120 three-plane pair, sigma_I = 2, sigma_W = 0.002, motion
    <= 2 deg / <= 3 cm, no holes beyond the 0.5-5 m range."""
    cam = camera_160()
    scene = planes3_scene()
    rng = _seed(1, i)
    pose_A = (np.eye(3), np.zeros(3))
    R, t = random_motion(rng, 2.0, 0.03)
    pose_B = compose(pose_A, (R, t))
    sI = 2.0 if noise else 0.0
    sW = 0.002 if noise else 0.0
    A = make_frame(scene, cam, pose_A, rng, sigma_I=sI, sigma_W="constant",
                   sigma_W_coef=sW, ss=ss, device=device)
    B = make_frame(scene, cam, pose_B, rng, sigma_I=sI, sigma_W="constant",
                   sigma_W_coef=sW, ss=ss, device=device)
    return Pair(cam, A, B, R, t)


def _room_pair(cam, scene_seed, rng, theta_max, t_max, ss, device, hole_frac=0.10,
               noise=True):
    scene = room_scene(scene_seed)
    yaw = Rotation.from_euler("y", rng.uniform(-15, 15), degrees=True).as_matrix()
    pose_A = (yaw @ _pitch_down(10.0), np.array([rng.uniform(-0.3, 0.3), 0.0,
                                                  rng.uniform(-0.3, 0.3)]))
    R, t = random_motion(rng, theta_max, t_max)
    pose_B = compose(pose_A, (R, t))
    kw = dict(sigma_I=2.0 if noise else 0.0, sigma_W="quadratic",
              sigma_W_coef=1.5e-3 if noise else 0.0, hole_frac=hole_frac, ss=ss,
              device=device)
    A = make_frame(scene, cam, pose_A, rng, **kw)
    B = make_frame(scene, cam, pose_B, rng, **kw)
    return Pair(cam, A, B, R, t)


def pair_c2(i: int, cam: Camera = None, ss: int = 4, device="cpu", noise=True) -> Pair:
    """640x480 room + boxes pair, 10% holes, sigma_W = 1.5e-3 W^2,
    motion <= 2 deg / <= 3 cm."""
    cam = cam or camera_640()
    rng = _seed(2, i, cam.w)
    return _room_pair(cam, 7000 + i % 16, rng, 2.0, 0.03, ss, device, noise=noise)


def pair_warm(i: int, split: str = "train", cam: Camera = None, ss: int = 2,
              device="cpu") -> Pair:
    """Large-motion room pair (<= 10 deg / <= 15 cm); train and eval draw from
    disjoint seed streams and disjoint scene seeds."""
    cam = cam or camera_640()
    sid = 5 if split == "train" else 6
    rng = _seed(sid, i)
    scene_seed = (20000 if split == "train" else 90000) + i % 997
    return _room_pair(cam, scene_seed, rng, 10.0, 0.15, ss, device)


def batch_c4(ss: int = 2, device="cpu", counts=(24, 32, 8)):
    """Mixed-size batch: 320x240, 640x480 and 1280x960 pairs from the room
    generator."""
    pairs = []
    for cam, n in zip((camera_320(), camera_640(), camera_1280()), counts):
        for i in range(n):
            pairs.append(pair_c2(1000 + i, cam=cam, ss=ss, device=device))
    return pairs


def keyframe_sequence(n_frames: int = 20, seed: int = 0, cam: Camera = None,
                      ss: int = 4, device="cpu", noise=True):
    """A keyframe and n_frames frames on a random walk (<= 2 deg / <= 3 cm per
    step) that starts at the keyframe pose.  Returns (cam, kf, frames, poses)
    with poses[k] = pose of frame k in the keyframe."""
    cam = cam or camera_640()
    rng = _seed(3, seed)
    scene = room_scene(8000 + seed)
    pose_kf = (_pitch_down(10.0), np.zeros(3))
    kw = dict(sigma_I=2.0 if noise else 0.0, sigma_W="quadratic",
              sigma_W_coef=1.5e-3 if noise else 0.0, hole_frac=0.10 if noise else 0.0,
              ss=ss, device=device)
    kf = make_frame(scene, cam, pose_kf, rng, **kw)
    frames, poses = [], []
    pose = pose_kf
    for _ in range(n_frames):
        pose = compose(pose, random_motion(rng, 2.0, 0.03))
        frames.append(make_frame(scene, cam, pose, rng, **kw))
        poses.append(relative(pose_kf, pose))
    return cam, kf, frames, poses


def _dist_to_surfaces(scene: Scene, p):
    d = min(abs(float(np.dot(n, p)) - dd) for n, dd in scene.planes)
    for lo, hi in scene.boxes:
        q = np.maximum(np.maximum(lo - p, p - hi), 0.0)
        d = min(d, float(np.linalg.norm(q)))
    return d


def walk_c3(n_frames: int = 300, seed: int = 0, cam: Camera = None, ss: int = 2,
            device="cpu", render_frames: bool = True):
    """Random-walk trajectory in a closed room (<= 2 deg / <= 3 cm per step;
    steps that come within 0.6 m of a surface are redrawn).  Frames are float32;
    round them with to_fp16_grid for FP16 storage."""
    cam = cam or camera_640()
    rng = _seed(4, seed)
    scene = closed_room_scene(9000 + seed)
    pose = (np.eye(3), np.array([0.0, 0.0, -0.5]))
    poses = [pose]
    while len(poses) < n_frames:
        cand = compose(poses[-1], random_motion(rng, 2.0, 0.03))
        if _dist_to_surfaces(scene, cand[1]) >= 0.6:
            poses.append(cand)
    frames = None
    if render_frames:
        kw = dict(sigma_I=2.0, sigma_W="quadratic", sigma_W_coef=1.5e-3,
                  hole_frac=0.0, ss=ss, device=device)
        frames = [make_frame(scene, cam, p, rng, **kw) for p in poses]
    return cam, scene, poses, frames


def track_sequence(n_frames: int, step_deg: float, step_m: float, seed: int = 0,
                   cam: Camera = None, ss: int = 2, device="cpu", noise: bool = True,
                   axis=(0.0, 1.0, 0.0)):
    """Constant-velocity sequence in the room scene: every step turns the
    camera by step_deg about `axis` (camera coordinates) and moves it step_m
    along its own x axis, so the view drifts steadily away from the first
    frame.  Returns (cam, poses, frames) with poses camera-to-world."""
    cam = cam or camera_160()
    rng = _seed(5, seed)
    scene = room_scene(9500 + seed)
    step = (Rotation.from_rotvec(np.radians(step_deg) * np.asarray(axis, float)).as_matrix(),
            np.array([step_m, 0.0, 0.0]))
    pose = (_pitch_down(10.0), np.array([-0.3, 0.0, 0.0]))
    kw = dict(sigma_I=2.0 if noise else 0.0, sigma_W="quadratic",
              sigma_W_coef=1.5e-3 if noise else 0.0, hole_frac=0.0, ss=ss, device=device)
    poses, frames = [], []
    for _ in range(n_frames):
        poses.append(pose)
        frames.append(make_frame(scene, cam, pose, rng, **kw))
        pose = compose(pose, step)
    return cam, poses, frames
