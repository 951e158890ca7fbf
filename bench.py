#!/usr/bin/env python3
"""Throughput of dense RGB-D alignment + keyframe fusion on one MI355X.

Workload (one "step"): a batch of 640x480 frame pairs from the room + boxes
generator (10% holes, inverse-depth noise 1.5e-3 W^2, motion <= 2 deg / 3 cm,
Kinect-like camera fx = fy = 525, cx = 319.5, cy = 239.5):
  1. pyramids (4 levels) of both frames of every pair, rebuilt from the
     resident level-0 images;
  2. batched coarse-to-fine alignment of all pairs: 4 levels x 10 Gauss-Newton
     iterations, paper-literal full-resolution warp, Huber weights, FP32
     per-pixel arithmetic;
  3. fusion of 20 frames (ground-truth poses) into one 640x480 keyframe
     (one batched launch; the same result as 20 single-frame calls).
value = aligned pairs per second over the timed steps (inputs already in HBM).

Also reported: the roofline of the dominant kernel (algorithmic bytes per
launch / HIP-event-timed average launch duration, against 8 TB/s; and, where
a counter summary of the current kernel sources is committed, its measured
HBM bytes and its VALU issue rate against the chip's), and the FP64 CPU
oracle timed on a bounded sample of the same workload.

python bench.py [--steps K] [--warmup W] [--pairs P] [--storage f32|f16]
                [--warp fullres|per_level] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "640×480 frame-pair alignments/s + HBM GB/s, warm-start vs plain GN"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(level, kernel, sizes, f16, warp_fullres, fused):
    """Bytes the method must move for one launch of (level, kernel) over the
    batch (sizes: level-0 (w, h) of every pair).  Per pixel, FP32 storage: a
    level-0 pixel of the full-resolution warp needs W_A (4 B) and I_B, W_B
    (8 B); the residual of a level pixel needs I_A, W_A (8 B); a stored warped
    level image is 8 B per level pixel (written once, read once).  FP16
    storage halves the image bytes."""
    e = 2 if f16 else 4
    total = 0
    for w0, h0 in sizes:
        n0 = w0 * h0
        nl = (w0 >> level) * (h0 >> level)
        nw = n0 if warp_fullres else nl       # pixels warped per iteration
        if kernel == "reduce":
            if fused:       # warp + residual in one kernel
                total += nw * 3 * e + nl * 2 * e - (nl * e if nw == nl else 0)
            else:
                total += nl * (2 * e + 8)
        elif kernel == "warp":
            if fused:       # sample pixels only: not a bandwidth kernel
                return None
            total += nw * 3 * e + nl * 8
        else:
            return None
    return total


# FP32 vector peak without packed math (the build disables packed FP32):
# 256 CUs x 64 lanes x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s; the published
# 157.3 TFLOP/s counts packed FP32.
FP32_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# VALU issue: one wave64 instruction per SIMD every 4 cycles
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4

# FP32 matrix-core peak (MI355X, dense FP32 MFMA): 157.3 TFLOP/s.
MFMA_FP32_PEAK_TFLOPS = 157.3

# Algorithmic FP32 flops (an FMA counts 2) the method needs, per unit, on
# the vector ALUs:
#   a warped full-resolution child: ray and rotation 22, projection 8,
#   bilinear weights 6 and two 4-tap interpolations 16, W* 5  -> 57;
#   its share of the level mean (two channels)                 -> 2;
#   a level pixel's residual terms: residuals 2, gradients 8, two Jacobians
#   38, lambda_n 12, two robust weights 12                     -> 72;
#   a sample residual pair                                      -> 2;
# and on the matrix cores: a level pixel's two rank-one updates of the
# 21 + 6 + 1 normal-equation sums (w J, then multiply-adds)     -> 124.
FLOPS_CHILD, FLOPS_MEAN, FLOPS_TERMS, FLOPS_SAMPLE = 57, 2, 72, 2
FLOPS_NE_MFMA = 124


def algorithmic_flops(level, kernel, sizes, warp_fullres, fused):
    """FP32 vector-ALU flops of one launch of (level, kernel) over the batch
    (the normal-equation sums, which run on the matrix cores, excluded)."""
    total = 0
    for w0, h0 in sizes:
        n0 = w0 * h0
        nl = (w0 >> level) * (h0 >> level)
        nw = n0 if warp_fullres else nl
        if kernel == "reduce":
            total += nl * FLOPS_TERMS
            if fused:
                total += nw * (FLOPS_CHILD + (FLOPS_MEAN if nw != nl else 0))
        elif kernel == "warp":
            if fused:
                return None
            total += nw * (FLOPS_CHILD + (FLOPS_MEAN if nw != nl else 0)) + nl * FLOPS_SAMPLE
        else:
            return None
    return total


def counter_summary():
    """The machine-readable block of the committed rocprofv3 counter summary
    of this workload, if it was taken on the current kernel sources."""
    from paper_1807_08271_amd.build import source_sha
    path = os.path.join(ROOT, "profiles", "rgbid_counters_64x640x480_fullres_f32.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    i = txt.find("```json")
    if i < 0:
        return None
    j = txt.find("```", i + 7)
    try:
        d = json.loads(txt[i + 7:j])
    except ValueError:
        return None
    return d if d.get("source_sha") == source_sha() else None


def make_inputs(npairs, device, mixed=False):
    import synth
    t0 = time.time()
    if mixed:
        pairs = synth.batch_c4(ss=2, device=device)
    else:
        pairs = [synth.pair_c2(i, ss=2, device=device) for i in range(npairs)]
    cam, kf, frames, poses = synth.keyframe_sequence(20, seed=0, ss=2, device=device)
    log("generated %d pairs + 21 fusion frames in %.1fs" % (npairs, time.time() - t0))
    return pairs, (cam, kf, frames, poses)


def cpu_baseline(pairs, fusion, oparams, budget_s):
    """The FP64 oracle on a bounded sample of the step, two ways:
    one core: whole alignments of the first pairs until budget_s is spent
    (at least one), plus one 20-frame fusion, scaled to the step (P
    alignments + one fusion);
    all cores: one pair per worker thread (the oracle's C call runs without
    the interpreter lock), four pairs per thread over the usable host cores
    (at most 16, this machine class's CPU share per GPU), timed on the wall
    clock; the step's fusion runs on one thread, as the oracle's fusion is
    one call per frame.  value is the all-core figure."""
    import concurrent.futures as cf
    import numpy as np
    import oracle
    oracle.build(force=False)
    t_al, n = 0.0, 0
    for p in pairs:
        t0 = time.perf_counter()
        oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, oparams)
        t_al += time.perf_counter() - t0
        n += 1
        if t_al >= budget_s:
            break
    cam, kf, frames, poses = fusion
    W = kf.W.astype(np.float64)
    C = np.ones_like(W)
    t0 = time.perf_counter()
    for f, (R, t) in zip(frames, poses):
        W, C, _ = oracle.fuse(cam, W, C, f.W, R, t, 0.01)
    t_fu = time.perf_counter() - t0
    per_align = t_al / n
    P = len(pairs)
    one = P / (P * per_align + t_fu)
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    threads = max(1, min(16, usable))
    jobs = [pairs[i % P] for i in range(4 * threads)]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda p: oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, oparams), jobs))
    t_all = time.perf_counter() - t0
    rate = len(jobs) / t_all
    value = P / (P / rate + t_fu)
    log("oracle: one core %.3f alignments/s; %d threads %.3f alignments/s (%d pairs in %.1f s)" % (
        one, threads, value, len(jobs), t_all))
    return {"value": round(value, 3), "unit": "alignments/s", "cores": threads, "kind": "oracle",
            "host_cpus": os.cpu_count(), "usable_cpus": usable,
            "one_core": {"value": round(one, 3), "cores": 1,
                         "s_per_alignment": round(per_align, 3)},
            "sample": "all cores: %d step pairs aligned by the FP64 C oracle, one pair per "
                      "thread on %d threads, %.1f s wall (%.2f alignments/s), plus one 20-frame "
                      "fusion on one thread (%.2f s), scaled to one step; one core: %d pairs at "
                      "%.2f s each + the fusion" % (len(jobs), threads, t_all, rate, t_fu, n,
                                                    per_align)}


def warmstart_compare(ctx, npairs, steps):
    """Plain Gauss-Newton from the identity against the learned warm start +
    Gauss-Newton on a batch of held-out large-motion pairs (<= 10 deg / 15 cm):
    alignments/s over `steps` timed repetitions (network input + forward
    included for the warm start) and the success rate (final pose within
    1e-5 rad / 1e-5 m of the Gauss-Newton optimum reached from the true pose),
    both with early stop at 1e-6."""
    import numpy as np
    import torch
    from paper_1807_08271_amd import rgbid as rg
    from paper_1807_08271_amd import warmstart as ws
    net = rg.rgbid_warmstart_create(ctx, ws.load_weights())
    st = ws.PairStream(ctx, npairs)
    m, truth = st.load(0, npairs, "eval")
    ref, rstats = rg.rgbid_align_batch(ctx, st.As[:m], st.Bs[:m], ws.label_params(), inits=truth)
    prm = ws.eval_params()
    res = {}
    for name in ("plain", "warm"):
        def run():
            if name == "warm":   # network, initial poses and alignment in one call
                return rg.rgbid_align_batch_warm(ctx, net, st.As[:m], st.Bs[:m], prm)
            return rg.rgbid_align_batch(ctx, st.As[:m], st.Bs[:m], prm)
        poses, stats = run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            poses, stats = run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = [ws._close(poses[i], ref[i], 1e-5, 1e-5) and stats[i]["status"] == 0
              for i in range(m) if rstats[i]["status"] == 0]
        iters = [sum(stats[i]["iters_done"]) for i in range(m) if rstats[i]["status"] == 0]
        res[name] = {"alignments_per_s": round(m * steps / dt, 1),
                     "success_rate": round(float(np.mean(ok)), 4),
                     "mean_gn_iters": round(float(np.mean(iters)), 2),
                     "ms_per_batch": round(1e3 * dt / steps, 4)}
        if name == "warm":
            # the network's share: input assembly, forward and the initial
            # poses, on their own
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                rg.rgbid_warmstart_predict(ctx, net, st.As[:m], st.Bs[:m], st.x)
            torch.cuda.synchronize()
            res[name]["predict_ms_per_batch"] = round(1e3 * (time.perf_counter() - t0) / steps, 4)
        log("warm-start comparison %-5s: %s" % (name, res[name]))
    st.close()
    rg.rgbid_warmstart_free(net)
    res["workload"] = ("%d held-out 640x480 pairs, motion <= 10 deg / 15 cm, 4 levels x <= 10 "
                       "iterations, early stop 1e-6" % m)
    return res


def batched_c4(ctx, steps, warmup, storage_name="f32"):
    """The batched form at its own shapes: 24 x 320x240 + 32 x 640x480 +
    8 x 1280x960 pairs (room + boxes, 10% holes; about 21.5 M level-0 pixels,
    a working set of ~400 MB in FP32, above the 256 MB Infinity Cache) aligned
    in one batch, 4 levels x 10 Huber iterations, FULLRES, autotuned launch
    shapes.  A step rebuilds the 128 pyramids and aligns the batch
    (asynchronous form).  Reports alignments/s and, per level, the
    warp-reduce kernels' algorithmic bytes over their HIP-event-timed launch
    durations against 8 TB/s."""
    import numpy as np
    import torch
    import synth
    from paper_1807_08271_amd import rgbid as rg
    t0 = time.time()
    pairs = synth.batch_c4(ss=2, device="cuda")
    log("c4: generated %d mixed-size pairs in %.1fs" % (len(pairs), time.time() - t0))
    f16 = storage_name == "f16"
    storage = rg.RGBID_F16 if f16 else rg.RGBID_F32
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    imgs = [(up(p.A.I), up(p.A.W), up(p.B.I), up(p.B.W)) for p in pairs]
    As = [rg.rgbid_pyramid(ctx, p.cam, 4, storage, x[0], x[1]) for p, x in zip(pairs, imgs)]
    Bs = [rg.rgbid_pyramid(ctx, p.cam, 4, storage, x[2], x[3]) for p, x in zip(pairs, imgs)]
    all_pyr = As + Bs
    all_I = [x[0] for x in imgs] + [x[2] for x in imgs]
    all_W = [x[1] for x in imgs] + [x[3] for x in imgs]
    sizes = [(p.cam.w, p.cam.h) for p in pairs]
    n = len(pairs)
    prm = rg.rgbid_default_params(levels=4, iters=[10] * 4, weight=rg.RGBID_W_HUBER)
    t0 = time.time()
    tuned = [round(1e3 * b, 2) for b in rg.rgbid_autotune(ctx, As, Bs, prm, reps=3)]
    log("c4: autotuned in %.1fs: us/iteration per level %s" % (time.time() - t0, tuned))
    tune_txt = os.path.join("/tmp", "rgbid_bench_c4_tune_%d.txt" % os.getpid())
    rg.rgbid_tune_save(ctx, tune_txt)
    key = "_".join("%dx%dx%d" % (w, h, sizes.count((w, h))) for w, h in dict.fromkeys(sizes))
    fused_level = {}
    for line in open(tune_txt):
        f = line.split()
        if len(f) == 6 and f[0].split("_", 1)[1] == "m0_f%d_%s" % (int(f16), key):
            fused_level[int(f[0].split("_")[0][1:])] = f[1] == "1"
    os.remove(tune_txt)
    pose_buf = torch.empty(n * rg.POSE_BYTES, dtype=torch.uint8, device="cuda")

    def step():
        rg.rgbid_pyramid_update_batch(ctx, all_pyr, all_I, all_W)
        rg.rgbid_align_batch_async(ctx, As, Bs, prm, pose_buf)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    poses = rg.unpack_poses(pose_buf, n)
    import oracle
    err = max(float(np.linalg.norm(oracle.log_so3(R.T @ p.R))) for (R, _), p in zip(poses, pairs))
    log("c4: %d steps, %.3f ms/step, %.1f alignments/s" % (steps, 1e3 * dt / steps, n * steps / dt))
    rg.rgbid_set_profiling(ctx, True)
    for _ in range(max(2, steps // 4)):
        rg.rgbid_align_batch(ctx, As, Bs, prm)
    torch.cuda.synchronize()
    kt = rg.rgbid_kernel_times(ctx)
    rg.rgbid_set_profiling(ctx, False)
    levels = {}
    for (lvl, kname), (ms, nl) in sorted(kt.items()):
        if kname not in ("warp", "reduce"):
            continue
        fused = fused_level.get(lvl, lvl == 0)
        b = algorithmic_bytes(lvl, kname, sizes, f16, True, fused)
        us = 1e3 * ms / nl
        e = levels.setdefault("level%d" % lvl, {"fused_warp_reduce": fused})
        e["%s_avg_us" % kname] = round(us, 2)
        if b is not None:
            e["%s_bytes" % kname] = b
            e["%s_GBs" % kname] = round(b / (us * 1e-6) / 1e9, 1)
            e["%s_hbm_frac" % kname] = round(b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
    for lvl, e in levels.items():
        b = e.get("warp_bytes", 0) + e.get("reduce_bytes", 0)
        us = (e.get("warp_avg_us", 0.0) if "warp_bytes" in e else 0.0) + e.get("reduce_avg_us", 0.0)
        e["warp_reduce_hbm_frac"] = round(b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
        log("c4 %s: %s" % (lvl, e))
    for P in all_pyr:
        rg.rgbid_pyramid_free(P)
    return {"workload": "24 x 320x240 + 32 x 640x480 + 8 x 1280x960 pairs (room+boxes, 10%% "
                        "holes), 4-level FULLRES warp, 10 Huber GN iterations per level, %s; "
                        "step = 128 pyramids + the batched alignment" % storage_name,
            "alignments_per_s": round(n * steps / dt, 1), "ms_per_step": round(1e3 * dt / steps, 4),
            "steps": steps, "level0_pixels": int(sum(w * h for w, h in sizes)),
            "autotuned_us_per_iteration": tuned, "max_rot_err_vs_truth_rad": err,
            "levels": levels}


# Synthetic Kinect-like calibration for the sensor input path (Brown
# coefficients k1 k2 p1 p2 k3, depth correction, spatial correction, depth ->
# colour extrinsics): values of the order such sensors have, not a fit.
SENSOR_K_COLOR = [0.12, -0.25, 0.0015, -0.001, 0.1]
SENSOR_K_DEPTH = [-0.08, 0.15, -0.001, 0.0008, -0.05]
SENSOR_Q0 = [1e-3, 2e-3, -1e-3, 5e-4, 1e-3, -2e-3, 1e-3, 5e-4, -5e-4]
SENSOR_Q1 = [1.01, -0.02, 0.01, 0.005, 0.01, -0.01, 0.005, 0.002, -0.002]


def frontend_measure(ctx, pair, reps=20):
    """The entry points around the alignment at 640x480, each timed per call
    on the host clock (the calls read their results back, so every figure
    includes launch and read-back): pose covariance (bilateral filter + one
    filtered linearisation), the covisibility ratio at level 2, the tracking
    front-end over a constant-velocity sequence (alignment against the
    reference, covisibility, switching, odometry covariance, fusion per
    frame), and the sensor input path (depth correction, undistortion and
    forward registration)."""
    import numpy as np
    import torch
    from scipy.spatial.transform import Rotation
    import synth
    from paper_1807_08271_amd import rgbid as rg
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()

    def per_call_us(fn, n):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return round((time.perf_counter() - t0) / n * 1e6, 1)

    out = {"workload": "640x480; pair 0 of the batch at its aligned pose; a 16-frame "
                       "constant-velocity room sequence (2 deg, 2 cm per frame); one rendered "
                       "room frame through a synthetic Kinect-like calibration"}
    prm = rg.rgbid_default_params(levels=4, iters=[10] * 4, weight=rg.RGBID_W_HUBER)
    A = rg.rgbid_pyramid(ctx, pair.cam, 4, rg.RGBID_F32, up(pair.A.I), up(pair.A.W))
    B = rg.rgbid_pyramid(ctx, pair.cam, 4, rg.RGBID_F32, up(pair.B.I), up(pair.B.W))
    R, t, _, _ = rg.rgbid_align(ctx, A, B, prm)
    out["align_one_pair_us"] = per_call_us(lambda: rg.rgbid_align(ctx, A, B, prm), reps)
    out["covariance_us"] = per_call_us(lambda: rg.rgbid_covariance(ctx, A, B, (R, t), prm), reps)
    out["covisibility_us"] = per_call_us(
        lambda: rg.rgbid_covisibility(ctx, A, B, 2, (R, t), 0.01), reps)
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)

    cam, _, frames = synth.track_sequence(16, 2.0, 0.02, seed=1, cam=synth.camera_640(), ss=2)
    tp = rg.rgbid_tracker_default_params(align=prm)
    trk = rg.rgbid_tracker_create(ctx, cam, 4, rg.RGBID_F32, tp)
    Is, Ws = [up(f.I) for f in frames], [up(f.W) for f in frames]
    rg.rgbid_track(ctx, trk, Is[0], Ws[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, len(frames)):
        rg.rgbid_track(ctx, trk, Is[k], Ws[k])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / (len(frames) - 1) * 1e3
    out["tracker_ms_per_frame"] = round(ms, 3)
    out["tracker_frames_per_s"] = round(1e3 / ms, 1)
    rg.rgbid_tracker_free(trk)

    color = synth.camera_640()
    depth = synth.Camera(640, 480, 575.8, 575.8, 319.5, 239.5)
    scene = synth.room_scene(7006)
    Z, I = synth.render(scene, color, (Rotation.from_euler("x", -10, degrees=True).as_matrix(),
                                       np.zeros(3)), ss=1)
    Z = np.where(np.isfinite(Z) & (Z > 0.5) & (Z < 5.0), Z, 0.0)
    S = rg.make_sensor(color, depth, k_color=SENSOR_K_COLOR, k_depth=SENSOR_K_DEPTH, beta0=0.002,
                       beta1=0.995, p0=(4, 4), spatial=True, q0=SENSOR_Q0, q1=SENSOR_Q1,
                       R_dc=Rotation.from_rotvec([0.002, -0.003, 0.001]).as_matrix(),
                       t_dc=np.array([0.025, 0.001, -0.002]))
    gI, gZ = up(I), up(Z)
    oI, oW = rg.rgbid_preprocess(ctx, S, gI, gZ)
    out["preprocess_us"] = per_call_us(lambda: rg.rgbid_preprocess(ctx, S, gI, gZ, oI, oW), reps)
    L = rg.make_lens(color, SENSOR_K_COLOR)
    out["undistort_us"] = per_call_us(lambda: rg.rgbid_undistort(ctx, L, gI, False, oI), reps)
    log("front-end (per call, host clock): %s" % {k: v for k, v in out.items() if k != "workload"})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pairs", type=int, default=64)
    ap.add_argument("--storage", choices=["f32", "f16"], default="f32")
    ap.add_argument("--warp", choices=["fullres", "per_level"], default="fullres")
    ap.add_argument("--weight", choices=["huber", "student_t"], default="huber")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--scale-cold", action="store_true",
                    help="every iteration's location / scale fixed point starts from mu = 0, "
                         "sigma^2 = mean r^2 and takes all 20 steps (default: warm start from "
                         "the previous iteration with the 2^-16 sigma convergence stop)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--batch", choices=["uniform", "mixed"], default="uniform",
                    help="uniform: --pairs pairs at 640x480 (the headline workload); mixed: "
                         "24 x 320x240 + 32 x 640x480 + 8 x 1280x960 pairs (batched form)")
    ap.add_argument("--no-warmstart", action="store_true")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the batched mixed-size block (24 x 320x240 + 32 x 640x480 + "
                         "8 x 1280x960 pairs, per-level warp-reduce HBM fractions)")
    ap.add_argument("--no-frontend", action="store_true",
                    help="skip the per-call timings of covariance, covisibility, tracker, sensor path")
    ap.add_argument("--frontend-only", action="store_true",
                    help="only the front-end timings (for a kernel trace of those entry points)")
    ap.add_argument("--ws-pairs", type=int, default=64)
    ap.add_argument("--tune-file", default=None, help="load tuned launch shapes from this file")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB float32 tensor 3 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": 4 * n, "copy_bytes_written_per_launch": 4 * n,
                          "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent pairs would shard across GPUs with no exchange); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import oracle
    from paper_1807_08271_amd import rgbid as rg

    torch.cuda.set_device(0)
    dev = "cuda"
    mixed = args.batch == "mixed"
    pairs, fusion = make_inputs(args.pairs, dev, mixed)
    if mixed:
        args.pairs = len(pairs)
    cam = pairs[0].cam
    sizes = [(p.cam.w, p.cam.h) for p in pairs]
    f16 = args.storage == "f16"
    storage = rg.RGBID_F16 if f16 else rg.RGBID_F32

    ctx = rg.rgbid_create(0)
    if args.frontend_only:
        print(json.dumps({"frontend": frontend_measure(ctx, pairs[0])}), flush=True)
        rg.rgbid_destroy(ctx)
        return
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    IA = [up(p.A.I) for p in pairs]
    WA = [up(p.A.W) for p in pairs]
    IB = [up(p.B.I) for p in pairs]
    WB = [up(p.B.W) for p in pairs]
    As = [rg.rgbid_pyramid(ctx, p.cam, 4, storage, i, w) for p, i, w in zip(pairs, IA, WA)]
    Bs = [rg.rgbid_pyramid(ctx, p.cam, 4, storage, i, w) for p, i, w in zip(pairs, IB, WB)]
    fcam, kf, frames, fposes = fusion
    kfW = up(kf.W)
    fW = [up(f.W) for f in frames]
    # The keyframe fusion does not depend on the alignments of the step, so
    # it runs in a context of its own on a second stream (default priority)
    # and overlaps them, as a tracking loop and a mapping loop would.
    fuse_stream = torch.cuda.Stream(device=dev)
    ctx_f = rg.rgbid_create(0, fuse_stream)
    K = rg.rgbid_keyframe_init(ctx_f, fcam, kfW)
    params = rg.rgbid_default_params(
        levels=4, iters=[10, 10, 10, 10],
        weight=rg.RGBID_W_HUBER if args.weight == "huber" else rg.RGBID_W_STUDENT_T,
        warp=rg.RGBID_WARP_FULLRES if args.warp == "fullres" else rg.RGBID_WARP_PER_LEVEL,
        scale_warm=0 if args.scale_cold else 1)
    all_pyr = As + Bs
    all_I = IA + IB
    all_W = WA + WB
    torch.cuda.synchronize()

    tuned = None
    if args.tune_file:
        rg.rgbid_tune_load(ctx, args.tune_file)
        tuned = "loaded"
    elif not args.no_autotune:
        t0 = time.time()
        best = rg.rgbid_autotune(ctx, As, Bs, params, reps=3)
        tuned = [round(1e3 * b, 2) for b in best]
        log("autotuned launch shapes in %.1fs: best us/iteration per level %s" % (
            time.time() - t0, tuned))
        os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
        rg.rgbid_tune_save(ctx, os.path.join(ROOT, "gpurun_out", "tune_%s_%s.txt" % (
            args.storage, args.warp)))

    # launch shape per level (fused warp + reduction or not), as tuned
    tune_txt = os.path.join("/tmp", "rgbid_bench_tune_%d.txt" % os.getpid())
    rg.rgbid_tune_save(ctx, tune_txt)
    fused_level = {}
    for line in open(tune_txt):
        f = line.split()
        if len(f) == 6:    # one batch shape per bench run
            fused_level[int(f[0].split("_")[0][1:])] = f[1] == "1"
    os.remove(tune_txt)

    def step():
        rg.rgbid_keyframe_reset(ctx_f, K, kfW)
        rg.rgbid_fuse_batch(ctx_f, K, fW, fposes, 0.01)
        rg.rgbid_pyramid_update_batch(ctx, all_pyr, all_I, all_W)
        poses, stats = rg.rgbid_align_batch(ctx, As, Bs, params)
        return poses, stats

    # The timed form enqueues a whole step without waiting: the poses land in
    # device memory (rgbid_align_batch_async) and the host prepares the next
    # step while the GPU works, as a serving loop would.
    pose_buf = torch.empty(args.pairs * rg.POSE_BYTES, dtype=torch.uint8, device=dev)

    def step_async():
        rg.rgbid_keyframe_reset(ctx_f, K, kfW)
        rg.rgbid_fuse_batch(ctx_f, K, fW, fposes, 0.01)
        rg.rgbid_pyramid_update_batch(ctx, all_pyr, all_I, all_W)
        rg.rgbid_align_batch_async(ctx, As, Bs, params, pose_buf)

    for i in range(args.warmup):
        poses, stats = step()
        log("warmup step %d done" % i)
    torch.cuda.synchronize()
    # sanity: the batch converged near the ground truth
    errs = [np.linalg.norm(oracle.log_so3(R.T @ p.R)) for (R, t), p in zip(poses, pairs)]
    terrs = [np.linalg.norm(t - p.t) for (R, t), p in zip(poses, pairs)]
    bad = sum(s["status"] != 0 for s in stats)

    # the asynchronous step gives the same poses as the synchronous one
    step_async()
    torch.cuda.synchronize()
    apose = rg.unpack_poses(pose_buf, args.pairs)
    assert all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
               for a, b in zip(apose, poses)), "asynchronous step disagrees with the synchronous one"

    # per-step GPU time from stream events, the total from the host clock
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(args.steps):
        step_async()
        evs[i + 1].record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    per_step = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps))
    pick = lambda q: per_step[min(len(per_step) - 1, int(q * len(per_step)))]
    step_ms = {"median": round(pick(0.5), 4), "p10": round(pick(0.1), 4), "p90": round(pick(0.9), 4)}
    log("timed %d steps: %.3f ms/step (median %.3f, p10 %.3f, p90 %.3f)" % (
        args.steps, 1e3 * dt / args.steps, step_ms["median"], step_ms["p10"], step_ms["p90"]))

    # the same steps again with per-kernel HIP-event timing on
    rg.rgbid_set_profiling(ctx, True)
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    kt = rg.rgbid_kernel_times(ctx)
    rg.rgbid_set_profiling(ctx, False)

    fullres = args.warp == "fullres"
    rows = []
    for (lvl, kname), (ms, nl) in sorted(kt.items()):
        fused = fused_level.get(lvl, lvl == 0) if kname in ("warp", "reduce") else False
        b = algorithmic_bytes(lvl, kname, sizes, f16, fullres, fused)
        avg_us = 1e3 * ms / nl
        rows.append((ms, lvl, kname, avg_us, b))
        log("kernel %-6s level %d: %6d launches, avg %8.2f us, total %8.2f ms%s" % (
            kname, lvl, nl, avg_us, ms,
            "" if b is None else ", %.1f GB/s algorithmic" % (b / (avg_us * 1e-6) / 1e9)))
    dom = max((r for r in rows if r[4] is not None), key=lambda r: r[0])
    _, lvl, kname, avg_us, b = dom
    achieved = b / (avg_us * 1e-6) / 1e9
    fused = fused_level.get(lvl, lvl == 0)
    fl = algorithmic_flops(lvl, kname, sizes, fullres, fused)
    tflops = fl / (avg_us * 1e-6) / 1e12 if fl else 0.0
    cs = None if mixed else counter_summary()
    ent = (cs or {}).get("kernels", {}).get("%s_l%d" % (kname, lvl))
    traffic = ent["hbm_bytes_per_launch"] if ent else None
    hbm = {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4)}
    alu = {"achieved": round(tflops, 2), "peak": round(FP32_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
           "frac": round(tflops / FP32_PEAK_TFLOPS, 4), "flops_per_launch": fl,
           "note": "vector-ALU flops only, against the non-packed FP32 rate"}
    if kname == "reduce":
        mf = FLOPS_NE_MFMA * sum((w0 >> lvl) * (h0 >> lvl) for w0, h0 in sizes)
        mt = mf / (avg_us * 1e-6) / 1e12
        alu["mfma"] = {"achieved": round(mt, 2), "peak": MFMA_FP32_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(mt / MFMA_FP32_PEAK_TFLOPS, 4),
                       "flops_per_launch": mf}
    # the roof with the larger fraction binds
    top = alu if alu["frac"] > hbm["frac"] else hbm
    roofline = {"bound": "alu" if top is alu else "hbm", "kernel": "k_%s level %d" % (kname, lvl),
                "achieved": top["achieved"], "peak": top["peak"], "unit": top["unit"],
                "frac": top["frac"], "traffic": traffic, "bytes_per_launch": b,
                "avg_launch_us": round(avg_us, 2), "hbm": hbm, "alu": alu}
    if traffic:
        hbm["measured_GBs"] = round(traffic / (avg_us * 1e-6) / 1e9, 1)
    if ent and ent.get("trace_avg_us"):
        # the same kernel's average duration in the committed rocprofv3 kernel trace
        roofline["profile_avg_launch_us"] = ent["trace_avg_us"]
    if ent and ent.get("valu_insts_per_launch"):
        # executed VALU wave instructions against one per SIMD every 4 cycles
        alu["valu_issue_frac"] = round(ent["valu_insts_per_launch"] / (avg_us * 1e-6) /
                                       VALU_ISSUE_PEAK, 4)

    value = args.pairs * args.steps / dt
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "alignments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 4),
        "step_ms": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16-storage/f32" if f16 else "f32",
        "data": "synthetic",
        "config": {"workload": "%s (room+boxes generator, 10%% holes), "
                               "4-level %s warp, 10 Huber GN iterations per level, + fusion of "
                               "20 frames into one 640x480 keyframe" % (
                                   "24 x 320x240 + 32 x 640x480 + 8 x 1280x960 pairs" if mixed
                                   else "%d pairs of 640x480" % args.pairs, args.warp),
                   "batch": args.batch,
                   "pairs_per_step": args.pairs, "width": cam.w, "height": cam.h, "levels": 4,
                   "iters_per_level": 10, "warp": args.warp, "weight": args.weight,
                   "scale_fixed_point": "cold, 20 steps" if args.scale_cold else
                   "warm start, stop at 2^-16 sigma, at most 20 steps",
                   "storage": args.storage, "parallelism": "single GPU",
                   "autotuned_us_per_iteration": tuned},
        "roofline": roofline,
        "accuracy": {"max_rot_err_vs_truth_rad": float(max(errs)),
                     "max_trans_err_vs_truth_m": float(max(terrs)), "degenerate_pairs": bad},
    }
    if not args.no_c4 and not mixed:
        out["batched_c4"] = batched_c4(ctx, max(5, args.steps // 2), 2, args.storage)
    if not args.no_warmstart:
        out["warmstart"] = warmstart_compare(ctx, args.ws_pairs, args.steps)
    if not args.no_frontend:
        out["frontend"] = frontend_measure(ctx, pairs[0])
    if not args.no_cpu:
        log("timing the FP64 oracle on a bounded sample ...")
        op = oracle.Params(levels=4, iters=[10] * 4, weight=args.weight, warp=args.warp,
                           storage=args.storage, scale_warm=not args.scale_cold)
        out["cpu_baseline"] = cpu_baseline(pairs, fusion, op, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    for p in As + Bs:
        rg.rgbid_pyramid_free(p)
    rg.rgbid_keyframe_free(K)
    rg.rgbid_destroy(ctx_f)
    rg.rgbid_destroy(ctx)


if __name__ == "__main__":
    main()
