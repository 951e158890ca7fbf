"""Training and evaluation driver of the learned warm start.

Every arithmetic step runs in the library's kernels through the C ABI:
pyramids (rgbid_pyramid_update_batch), labels (rgbid_align_batch started at
the true pose: the method's own optimum next to the truth), the network input
(rgbid_warmstart_input), training (rgbid_warmstart_train_step: forward,
backward and AdamW kernels), and the evaluation (rgbid_warmstart_predict and
rgbid_align_batch).  This module only schedules batches.

    python -m paper_1807_08271_amd.warmstart --train-pairs 50000 --epochs 30 \
        --out paper_1807_08271_amd/weights/warmstart.npy --eval-pairs 1000
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import rgbid as rg

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart.npy")
LEVELS = 4


def label_params():
    """Gauss-Newton started at the true pose (labels)."""
    return rg.rgbid_default_params(levels=LEVELS, iters=[5, 5, 5, 5])


def eval_params(iters=(10, 10, 10, 10), eps=1e-6):
    return rg.rgbid_default_params(levels=LEVELS, iters=list(iters), stop_eps_t=eps, stop_eps_r=eps)


class PairStream:
    """Renders chunks of large-motion pairs into reusable pyramids."""

    def __init__(self, ctx, chunk=64, storage=rg.RGBID_F32):
        import torch
        import synth
        self.ctx, self.chunk = ctx, chunk
        self.cam = synth.camera_640()
        z = torch.zeros((self.cam.h, self.cam.w), dtype=torch.float32, device="cuda")
        self.As = [rg.rgbid_pyramid(ctx, self.cam, LEVELS, storage, z, z) for _ in range(chunk)]
        self.Bs = [rg.rgbid_pyramid(ctx, self.cam, LEVELS, storage, z, z) for _ in range(chunk)]
        self.x = torch.zeros((chunk, 4, 60, 80), dtype=torch.float32, device="cuda")

    def load(self, first, count, split):
        from synth import batch
        IA, WA, IB, WB, truth = batch.warm_pairs(first, count, split)
        m = len(truth)
        rg.rgbid_pyramid_update_batch(self.ctx, self.As[:m] + self.Bs[:m],
                                      [IA[i] for i in range(m)] + [IB[i] for i in range(m)],
                                      [WA[i] for i in range(m)] + [WB[i] for i in range(m)])
        return m, truth

    def close(self):
        for p in self.As + self.Bs:
            rg.rgbid_pyramid_free(p)


def _close(pose, ref, rot_tol, t_tol):
    R, t = pose
    Rr, tr = ref
    xi = rg.rgbid_pose_log(Rr.T @ R, np.zeros(3))
    return np.linalg.norm(xi[3:]) <= rot_tol and np.linalg.norm(t - tr) <= t_tol


def make_dataset(ctx, n_pairs, split="train", chunk=64, log=print):
    """Network inputs (device tensor n x 4 x 60 x 80), labels xi = log(T*) of
    the Gauss-Newton optimum reached from the true pose, and that optimum.
    Pairs whose labelling fails (degenerate, or more than 1 deg / 2 cm from the
    truth) are dropped."""
    import torch
    st = PairStream(ctx, chunk)
    xs, xis, refs = [], [], []
    t0 = time.time()
    done = 0
    while done < n_pairs:
        m, truth = st.load(done, min(chunk, n_pairs - done), split)
        poses, stats = rg.rgbid_align_batch(ctx, st.As[:m], st.Bs[:m], label_params(), inits=truth)
        rg.rgbid_warmstart_input(ctx, st.As[:m], st.Bs[:m], st.x)
        keep = [i for i in range(m) if stats[i]["status"] == 0 and
                _close(poses[i], truth[i], math.radians(1.0), 0.02)]
        if keep:
            idx = torch.as_tensor(keep, device="cuda")
            xs.append(st.x[:m].index_select(0, idx).clone())
            for i in keep:
                xis.append(rg.rgbid_pose_log(*poses[i]))
                refs.append(poses[i])
        done += m
        if log and (done // chunk) % 50 == 0:
            log("dataset %s: %d / %d pairs (%.0f s)" % (split, done, n_pairs, time.time() - t0))
    st.close()
    return torch.cat(xs), np.array(xis), refs


def train(ctx, net, x, xi, epochs=30, batch=256, lr=1e-3, wd=1e-4, seed=0, log=print):
    """AdamW with a cosine learning-rate schedule over shuffled mini-batches."""
    import torch
    n = x.shape[0]
    rng = np.random.default_rng(seed)
    steps = epochs * (n // batch)
    step = 0
    xb = torch.empty((batch, 4, 60, 80), dtype=torch.float32, device="cuda")
    hist = []
    t0 = time.time()
    for ep in range(epochs):
        perm = rng.permutation(n)
        ep_loss = []
        for b in range(n // batch):
            idx = perm[b * batch:(b + 1) * batch]
            torch.index_select(x, 0, torch.as_tensor(idx, device="cuda"), out=xb)
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * step / max(1, steps)))
            want = b == n // batch - 1
            l = rg.rgbid_warmstart_train_step(ctx, net, xb, xi[idx], cur, wd, want_loss=want)
            if want:
                ep_loss.append(l)
            step += 1
        hist.append(float(np.mean(ep_loss)) if ep_loss else float("nan"))
        if log:
            log("epoch %d: loss %.4f (%.0f s)" % (ep, hist[-1], time.time() - t0))
    return hist


def evaluate(ctx, net, n_pairs=1000, chunk=64, schedules=None, log=print):
    """Plain Gauss-Newton from the identity against network + Gauss-Newton, with
    early stop at 1e-6, on held-out large-motion pairs.  Success: the final
    pose within 1e-5 rad / 1e-5 m of the optimum reached from the true pose."""
    import torch
    schedules = schedules or {"plain": (False, (10, 10, 10, 10)),
                              "warm": (True, (10, 10, 10, 10)),
                              "warm_short": (True, (0, 0, 10, 10))}
    st = PairStream(ctx, chunk)
    res = {k: {"ok": 0, "iters": 0, "time": 0.0} for k in schedules}
    total = 0
    done = 0
    while done < n_pairs:
        m, truth = st.load(done, min(chunk, n_pairs - done), "eval")
        ref, rstats = rg.rgbid_align_batch(ctx, st.As[:m], st.Bs[:m], label_params(), inits=truth)
        for name, (warm, iters) in schedules.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if warm:
                # network and alignment in one call, the initial poses formed on the device
                poses, stats = rg.rgbid_align_batch_warm(ctx, net, st.As[:m], st.Bs[:m],
                                                         eval_params(iters))
            else:
                poses, stats = rg.rgbid_align_batch(ctx, st.As[:m], st.Bs[:m], eval_params(iters))
            torch.cuda.synchronize()
            res[name]["time"] += time.perf_counter() - t0
            for i in range(m):
                if rstats[i]["status"] != 0:
                    continue
                res[name]["ok"] += int(stats[i]["status"] == 0 and _close(poses[i], ref[i], 1e-5, 1e-5))
                res[name]["iters"] += sum(stats[i]["iters_done"])
        total += sum(s["status"] == 0 for s in rstats)
        done += m
    st.close()
    out = {}
    for name, r in res.items():
        out[name] = {"success_rate": r["ok"] / max(1, total), "mean_gn_iters": r["iters"] / max(1, total),
                     "alignments_per_s": done / r["time"], "pairs": total}
        if log:
            log("%-10s success %.3f  mean GN iterations %.1f  %.0f alignments/s" % (
                name, out[name]["success_rate"], out[name]["mean_gn_iters"],
                out[name]["alignments_per_s"]))
    return out


def init_params(seed=0):
    """He-normal convolution weights (std sqrt(2 / fan_in)), FC weights with std
    sqrt(1 / fan_in), zero biases, drawn from a seeded generator."""
    rng = np.random.default_rng(np.random.SeedSequence([1807, 77, seed]))
    ch = [4, 32, 64, 128, 128]
    parts = []
    for ci, co in zip(ch[:-1], ch[1:]):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / (ci * 9)), size=co * ci * 9))
        parts.append(np.zeros(co))
    parts.append(rng.normal(0.0, math.sqrt(1.0 / 128), size=6 * 128))
    parts.append(np.zeros(6))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == rg.rgbid_warmstart_param_count()
    return w


def load_weights(path=DEFAULT_WEIGHTS):
    return np.load(path, allow_pickle=False).astype(np.float32)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-pairs", type=int, default=50000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--wd", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--eval-pairs", type=int, default=1000)
    ap.add_argument("--eval-only", action="store_true")
    args = ap.parse_args(argv)
    import torch
    log = lambda *a: print("[warmstart]", *a, flush=True)
    ctx = rg.rgbid_create(0)
    if args.eval_only:
        net = rg.rgbid_warmstart_create(ctx, load_weights(args.out))
    else:
        t0 = time.time()
        x, xi, _ = make_dataset(ctx, args.train_pairs, "train", log=log)
        log("dataset: %d labelled pairs in %.0f s" % (x.shape[0], time.time() - t0))
        net = rg.rgbid_warmstart_create(ctx, init_params(args.seed))
        hist = train(ctx, net, x, xi, args.epochs, args.batch, args.lr, args.wd, args.seed, log=log)
        w = rg.rgbid_warmstart_get_params(ctx, net)
        os.makedirs(os.path.dirname(args.out), exist_ok=True)
        np.save(args.out, w)
        with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
            json.dump({"train_pairs": int(x.shape[0]), "epochs": args.epochs, "batch": args.batch,
                       "lr": args.lr, "wd": args.wd, "seed": args.seed, "loss_per_epoch": hist},
                      f, indent=1)
        del x
        torch.cuda.empty_cache()
    out = evaluate(ctx, net, args.eval_pairs, log=log)
    print(json.dumps(out))
    # the evaluation goes into the run record beside the weights
    rec_path = os.path.splitext(args.out)[0] + ".json"
    rec = json.load(open(rec_path)) if os.path.exists(rec_path) else {}
    rec["eval_%d_heldout" % args.eval_pairs] = out
    with open(rec_path, "w") as f:
        json.dump(rec, f, indent=1)
    rg.rgbid_warmstart_free(net)
    rg.rgbid_destroy(ctx)
    return 0


if __name__ == "__main__":
    sys.exit(main())
