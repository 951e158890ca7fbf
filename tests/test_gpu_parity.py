"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

Tolerances (the targets of this build):
  normal equations  |dH_ij| <= 1e-4 sqrt(H_ii H_jj), |dg_i| <= 1e-4 sqrt(H_ii cost),
                    valid counts within 20 threshold flips;
  poses             <= 1e-5 rad and <= 1e-5 m after the same schedule;
  fused W           <= 1e-5 relative where both sides take the same
                    covisibility decision.
"""
import numpy as np
import pytest

import oracle
import synth
from _parity import check_normal_equations, rot_err, upload

pytestmark = pytest.mark.gpu


def _rg():
    from paper_1807_08271_amd import rgbid
    return rgbid


def _pyr(ctx, cam, levels, frame, storage=0):
    rg = _rg()
    I, W = upload(frame.I, frame.W)
    return rg.rgbid_pyramid(ctx, cam, levels, storage, I, W)


def _params(levels, iters, weight="huber", warp="fullres", **kw):
    rg = _rg()
    return rg.rgbid_default_params(
        levels=levels, iters=iters,
        weight=rg.RGBID_W_HUBER if weight == "huber" else rg.RGBID_W_STUDENT_T,
        warp=rg.RGBID_WARP_FULLRES if warp == "fullres" else rg.RGBID_WARP_PER_LEVEL, **kw)


def _oparams(levels, iters, weight="huber", warp="fullres", storage="f32", **kw):
    return oracle.Params(levels=levels, iters=iters, weight=weight, warp=warp, storage=storage, **kw)


# ----------------------------------------------------------------- pyramid


@pytest.mark.parametrize("storage", [0, 1])
def test_pyramid_matches_oracle(ctx, c2_pairs, storage):
    rg = _rg()
    p = c2_pairs[0]
    I0, W0 = p.A.I, p.A.W
    if storage == 1:
        I0, W0 = synth.to_fp16_grid(I0), synth.to_fp16_grid(W0)
    pyr = _pyr(ctx, p.cam, 4, p.A, storage)
    ref = oracle.pyramid(p.cam, 4, I0, W0, storage="f16" if storage else "f32")
    for l in range(4):
        Ig, Wg = rg.rgbid_pyramid_read(ctx, pyr, l)
        Ig, Wg = Ig.cpu().numpy(), Wg.cpu().numpy()
        Ir, Wr = ref[l]
        assert Ig.shape == Ir.shape
        np.testing.assert_array_equal(Wg > 0, Wr > 0)
        if storage == 0:
            # A level is the mean of up to four non-negative FP32 values of
            # the level below: the sum rounds at most three times (each
            # <= u = 2^-24 of the partial sum, so <= 3u of the total) and the
            # division by 4 is exact, by 2 exact, by 3 rounds once after two
            # additions: <= 3u per level.  The inputs of level l carry level
            # l-1's relative error, which a mean of positives keeps, so level
            # l is within 3 l u of the FP64 recursion (level 0 is the input).
            rtol = 3 * l * 2.0 ** -24
            np.testing.assert_allclose(Ig, Ir, rtol=rtol, atol=0)
            np.testing.assert_allclose(Wg, Wr, rtol=rtol, atol=0)
        else:
            # FP16 levels: identical rounding except rare double-rounding ties
            assert np.mean(Ig != Ir) < 1e-3 and np.mean(Wg != Wr) < 1e-3
            np.testing.assert_allclose(Wg, Wr, rtol=1e-3)
    rg.rgbid_pyramid_free(pyr)


def test_pyramid_row_pitch_and_alignment(ctx, c2_pairs):
    # When the rows allow it (width and pitch multiples of 4, 16-byte aligned
    # rows, even height) levels 0 and 1 and the level-0 flags come from one
    # pass over 2x2 blocks; otherwise level 0 moves one pixel per thread and
    # levels and flags follow in passes of their own.  A contiguous image, the
    # same image inside wider rows, and inside rows whose start is 4 bytes off
    # 16-byte alignment give identical pyramids (all planes: I and W read
    # back, W_A and the flags through the normal equations at every level).
    rg = _rg()
    import torch
    p = c2_pairs[0]
    I0, W0 = upload(p.A.I, p.A.W)
    h, w = I0.shape
    wide = lambda t, extra, off: torch.zeros((h, w + extra), device="cuda").copy_(
        torch.nn.functional.pad(t, (off, extra - off)))[:, off:off + w]
    views = [(I0, W0), (wide(I0, 8, 0), wide(W0, 8, 0)), (wide(I0, 5, 1), wide(W0, 5, 1))]
    assert views[1][0].stride(0) == w + 8 and views[2][0].data_ptr() % 16 == 4
    prm = _params(4, [1] * 4)
    R, t = oracle.exp_so3(oracle.log_so3(p.R) * 0.5), p.t * 0.5
    for storage in (0, 1):
        pyrs = [rg.rgbid_pyramid(ctx, p.cam, 4, storage, I, W) for I, W in views]
        Bs = _pyr(ctx, p.cam, 4, p.B, storage)
        for level in range(4):
            ref = rg.rgbid_pyramid_read(ctx, pyrs[0], level)
            for P in pyrs[1:]:
                got = rg.rgbid_pyramid_read(ctx, P, level)
                assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), (storage, level)
        for level in range(4):
            ne = [rg.rgbid_normal_equations(ctx, P, Bs, level, (R, t), prm) for P in pyrs]
            for g in ne[1:]:
                np.testing.assert_array_equal(g["H"], ne[0]["H"])
                np.testing.assert_array_equal(g["g"], ne[0]["g"])
                assert g["n_valid_I"] == ne[0]["n_valid_I"], (storage, level)
                assert g["n_valid_W"] == ne[0]["n_valid_W"], (storage, level)
        for P in pyrs + [Bs]:
            rg.rgbid_pyramid_free(P)


# ----------------------------------------------------------------- normal equations


@pytest.mark.parametrize("weight", ["huber", "student_t"])
@pytest.mark.parametrize("warp", ["fullres", "per_level"])
def test_normal_equations_c2_all_levels(ctx, c2_pairs, weight, warp):
    rg = _rg()
    p = c2_pairs[1]
    A = _pyr(ctx, p.cam, 4, p.A)
    B = _pyr(ctx, p.cam, 4, p.B)
    # a pose between identity and the truth
    th = oracle.log_so3(p.R) * 0.6
    R = oracle.exp_so3(th)
    t = p.t * 0.6
    gp = _params(4, [1] * 4, weight, warp)
    op = _oparams(4, [1] * 4, weight, warp)
    for level in range(4):
        g = rg.rgbid_normal_equations(ctx, A, B, level, (R, t), gp)
        r = oracle.normal_equations_at(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, level, R, t, op)
        check_normal_equations(g, r, what="c2 %s %s level %d" % (weight, warp, level))
        assert g["sigma_I"] == pytest.approx(r["sigma_I"], rel=1e-4)
        assert g["sigma_W"] == pytest.approx(r["sigma_W"], rel=1e-4)
        if weight == "student_t":
            assert g["nu_I"] == pytest.approx(r["nu_I"], abs=1e-3)
            assert g["nu_W"] == pytest.approx(r["nu_W"], abs=1e-3)
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


# (crop, sample_max) giving level-0 samples of 4800, 8560, 12288, 19200 and
# 22400 entries: every length the scale kernel is built for (5, 10, 15, 19
# and 24 entries per thread), with a partly filled last slot after the
# undefined residuals are dropped.
_SAMPLE_CASES = [((480, 640), 5000), ((480, 640), 9000), ((480, 640), 15000),
                 ((480, 640), 19200), ((420, 480), 24576)]


@pytest.mark.parametrize("weight", ["huber", "student_t"])
@pytest.mark.parametrize("case", range(len(_SAMPLE_CASES)))
def test_scale_every_sample_length(ctx, c2_pairs, weight, case):
    rg = _rg()
    (h, w), smax = _SAMPLE_CASES[case]
    p = c2_pairs[0]
    crop = lambda a: np.ascontiguousarray(a[:h, :w])
    IA, WA, IB, WB = crop(p.A.I), crop(p.A.W), crop(p.B.I), crop(p.B.W)
    cam = (w, h) + p.cam.as_tuple()[2:]
    A = rg.rgbid_pyramid(ctx, cam, 1, 0, *upload(IA, WA))
    B = rg.rgbid_pyramid(ctx, cam, 1, 0, *upload(IB, WB))
    th = oracle.log_so3(p.R) * 0.6
    R, t = oracle.exp_so3(th), p.t * 0.6
    g = rg.rgbid_normal_equations(ctx, A, B, 0, (R, t), _params(1, [1], weight, sample_max=smax))
    r = oracle.normal_equations_at(cam, IA, WA, IB, WB, 0, R, t,
                                   _oparams(1, [1], weight, sample_max=smax))
    what = "%s %dx%d sample_max %d" % (weight, w, h, smax)
    check_normal_equations(g, r, what=what)
    assert g["sigma_I"] == pytest.approx(r["sigma_I"], rel=1e-4), what
    assert g["sigma_W"] == pytest.approx(r["sigma_W"], rel=1e-4), what
    if weight == "student_t":
        assert g["nu_I"] == pytest.approx(r["nu_I"], abs=1e-3), what
        assert g["nu_W"] == pytest.approx(r["nu_W"], abs=1e-3), what
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


def test_graph_cache_follows_sample_max(ctx, c2_pairs):
    # Same sizes and schedule, different sample_max, one context: every call
    # must use launch tables and a scale kernel for its own sample length
    # (a captured graph holds both).
    rg = _rg()
    p = c2_pairs[1]
    A = _pyr(ctx, p.cam, 2, p.A)
    B = _pyr(ctx, p.cam, 2, p.B)
    R, t = oracle.exp_so3(oracle.log_so3(p.R) * 0.5), p.t * 0.5
    for smax in (19200, 9000, 5000, 19200, 9000):
        g = rg.rgbid_normal_equations(ctx, A, B, 0, (R, t), _params(2, [1, 1], sample_max=smax))
        r = oracle.normal_equations_at(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, 0, R, t,
                                       _oparams(2, [1, 1], sample_max=smax))
        check_normal_equations(g, r, what="sample_max %d" % smax)
        assert g["sigma_I"] == pytest.approx(r["sigma_I"], rel=1e-4)
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


def test_normal_equations_identity_zero_gradient(ctx, c1_pairs):
    # B = A at the identity: residuals vanish, so g ~ 0 and the step is ~0.
    rg = _rg()
    p = c1_pairs[0]
    A = _pyr(ctx, p.cam, 1, p.A)
    g = rg.rgbid_normal_equations(ctx, A, A, 0, (np.eye(3), np.zeros(3)), _params(1, [1]))
    xi = np.linalg.solve(g["H"], -g["g"])
    assert np.abs(xi).max() < 1e-6
    assert g["n_valid_I"] > 0.9 * 158 * 118
    rg.rgbid_pyramid_free(A)


# ----------------------------------------------------------------- alignment


@pytest.mark.parametrize("i", [0, 1, 2])
def test_align_c1_matches_oracle(ctx, c1_pairs, i):
    rg = _rg()
    p = c1_pairs[i]
    A = _pyr(ctx, p.cam, 1, p.A)
    B = _pyr(ctx, p.cam, 1, p.B)
    R, t, st, rc = rg.rgbid_align(ctx, A, B, _params(1, [10]))
    Ro, to, sto = oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, _oparams(1, [10]))
    assert rc == 0 and sto["status"] == 0
    assert st["iters_done"][0] == 10
    assert rot_err(R, Ro) <= 1e-5, rot_err(R, Ro)
    assert np.linalg.norm(t - to) <= 1e-5, np.linalg.norm(t - to)
    # and the estimate is near the truth (noise-limited)
    assert rot_err(R, p.R) < 2e-3 and np.linalg.norm(t - p.t) < 5e-3
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


@pytest.mark.parametrize("warp", ["fullres", "per_level"])
@pytest.mark.parametrize("weight", ["huber", "student_t"])
def test_align_c2_matches_oracle(ctx, c2_pairs, warp, weight):
    rg = _rg()
    p = c2_pairs[0]
    A = _pyr(ctx, p.cam, 4, p.A)
    B = _pyr(ctx, p.cam, 4, p.B)
    R, t, st, rc = rg.rgbid_align(ctx, A, B, _params(4, [10] * 4, weight, warp))
    Ro, to, sto = oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W,
                               _oparams(4, [10] * 4, weight, warp))
    assert rc == 0 and sto["status"] == 0
    assert st["iters_done"][:4] == [10, 10, 10, 10]
    assert rot_err(R, Ro) <= 1e-5, rot_err(R, Ro)
    assert np.linalg.norm(t - to) <= 1e-5, np.linalg.norm(t - to)
    assert rot_err(R, p.R) < 1e-3 and np.linalg.norm(t - p.t) < 2e-3
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


@pytest.mark.parametrize("weight", ["huber", "student_t"])
def test_align_scale_schedules_match_oracle(ctx, c2_pairs, weight):
    # Both schedules of the mu, sigma fixed point (sec. 6.3): warm-started
    # with the convergence stop (default) and cold with all scale_iters
    # steps, each against the oracle run the same way.  The two schedules end
    # at the same fixed point to about 1e-6 of sigma, so after 10 iterations
    # per level their poses agree within the pose bar as well.
    rg = _rg()
    p = c2_pairs[1]
    A = _pyr(ctx, p.cam, 4, p.A)
    B = _pyr(ctx, p.cam, 4, p.B)
    got = {}
    for warm in (1, 0):
        R, t, st, rc = rg.rgbid_align(ctx, A, B, _params(4, [10] * 4, weight, scale_warm=warm))
        Ro, to, sto = oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W,
                                   _oparams(4, [10] * 4, weight, scale_warm=bool(warm)))
        what = "%s scale_warm %d" % (weight, warm)
        assert rc == 0 and sto["status"] == 0, what
        assert rot_err(R, Ro) <= 1e-5, (what, rot_err(R, Ro))
        assert np.linalg.norm(t - to) <= 1e-5, (what, np.linalg.norm(t - to))
        for k in ("sigma_I", "sigma_W"):
            assert st[k] == pytest.approx(sto[k], rel=1e-4), (what, k)
        got[warm] = (R, t)
    assert rot_err(got[0][0], got[1][0]) <= 1e-5
    assert np.linalg.norm(got[0][1] - got[1][1]) <= 1e-5
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


def test_align_fp16_storage_matches_oracle_on_rounded_inputs(ctx, c2_pairs):
    rg = _rg()
    p = c2_pairs[1]
    A = _pyr(ctx, p.cam, 4, p.A, storage=1)
    B = _pyr(ctx, p.cam, 4, p.B, storage=1)
    R, t, st, rc = rg.rgbid_align(ctx, A, B, _params(4, [10] * 4))
    h = synth.to_fp16_grid
    Ro, to, _ = oracle.align(p.cam, h(p.A.I), h(p.A.W), h(p.B.I), h(p.B.W),
                             _oparams(4, [10] * 4, storage="f16"))
    assert rc == 0
    assert rot_err(R, Ro) <= 1e-5 and np.linalg.norm(t - to) <= 1e-5
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


def test_align_initial_guess(ctx, c1_pairs):
    rg = _rg()
    p = c1_pairs[1]
    A = _pyr(ctx, p.cam, 1, p.A)
    B = _pyr(ctx, p.cam, 1, p.B)
    R, t, st, rc = rg.rgbid_align(ctx, A, B, _params(1, [3]), init=(p.R, p.t))
    Ro, to, _ = oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, _oparams(1, [3]), R0=p.R, t0=p.t)
    assert rot_err(R, Ro) <= 1e-5 and np.linalg.norm(t - to) <= 1e-5
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


def test_align_batch_mixed_sizes_equals_single(ctx, c1_pairs, c2_pairs):
    rg = _rg()
    pairs = [c2_pairs[0], c1_pairs[0], c2_pairs[1], c1_pairs[2]]
    As = [_pyr(ctx, p.cam, 3, p.A) for p in pairs]
    Bs = [_pyr(ctx, p.cam, 3, p.B) for p in pairs]
    prm = _params(3, [5, 5, 5])
    poses, stats = rg.rgbid_align_batch(ctx, As, Bs, prm)
    for i, p in enumerate(pairs):
        R1, t1, _, _ = rg.rgbid_align(ctx, As[i], Bs[i], prm)
        np.testing.assert_array_equal(poses[i][0], R1)     # deterministic reduction order
        np.testing.assert_array_equal(poses[i][1], t1)
        Ro, to, _ = oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, _oparams(3, [5, 5, 5]))
        assert rot_err(poses[i][0], Ro) <= 1e-5 and np.linalg.norm(poses[i][1] - to) <= 1e-5
        assert stats[i]["status"] == 0
    for x in As + Bs:
        rg.rgbid_pyramid_free(x)


def test_align_is_deterministic(ctx, c2_pairs):
    rg = _rg()
    p = c2_pairs[0]
    A = _pyr(ctx, p.cam, 4, p.A)
    B = _pyr(ctx, p.cam, 4, p.B)
    prm = _params(4, [10] * 4)
    a = rg.rgbid_align(ctx, A, B, prm)
    b = rg.rgbid_align(ctx, A, B, prm)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2]["H"], b[2]["H"])
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


def test_bench_workload_sampled_against_oracle(ctx):
    # The timed step's alignment as the bench runs it: 64 pairs of 640x480
    # (room + boxes, 10% holes), 4 levels x 10 Huber iterations, FULLRES, FP32,
    # autotuned launch shapes, the default launch chains, one batch.  Four
    # pairs spread over the batch (0, 21, 42, 63: every default launch chain
    # holds at least one) against the oracle.
    rg = _rg()
    pairs = [synth.pair_c2(i, ss=2, device="cuda") for i in range(64)]
    As = [_pyr(ctx, p.cam, 4, p.A) for p in pairs]
    Bs = [_pyr(ctx, p.cam, 4, p.B) for p in pairs]
    prm = _params(4, [10] * 4)
    rg.rgbid_autotune(ctx, As, Bs, prm, reps=1)
    got, stats = rg.rgbid_align_batch(ctx, As, Bs, prm)
    for i in (0, 21, 42, 63):
        p = pairs[i]
        Ro, to, so = oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, _oparams(4, [10] * 4))
        assert stats[i]["status"] == 0 and so["status"] == 0, i
        assert rot_err(got[i][0], Ro) <= 1e-5 and np.linalg.norm(got[i][1] - to) <= 1e-5, i
    for P in As + Bs:
        rg.rgbid_pyramid_free(P)


def test_mixed_batch_c4_sampled_against_oracle(ctx):
    # The batched form at its own shapes: 24 x 320x240 + 32 x 640x480 +
    # 8 x 1280x960 pairs (room + boxes, 10% holes) aligned in one batch, 4
    # levels x 10 Huber iterations, FULLRES, FP32, autotuned launch shapes,
    # the default launch chains.  Two pairs of every size (the first and the
    # last of each group, so sample strides 1..8 and the largest chunk tables
    # are all exercised) against the oracle.
    rg = _rg()
    pairs = synth.batch_c4(ss=2, device="cuda")
    assert [p.cam.w for p in pairs] == [320] * 24 + [640] * 32 + [1280] * 8
    As = [_pyr(ctx, p.cam, 4, p.A) for p in pairs]
    Bs = [_pyr(ctx, p.cam, 4, p.B) for p in pairs]
    prm = _params(4, [10] * 4)
    rg.rgbid_autotune(ctx, As, Bs, prm, reps=1)
    got, stats = rg.rgbid_align_batch(ctx, As, Bs, prm)
    for i in (0, 23, 24, 55, 56, 63):
        p = pairs[i]
        print("c4 pair %d (%dx%d) against the oracle" % (i, p.cam.w, p.cam.h), flush=True)
        Ro, to, so = oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, _oparams(4, [10] * 4))
        assert stats[i]["status"] == 0 and so["status"] == 0, i
        assert rot_err(got[i][0], Ro) <= 1e-5 and np.linalg.norm(got[i][1] - to) <= 1e-5, i
    for P in As + Bs:
        rg.rgbid_pyramid_free(P)


def test_align_batch_async_matches_sync(ctx, c2_pairs):
    # the asynchronous batch writes the same poses and statistics to device
    # memory, bit for bit, including a degenerate pair and two calls in a row
    rg = _rg()
    import torch
    pairs = list(c2_pairs)
    As = [_pyr(ctx, p.cam, 4, p.A) for p in pairs]
    Bs = [_pyr(ctx, p.cam, 4, p.B) for p in pairs]
    prm = _params(4, [10] * 4)
    poses, stats = rg.rgbid_align_batch(ctx, As, Bs, prm)
    n = len(As)
    out = torch.zeros(n * rg.POSE_BYTES, dtype=torch.uint8, device="cuda")
    st = torch.zeros(n * rg.STATS_BYTES, dtype=torch.uint8, device="cuda")
    for _ in range(2):
        rg.rgbid_align_batch_async(ctx, As, Bs, prm, out, st)
    torch.cuda.synchronize()
    ap = rg.unpack_poses(out, n)
    ast = rg.unpack_stats(st, n)
    for i in range(n):
        np.testing.assert_array_equal(ap[i][0], poses[i][0])
        np.testing.assert_array_equal(ap[i][1], poses[i][1])
        for key in ("H", "g", "cost", "mu_I", "sigma_I", "mu_W", "sigma_W", "n_valid_I",
                    "n_valid_W", "iters_done", "status"):
            np.testing.assert_array_equal(np.asarray(ast[i][key]), np.asarray(stats[i][key]), key)
    with pytest.raises(ValueError):
        rg.rgbid_align_batch_async(ctx, As, Bs, prm, out[:8])
    for P in As + Bs:
        rg.rgbid_pyramid_free(P)


# ----------------------------------------------------------------- edge cases


def test_degenerate_all_holes(ctx):
    rg = _rg()
    import torch
    cam = (64, 48, 60.0, 60.0, 31.5, 23.5)
    I = torch.rand(48, 64, device="cuda") * 255
    W = torch.zeros(48, 64, device="cuda")
    A = rg.rgbid_pyramid(ctx, cam, 2, 0, I, W)
    R, t, st, rc = rg.rgbid_align(ctx, A, A, _params(2, [3, 3]))
    assert rc == rg.RGBID_E_DEGENERATE and st["status"] == rg.RGBID_E_DEGENERATE
    np.testing.assert_array_equal(R, np.eye(3))
    np.testing.assert_array_equal(t, np.zeros(3))
    rg.rgbid_pyramid_free(A)


def test_degenerate_constant_image(ctx):
    # Constant intensity and inverse depth (sec. 6.2): no intensity gradient
    # and a plane without structure leave the 6x6 normal equations singular;
    # both sides stop on the first iteration, keep the initial pose and
    # report the degenerate system.
    rg = _rg()
    import torch
    cam = (96, 72, 80.0, 80.0, 47.5, 35.5)
    I = torch.full((72, 96), 128.0, device="cuda")
    W = torch.full((72, 96), 0.5, device="cuda")
    A = rg.rgbid_pyramid(ctx, cam, 2, 0, I, W)
    R, t, st, rc = rg.rgbid_align(ctx, A, A, _params(2, [3, 3]))
    Ro, to, so = oracle.align(cam, I.cpu().numpy(), W.cpu().numpy(), I.cpu().numpy(),
                              W.cpu().numpy(), _oparams(2, [3, 3]))
    assert rc == rg.RGBID_E_DEGENERATE and st["status"] == rg.RGBID_E_DEGENERATE
    assert so["status"] == rg.RGBID_E_DEGENERATE
    np.testing.assert_array_equal(R, np.eye(3))
    np.testing.assert_array_equal(t, np.zeros(3))
    np.testing.assert_array_equal(Ro, np.eye(3))
    np.testing.assert_array_equal(to, np.zeros(3))
    rg.rgbid_pyramid_free(A)


def test_degenerate_out_of_view_pose(ctx, c1_pairs):
    # An initial pose that transfers every pixel of A out of B's image (or
    # behind the camera): no residual is defined, so the first linearisation
    # has fewer than 6 valid residuals; both sides stop, keep the initial
    # pose and report the degenerate system.
    rg = _rg()
    p = c1_pairs[0]
    A = _pyr(ctx, p.cam, 2, p.A)
    B = _pyr(ctx, p.cam, 2, p.B)
    R0, t0 = np.eye(3), np.array([40.0, 0.0, 0.0])
    R, t, st, rc = rg.rgbid_align(ctx, A, B, _params(2, [3, 3]), init=(R0, t0))
    Ro, to, so = oracle.align(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, _oparams(2, [3, 3]),
                              R0=R0, t0=t0)
    assert rc == rg.RGBID_E_DEGENERATE and st["status"] == rg.RGBID_E_DEGENERATE
    assert so["status"] == rg.RGBID_E_DEGENERATE
    assert st["n_valid_I"] == 0 and st["n_valid_W"] == 0
    np.testing.assert_array_equal(R, R0)
    np.testing.assert_array_equal(t, t0)
    np.testing.assert_array_equal(Ro, R0)
    np.testing.assert_array_equal(to, t0)
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


def test_ragged_size_and_small_sample(ctx):
    # 157x113: odd sizes (floor at every level), tiles with a ragged tail, and a
    # sample of at most 1000 pixels (stride 5 at level 0).
    rg = _rg()
    p = synth.pair_c1(7)
    I = np.ascontiguousarray(p.A.I[:113, :157])
    W = np.ascontiguousarray(p.A.W[:113, :157])
    Ib = np.ascontiguousarray(p.B.I[:113, :157])
    Wb = np.ascontiguousarray(p.B.W[:113, :157])
    cam = (157, 113, 131.25, 131.25, 79.5, 59.5)
    A = rg.rgbid_pyramid(ctx, cam, 3, 0, *upload(I, W))
    B = rg.rgbid_pyramid(ctx, cam, 3, 0, *upload(Ib, Wb))
    prm = _params(3, [4, 4, 4], sample_max=1000)
    R, t, st, rc = rg.rgbid_align(ctx, A, B, prm)
    Ro, to, sto = oracle.align(cam, I, W, Ib, Wb, _oparams(3, [4, 4, 4], sample_max=1000))
    assert rc == 0 and sto["status"] == 0
    assert rot_err(R, Ro) <= 1e-5 and np.linalg.norm(t - to) <= 1e-5
    for level in range(3):
        g = rg.rgbid_normal_equations(ctx, A, B, level, (Ro, to), prm)
        r = oracle.normal_equations_at(cam, I, W, Ib, Wb, level, Ro, to,
                                       _oparams(3, [1] * 3, sample_max=1000))
        check_normal_equations(g, r, what="ragged level %d" % level)
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("size", [(17, 5), (31, 11), (48, 12), (65, 9)])
def test_level0_block_edges_match_oracle(ctx, storage, size):
    # Level 0 is reduced in 16 x 4 pixel blocks with the neighbours from a
    # per-wave tile (block plus a halo row / column on each side) and the
    # validity flags formed in the kernel.  Widths and heights below, at and
    # just past a block multiple (partial blocks on the right and at the
    # bottom, halos clamped to the plane's guards), in FP32 and FP16 storage,
    # against the oracle's normal equations at a pose short of the truth.
    rg = _rg()
    w, h = size
    p = synth.pair_c1(3)
    crop = lambda a: np.ascontiguousarray(a[:h, :w])
    I, W, Ib, Wb = crop(p.A.I), crop(p.A.W), crop(p.B.I), crop(p.B.W)
    if storage == 1:
        I, W, Ib, Wb = (synth.to_fp16_grid(a) for a in (I, W, Ib, Wb))
    cam = (w, h, 131.25, 131.25, 79.5, 59.5)
    print("level-0 block edges %dx%d storage %d" % (w, h, storage), flush=True)
    A = rg.rgbid_pyramid(ctx, cam, 1, storage, *upload(I, W))
    B = rg.rgbid_pyramid(ctx, cam, 1, storage, *upload(Ib, Wb))
    R, t = oracle.exp_so3(oracle.log_so3(p.R) * 0.6), p.t * 0.6
    g = rg.rgbid_normal_equations(ctx, A, B, 0, (R, t), _params(1, [1]))
    r = oracle.normal_equations_at(cam, I, W, Ib, Wb, 0, R, t,
                                   _oparams(1, [1], storage="f16" if storage else "f32"))
    assert r["n_valid_I"] > 0
    check_normal_equations(g, r, what="%dx%d storage %d" % (w, h, storage))
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("axis,sign", [(1, 1), (1, -1), (0, 1), (0, -1)])
def test_edge_taps_match_oracle(ctx, storage, axis, sign):
    # A rotation about the y (x) axis that moves the first interior column
    # (row) of the middle line to -0.25, or the last interior one to w - 0.75
    # (h - 0.75): those pixels and their neighbours along the line sample B
    # where the bilinear taps are clamped to the image.  The kernels load the second
    # tap unclamped and give it weight 0 there; the oracle clamps the taps.
    rg = _rg()
    p = synth.pair_c1(5)
    I, W, Ib, Wb = p.A.I, p.A.W, p.B.I, p.B.W
    if storage == 1:
        I, W, Ib, Wb = (synth.to_fp16_grid(a) for a in (I, W, Ib, Wb))
    cam = p.cam
    K = np.array([[cam.fx, 0.0, cam.cx], [0.0, cam.fy, cam.cy], [0.0, 0.0, 1.0]])
    n = cam.h if axis == 0 else cam.w
    # the first (last) interior pixel of the middle line to n[-0.25] (n - 0.75)
    src = 1.0 if sign > 0 else n - 2.0
    dst = -0.25 if sign > 0 else n - 0.75
    mid = (cam.cx, cam.cy)

    def proj(a):
        th = np.zeros(3)
        th[axis] = a
        x = np.array([src, mid[1], 1.0]) if axis == 1 else np.array([mid[0], src, 1.0])
        q = K @ oracle.exp_so3(th).T @ np.linalg.solve(K, x)
        return q[1 - axis] / q[2] if axis == 0 else q[0] / q[2]

    lo, hi = -0.05, 0.05   # radians; the projection is monotone in the angle
    flo = proj(lo) - dst
    for _ in range(80):
        m = 0.5 * (lo + hi)
        if (proj(m) - dst) * flo > 0:
            lo, flo = m, proj(m) - dst
        else:
            hi = m
    th = np.zeros(3)
    th[axis] = 0.5 * (lo + hi)
    Rq, tq = oracle.exp_so3(th), np.zeros(3)
    print("edge taps axis %d sign %d storage %d" % (axis, sign, storage), flush=True)
    A = rg.rgbid_pyramid(ctx, cam, 1, storage, *upload(I, W))
    B = rg.rgbid_pyramid(ctx, cam, 1, storage, *upload(Ib, Wb))
    g = rg.rgbid_normal_equations(ctx, A, B, 0, (Rq, tq), _params(1, [1]))
    r = oracle.normal_equations_at(cam, I, W, Ib, Wb, 0, Rq, tq,
                                   _oparams(1, [1], storage="f16" if storage else "f32"))
    check_normal_equations(g, r, what="edge taps axis %d sign %d storage %d" % (
        axis, sign, storage))
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


def test_argument_errors(ctx):
    rg = _rg()
    import torch
    I = torch.zeros(8, 8, device="cuda")
    with pytest.raises(rg.RgbidError) as e:
        rg.rgbid_pyramid(ctx, (8, 8, 5.0, 5.0, 3.5, 3.5), 9, 0, I, I)
    assert e.value.code == rg.RGBID_E_ARG
    A = rg.rgbid_pyramid(ctx, (8, 8, 5.0, 5.0, 3.5, 3.5), 2, 0, I, I)
    B = rg.rgbid_pyramid(ctx, (8, 8, 5.0, 5.0, 3.5, 3.5), 1, 0, I, I)
    with pytest.raises(rg.RgbidError) as e:
        rg.rgbid_align(ctx, A, B, _params(2, [1, 1]))
    assert e.value.code == rg.RGBID_E_SHAPE
    with pytest.raises(rg.RgbidError) as e:
        rg.rgbid_align(ctx, A, A, _params(6, [1] * 6))
    assert e.value.code == rg.RGBID_E_ARG
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


# ----------------------------------------------------------------- fusion


def test_fuse_batch_equals_sequential(ctx):
    # One launch over 20 frames gives the maps of 20 single-frame calls bit for
    # bit (the same per-pixel steps in the same order), and the same counts;
    # a batch of one is one call.
    rg = _rg()
    import torch
    cam, kf, frames, poses = synth.keyframe_sequence(20, seed=1, ss=2)
    Ws = [torch.from_numpy(f.W).cuda() for f in frames]
    K1 = rg.rgbid_keyframe_init(ctx, cam, torch.from_numpy(kf.W).cuda())
    K2 = rg.rgbid_keyframe_init(ctx, cam, torch.from_numpy(kf.W).cuda())
    n1 = [rg.rgbid_fuse(ctx, K1, w, T, 0.01) for w, T in zip(Ws, poses)]
    n2 = rg.rgbid_fuse_batch(ctx, K2, Ws, poses, 0.01, count=True)
    assert n1 == n2 and sum(n1) > 0
    W1, C1 = rg.rgbid_keyframe_read(ctx, K1, (cam.h, cam.w))
    W2, C2 = rg.rgbid_keyframe_read(ctx, K2, (cam.h, cam.w))
    assert torch.equal(W1, W2) and torch.equal(C1, C2)
    m1 = rg.rgbid_fuse(ctx, K1, Ws[3], poses[3], 0.01)
    m2 = rg.rgbid_fuse_batch(ctx, K2, Ws[3:4], poses[3:4], 0.01, count=True)
    assert [m1] == m2
    W1, C1 = rg.rgbid_keyframe_read(ctx, K1, (cam.h, cam.w))
    W2, C2 = rg.rgbid_keyframe_read(ctx, K2, (cam.h, cam.w))
    assert torch.equal(W1, W2) and torch.equal(C1, C2)
    with pytest.raises(rg.RgbidError):
        rg.rgbid_fuse_batch(ctx, K2, [], [], 0.01)
    with pytest.raises(rg.RgbidError):
        rg.rgbid_fuse_batch(ctx, K2, Ws[:2], poses[:2], 0.0)
    rg.rgbid_keyframe_free(K1)
    rg.rgbid_keyframe_free(K2)


def _fuse_margins(cam, Wkf, Wk, R, t, tol):
    """Per keyframe pixel, in FP64: the covisibility margin |W_k(p_w) - 1/Y_z|
    - tol of the fusion test (sec. 7.2, sec. 6.4) where the transfer reaches
    it (NaN elsewhere), and the distance of p_w to the bilinear bounds
    [-0.5, w - 0.5) x [-0.5, h - 0.5) (inf where Y_z <= 0)."""
    h, w = Wkf.shape
    v, u = np.mgrid[0:h, 0:w].astype(np.float64)
    ok = Wkf > 0
    wa = np.where(ok, Wkf, 1.0)
    ray = np.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, np.ones_like(u)], -1)
    Y = (ray / wa[..., None] - np.asarray(t)) @ np.asarray(R)     # R^T (X - t), row form
    front = ok & (Y[..., 2] > 0)
    z = np.where(front, Y[..., 2], 1.0)
    ub = cam.fx * Y[..., 0] / z + cam.cx
    vb = cam.fy * Y[..., 1] / z + cam.cy
    dist = np.minimum.reduce([np.abs(ub + 0.5), np.abs(ub - (w - 0.5)),
                              np.abs(vb + 0.5), np.abs(vb - (h - 0.5))])
    dist = np.where(front, dist, np.inf)
    inb = front & (ub >= -0.5) & (ub < w - 0.5) & (vb >= -0.5) & (vb < h - 0.5)
    x0 = np.floor(np.where(inb, ub, 0)).astype(int)
    y0 = np.floor(np.where(inb, vb, 0)).astype(int)
    a, b = np.where(inb, ub, 0) - x0, np.where(inb, vb, 0) - y0
    xa, xb = np.clip(x0, 0, w - 1), np.clip(x0 + 1, 0, w - 1)
    ya, yb = np.clip(y0, 0, h - 1), np.clip(y0 + 1, 0, h - 1)
    taps = [Wk[ya, xa], Wk[ya, xb], Wk[yb, xa], Wk[yb, xb]]
    good = inb & np.all([(x > 0) & np.isfinite(x) for x in taps], axis=0)
    wb = (1 - a) * (1 - b) * taps[0] + a * (1 - b) * taps[1] + (1 - a) * b * taps[2] + a * b * taps[3]
    margin = np.where(good, np.abs(wb - 1.0 / z) - tol, np.nan)
    return margin, dist


def test_fuse_20_frames_matches_oracle(ctx):
    # Decisions are compared frame by frame (a pixel was fused iff its C grew).
    # A decision may differ only where FP32 can legitimately take it the other
    # way: the oracle's covisibility margin |W_k(p_w) - 1/Y_z| - tol within
    # 1e-6 (a few FP32 ulps of inverse depths up to 2 m^-1: both sides carry
    # about four roundings of such values), or p_w within 1e-4 px of the image
    # bounds.  W and C are compared on every pixel whose 20 decisions agree at
    # 1e-5 relative, occlusion edges included (the transfer is formed as a
    # displacement, so its sample position is exact to ~3e-6 px).
    rg = _rg()
    import torch
    cam, kf, frames, poses = synth.keyframe_sequence(20, seed=0, ss=2)
    Wkf0 = kf.W.astype(np.float64)
    Wd = torch.from_numpy(kf.W).cuda()
    K = rg.rgbid_keyframe_init(ctx, cam, Wd)
    Wr, Cr = Wkf0.copy(), np.ones_like(Wkf0)
    tol = 0.01
    agree = np.ones(Wkf0.shape, dtype=bool)
    Cg_prev = np.ones_like(Wkf0)
    total_fused = 0
    for k, (f, (R, t)) in enumerate(zip(frames, poses)):
        n = rg.rgbid_fuse(ctx, K, torch.from_numpy(f.W).cuda(), (R, t), tol)
        Cr_prev, Wr_prev = Cr, Wr
        Wr, Cr, nr = oracle.fuse(cam, Wr, Cr, f.W, R, t, tol)
        _, Cg = rg.rgbid_keyframe_read(ctx, K, (cam.h, cam.w))
        Cg = Cg.cpu().numpy().astype(np.float64)
        dec_g, dec_r = Cg > Cg_prev, Cr > Cr_prev
        flip = dec_g != dec_r
        assert int(dec_g.sum()) == n and int(dec_r.sum()) == nr
        if flip.any():
            margin, dist = _fuse_margins(cam, Wr_prev, f.W.astype(np.float64), R, t, tol)
            vv, uu = np.nonzero(flip)
            print("frame %d: %d decision(s) differ:" % (k, len(vv)),
                  [(int(a), int(b), float(margin[a, b]), float(dist[a, b])) for a, b in zip(vv, uu)])
            near = (np.abs(np.nan_to_num(margin, nan=np.inf)) <= 1e-6) | (dist <= 1e-4)
            assert np.all(near[flip]), "a decision differs away from the threshold"
        assert int(flip.sum()) <= 20
        agree &= ~flip
        Cg_prev = Cg
        total_fused += n
    assert total_fused > 20 * 0.5 * cam.w * cam.h
    Wg, Cg = rg.rgbid_keyframe_read(ctx, K, (cam.h, cam.w))
    Wg, Cg = Wg.cpu().numpy().astype(np.float64), Cg.cpu().numpy().astype(np.float64)
    assert agree.mean() > 0.999
    np.testing.assert_allclose(Wg[agree], Wr[agree], rtol=1e-5)
    np.testing.assert_allclose(Cg[agree], Cr[agree], rtol=1e-5)
    assert np.all((Wg > 0) == (Wkf0 > 0))       # keyframe holes stay holes
    rg.rgbid_keyframe_free(K)


# ----------------------------------------------------------------- covisibility


def _fragile_counts(cl, WA, WB, R, t, tol):
    """How far the oracle's own |S_V| counts move when the decisions are
    re-taken at perturbations above FP32 rounding (pose by 2e-6 rad / 2e-6 m
    along each axis, tol by 5e-5 relative: a few FP32 ulps of W ~ 1 against
    tol = 0.01): a bound on the pixels whose
    visibility FP32 arithmetic may legitimately decide the other way."""
    from scipy.spatial.transform import Rotation
    _, base = oracle.covisibility_ratio(cl, WA, WB, R, t, tol)
    worst = [0, 0]
    perts = [(Rotation.from_rotvec(2e-6 * e).as_matrix() @ R, t) for e in np.eye(3)]
    perts += [(R, t + 2e-6 * e) for e in np.eye(3)]
    for Rp, tp in perts:
        for tt in (tol * (1 - 5e-5), tol * (1 + 5e-5)):
            _, c = oracle.covisibility_ratio(cl, WA, WB, Rp, tp, tt)
            worst[0] = max(worst[0], abs(c[1] - base[1]))
            worst[1] = max(worst[1], abs(c[3] - base[3]))
    return worst


@pytest.mark.parametrize("level", [0, 2])
def test_covisibility_matches_oracle(ctx, c2_pairs, level):
    # counts decided in FP32 on the GPU and FP64 in the oracle: hole masks
    # equal, visible counts equal up to twice the oracle's own sensitivity to
    # perturbations above FP32 rounding (plus 2)
    rg = _rg()
    p = c2_pairs[0]
    A = _pyr(ctx, p.cam, 3, p.A)
    B = _pyr(ctx, p.cam, 3, p.B)
    WA = oracle.pyramid(p.cam, 3, p.A.I, p.A.W, storage="f32")[level][1]
    WB = oracle.pyramid(p.cam, 3, p.B.I, p.B.W, storage="f32")[level][1]
    cl = oracle.camera_level(p.cam, level)
    for (R, t) in [(np.eye(3), np.zeros(3)), (p.R, p.t)]:
        r, cnt = rg.rgbid_covisibility(ctx, A, B, level, (R, t), 0.01)
        rr, cr = oracle.covisibility_ratio(cl, WA, WB, R, t, 0.01)
        assert cnt[0] == cr[0] and cnt[2] == cr[2]          # hole masks: exact
        fa, fb = _fragile_counts(cl, WA, WB, R, t, 0.01)
        assert abs(cnt[1] - cr[1]) <= 2 * fa + 2 and abs(cnt[3] - cr[3]) <= 2 * fb + 2, \
            (cnt, cr, fa, fb)
        assert abs(r - rr) <= (2 * max(fa, fb) + 2) / min(cr[0], cr[2])
        assert 0.3 < r <= 1.0
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)


# ----------------------------------------------------------------- covariance


def test_covariance_matches_oracle(ctx, c2_pairs):
    # Sigma = H_filt^-1 from the bilateral-filtered reference at the final pose:
    # the filtered normal equations meet the normal-equation bound, and the GPU
    # covariance inverts the oracle's filtered Hessian.
    rg = _rg()
    p = c2_pairs[1]
    A = _pyr(ctx, p.cam, 4, p.A)
    B = _pyr(ctx, p.cam, 4, p.B)
    prm = _params(4, [10] * 4)
    R, t, _, rc = rg.rgbid_align(ctx, A, B, prm)
    S, st = rg.rgbid_covariance(ctx, A, B, (R, t), prm)
    So, sto = oracle.covariance(p.cam, p.A.I, p.A.W, p.B.I, p.B.W, R, t, _oparams(4, [1] * 4))
    check_normal_equations(st, sto, what="filtered covariance iteration")
    np.testing.assert_allclose(S @ sto["H"], np.eye(6), atol=2e-3)
    d = np.sqrt(np.diag(So))
    assert np.all(np.abs(S - So) <= 2e-3 * np.outer(d, d) + 1e-30)
    rg.rgbid_pyramid_free(A)
    rg.rgbid_pyramid_free(B)
