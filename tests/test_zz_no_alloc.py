"""The allocation-free alignment (rgbid_align_noalloc) against rgbid_align
through the C ABI: two calls in a row on one context, the second on a
smaller pair, each equal to rgbid_align bit for bit (both use the default
launch shapes on a fresh context) and so within the parity bar of the oracle
comparisons (1e-5 rad / 1e-5 m); the statistics of the last linearisation
equal too.  A pair too large for the scratch array is refused."""
import numpy as np
import pytest

import synth
from _parity import upload

pytestmark = pytest.mark.gpu


def _rg():
    from paper_1807_08271_amd import rgbid
    return rgbid


def test_noalloc_matches_align_twice_then_smaller():
    rg = _rg()
    import torch
    assert torch.cuda.is_available()
    ctx = rg.rgbid_create(0)     # fresh context: no tuned launch shapes
    try:
        cases = [(synth.pair_c2(0, ss=2), 4, [10] * 4, "fullres"),
                 (synth.pair_c1(1), 2, [6, 6], "per_level")]
        for p, levels, iters, warp in cases:
            print("noalloc case %dx%d, %d levels, %s" % (p.cam.w, p.cam.h, levels, warp), flush=True)
            A = rg.rgbid_pyramid(ctx, p.cam, levels, 0, *upload(p.A.I, p.A.W))
            B = rg.rgbid_pyramid(ctx, p.cam, levels, 0, *upload(p.B.I, p.B.W))
            prm = rg.rgbid_default_params(
                levels=levels, iters=iters,
                warp=rg.RGBID_WARP_FULLRES if warp == "fullres" else rg.RGBID_WARP_PER_LEVEL)
            R0, t0, s0, rc0 = rg.rgbid_align(ctx, A, B, prm)
            R1, t1, s1, rc1 = rg.rgbid_align_noalloc(ctx, A, B, prm)
            assert rc0 == rc1 == 0
            ang = np.linalg.norm(np.array([R1[2, 1] - R1[1, 2], R1[0, 2] - R1[2, 0],
                                           R1[1, 0] - R1[0, 1]]) - np.array(
                [R0[2, 1] - R0[1, 2], R0[0, 2] - R0[2, 0], R0[1, 0] - R0[0, 1]])) / 2
            assert ang <= 1e-5 and np.linalg.norm(t1 - t0) <= 1e-5
            np.testing.assert_array_equal(R1, R0)
            np.testing.assert_array_equal(t1, t0)
            for k in ("H", "g", "cost", "mu_I", "sigma_I", "mu_W", "sigma_W", "n_valid_I",
                      "n_valid_W", "iters_done", "status"):
                np.testing.assert_array_equal(np.asarray(s1[k]), np.asarray(s0[k]), k)
            # an initial guess goes in the same way
            R2, t2, _, _ = rg.rgbid_align_noalloc(ctx, A, B, prm, init=(p.R, p.t))
            R3, t3, _, _ = rg.rgbid_align(ctx, A, B, prm, init=(p.R, p.t))
            np.testing.assert_array_equal(R2, R3)
            np.testing.assert_array_equal(t2, t3)
            rg.rgbid_pyramid_free(A)
            rg.rgbid_pyramid_free(B)
        # beyond the scratch array: a 2048x2000 pair (its stored 1024x1000
        # warped level alone is 8.19 MB, with the partial sums and the sample
        # past 8 MiB) is refused before any launch
        cam = (2048, 2000, 1500.0, 1500.0, 1023.5, 999.5)
        I = torch.full((2000, 2048), 100.0, device="cuda")
        W = torch.full((2000, 2048), 0.5, device="cuda")
        big = rg.rgbid_pyramid(ctx, cam, 3, 0, I, W)
        with pytest.raises(rg.RgbidError) as e:
            rg.rgbid_align_noalloc(ctx, big, big, rg.rgbid_default_params(levels=3, iters=[1] * 3,
                                                                          sample_max=24576))
        assert e.value.code == rg.RGBID_E_ARG
        rg.rgbid_pyramid_free(big)
    finally:
        torch.cuda.synchronize()
        rg.rgbid_destroy(ctx)
