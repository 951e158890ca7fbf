"""GPU parity of the warm-start network kernels against the FP64 numpy oracle
(oracle/cnn.py): input assembly from the pyramids, forward output, loss,
every parameter gradient, and one AdamW step.

Tolerances: the GPU keeps activations and sums in FP32 over up to 307k terms
per gradient entry, so each parameter tensor's gradient must agree within
1e-4 of that tensor's largest entry; outputs and the loss within 1e-5."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import cnn
from _parity import upload

pytestmark = pytest.mark.gpu


def _rg():
    from paper_1807_08271_amd import rgbid
    return rgbid


@pytest.fixture(scope="module")
def batch(ctx):
    rg = _rg()
    pairs = [synth.pair_c2(i, ss=2) for i in range(3)] + [synth.pair_warm(0, "eval", ss=2)]
    As = [rg.rgbid_pyramid(ctx, p.cam, 4, rg.RGBID_F32, *upload(p.A.I, p.A.W)) for p in pairs]
    Bs = [rg.rgbid_pyramid(ctx, p.cam, 4, rg.RGBID_F32, *upload(p.B.I, p.B.W)) for p in pairs]
    n = len(pairs)
    x = torch.zeros((n, 4, 60, 80), dtype=torch.float32, device="cuda")
    rg.rgbid_warmstart_input(ctx, As, Bs, x)
    torch.cuda.synchronize()
    # oracle input from the oracle's own pyramid (FP32-rounded levels)
    xr = np.zeros((n, 4, 60, 80))
    for i, p in enumerate(pairs):
        IA, WA = oracle.pyramid(p.cam, 4, p.A.I, p.A.W, storage="f32")[3]
        IB, WB = oracle.pyramid(p.cam, 4, p.B.I, p.B.W, storage="f32")[3]
        xr[i] = [IA / 255.0, WA / 2.0, IB / 255.0, WB / 2.0]
    labels = np.array([np.concatenate([p.t, oracle.log_so3(p.R)]) for p in pairs])
    yield dict(pairs=pairs, As=As, Bs=Bs, x=x, xr=xr, labels=labels, n=n)
    for q in As + Bs:
        rg.rgbid_pyramid_free(q)


def test_input_matches_oracle_pyramid(batch):
    xg = batch["x"].cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(xg, batch["xr"], rtol=5e-7, atol=1e-7)


def test_forward_loss_and_gradients_match_oracle(ctx, batch):
    rg = _rg()
    params = cnn.init_params(7)
    net = rg.rgbid_warmstart_create(ctx, params)
    eff = cnn.effective_params(params)
    out_r, cache = cnn.forward(eff, batch["xr"])
    xi_g = rg.rgbid_warmstart_forward(ctx, net, batch["x"], batch["n"])
    np.testing.assert_allclose(xi_g, out_r * cnn.SCALE, rtol=1e-5, atol=1e-6)
    loss_g, grad_g = rg.rgbid_warmstart_gradient(ctx, net, batch["x"], batch["labels"])
    loss_r = cnn.loss(out_r, batch["labels"])
    grad_r, _ = cnn.backward(eff, cache, out_r, batch["labels"])
    assert loss_g == pytest.approx(loss_r, rel=1e-5)
    off = 0
    for i, shp in enumerate(cnn.param_shapes()):
        k = int(np.prod(shp))
        g, r = grad_g[off:off + k].astype(np.float64), grad_r[off:off + k]
        scale = np.abs(r).max()
        assert scale > 0
        err = np.abs(g - r).max() / scale
        assert err <= 1e-4, (i, shp, err)
        off += k
    rg.rgbid_warmstart_free(net)


def test_matrix_core_forward_matches_oracle(ctx, batch):
    # The inference forward on the matrix cores (implicit-GEMM convolutions
    # of bf16 weights and three-limb bf16 activations, FP32 accumulation)
    # reads the pyramids itself and must give the FP32 forward's result: the
    # oracle's within the same 1e-5 / 1e-6, and the FP32 kernels' within FP32
    # summation-order differences.  Then a few training steps later (the
    # GEMM-order weights follow the updated parameters).
    rg = _rg()
    params = cnn.init_params(11)
    net = rg.rgbid_warmstart_create(ctx, params)
    for step in range(2):
        eff = cnn.effective_params(rg.rgbid_warmstart_get_params(ctx, net))
        out_r, _ = cnn.forward(eff, batch["xr"])
        xi_m = rg.rgbid_warmstart_forward_pyr(ctx, net, batch["As"], batch["Bs"])
        xi_f = rg.rgbid_warmstart_forward(ctx, net, batch["x"], batch["n"])
        np.testing.assert_allclose(xi_m, out_r * cnn.SCALE, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(xi_m, xi_f, rtol=1e-5, atol=1e-6)
        poses = rg.rgbid_warmstart_predict(ctx, net, batch["As"], batch["Bs"], batch["x"])
        for i, (R, t) in enumerate(poses):
            np.testing.assert_allclose(t, xi_m[i, :3], rtol=0, atol=0)
            np.testing.assert_allclose(oracle.log_so3(R), xi_m[i, 3:], atol=1e-12)
        for _ in range(3):
            rg.rgbid_warmstart_train_step(ctx, net, batch["x"], batch["labels"], lr=1e-3)
    rg.rgbid_warmstart_free(net)


def test_align_batch_warm_matches_predict_then_align(ctx, batch):
    # The one-call warm start (initial poses formed on the device) against
    # predict + rgbid_align_batch: the same initial poses up to the last bits
    # of FP64 sin / cos, so the same converged poses within 1e-9, and the
    # same statuses.
    rg = _rg()
    from paper_1807_08271_amd import warmstart as ws
    net = rg.rgbid_warmstart_create(ctx, ws.load_weights())
    prm = rg.rgbid_default_params(levels=4, iters=[10] * 4)   # fixed schedule
    inits = rg.rgbid_warmstart_predict(ctx, net, batch["As"], batch["Bs"], batch["x"])
    p1, s1 = rg.rgbid_align_batch(ctx, batch["As"], batch["Bs"], prm, inits=inits)
    p2, s2 = rg.rgbid_align_batch_warm(ctx, net, batch["As"], batch["Bs"], prm)
    for i in range(batch["n"]):
        assert s1[i]["status"] == s2[i]["status"], i
        np.testing.assert_allclose(p2[i][0], p1[i][0], atol=1e-9)
        np.testing.assert_allclose(p2[i][1], p1[i][1], atol=1e-9)
    rg.rgbid_warmstart_free(net)


def test_adamw_step_matches_oracle(ctx, batch):
    rg = _rg()
    params = cnn.init_params(8)
    net = rg.rgbid_warmstart_create(ctx, params)
    _, g = rg.rgbid_warmstart_gradient(ctx, net, batch["x"], batch["labels"])
    rg.rgbid_warmstart_train_step(ctx, net, batch["x"], batch["labels"], lr=1e-3, wd=1e-2)
    w1 = rg.rgbid_warmstart_get_params(ctx, net)
    # the optimiser arithmetic on the GPU's own (deterministic) gradient
    wr, _, _ = cnn.adamw_step(params.astype(np.float64), g.astype(np.float64),
                              np.zeros(len(g)), np.zeros(len(g)), 1, 1e-3, wd=1e-2,
                              decay_mask=cnn.weight_mask())
    np.testing.assert_allclose(w1, wr, rtol=1e-6, atol=1e-9)
    rg.rgbid_warmstart_free(net)


def test_training_reduces_loss_deterministically(ctx, batch):
    rg = _rg()
    params = cnn.init_params(9)
    runs = []
    for _ in range(2):
        net = rg.rgbid_warmstart_create(ctx, params)
        losses = [rg.rgbid_warmstart_train_step(ctx, net, batch["x"], batch["labels"], lr=3e-3,
                                                want_loss=True) for _ in range(60)]
        runs.append((losses, rg.rgbid_warmstart_get_params(ctx, net)))
        rg.rgbid_warmstart_free(net)
    assert runs[0][0][-1] < 0.05 * runs[0][0][0]
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
