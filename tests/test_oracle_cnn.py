"""Pins of the warm-start network oracle: brute-force convolution loops,
central finite differences of the loss, bf16 rounding against torch, and the
AdamW update against torch.optim.AdamW."""
import numpy as np
import pytest
import torch

from oracle import cnn


def test_param_count_and_shapes():
    assert cnn.n_params() == 241894
    x = np.zeros((1, 4, 60, 80))
    out, (acts, pooled) = cnn.forward(cnn.effective_params(cnn.init_params(0)), x)
    assert [a.shape[2:] for a in acts] == [(60, 80), (30, 40), (15, 20), (8, 10), (4, 5)]
    assert out.shape == (1, 6)


def test_conv_against_brute_force_loops():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 7, 9))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    z = cnn.conv_fwd(x, w, b)
    assert z.shape == (2, 4, 4, 5)
    for n in range(2):
        for o in range(4):
            for y in range(4):
                for xx in range(5):
                    acc = b[o]
                    for c in range(3):
                        for ky in range(3):
                            for kx in range(3):
                                iy, ix = 2 * y - 1 + ky, 2 * xx - 1 + kx
                                if 0 <= iy < 7 and 0 <= ix < 9:
                                    acc += w[o, c, ky, kx] * x[n, c, iy, ix]
                    assert z[n, o, y, xx] == pytest.approx(acc, rel=1e-12, abs=1e-12)


def test_conv_against_torch_conv2d():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 4, 60, 80))
    w = rng.normal(size=(8, 4, 3, 3))
    b = rng.normal(size=8)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x), torch.from_numpy(w),
                                     torch.from_numpy(b), stride=2, padding=1).numpy()
    np.testing.assert_allclose(cnn.conv_fwd(x, w, b), ref, rtol=1e-12, atol=1e-12)


def test_round_bf16_against_torch():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(size=5000).astype(np.float32),
                        (rng.normal(size=5000) * 1e-3).astype(np.float32),
                        np.array([0.0, -0.0, 1.0, 3.0e38], dtype=np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(cnn.round_bf16(x), ref)


def test_gradients_against_finite_differences():
    rng = np.random.default_rng(3)
    flat = cnn.init_params(5).astype(np.float64)
    params = cnn.unpack(flat)
    x = rng.uniform(0, 1, size=(2, 4, 60, 80))
    xi = rng.normal(size=(2, 6)) * cnn.SCALE * 0.3
    out, cache = cnn.forward(params, x)
    g, gx = cnn.backward(params, cache, out, xi)

    def L(f):
        o, _ = cnn.forward(cnn.unpack(f), x)
        return cnn.loss(o, xi)

    idx = np.concatenate([rng.integers(0, cnn.n_params(), 40),
                          np.arange(cnn.n_params() - 6, cnn.n_params())])
    for i in idx:
        e = np.zeros_like(flat)
        h = 1e-5 * max(1.0, abs(flat[i]))
        e[i] = h
        fd = (L(flat + e) - L(flat - e)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-8), i
    # input gradient at a few positions
    for (c, yy, xx) in [(0, 10, 10), (3, 59, 79), (1, 0, 0)]:
        def Lx(d):
            x2 = x.copy()
            x2[0, c, yy, xx] += d
            o, _ = cnn.forward(params, x2)
            return cnn.loss(o, xi)
        fd = (Lx(1e-5) - Lx(-1e-5)) / 2e-5
        assert gx[0, c, yy, xx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_adamw_against_torch():
    rng = np.random.default_rng(4)
    w0 = rng.normal(size=50)
    mask = (np.arange(50) < 30).astype(float)
    grads = [rng.normal(size=50) for _ in range(5)]
    tw = torch.nn.Parameter(torch.from_numpy(w0[:30].copy()))
    tb = torch.nn.Parameter(torch.from_numpy(w0[30:].copy()))
    opt = torch.optim.AdamW([{"params": [tw], "weight_decay": 1e-2},
                             {"params": [tb], "weight_decay": 0.0}], lr=1e-2, eps=1e-8)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for step, g in enumerate(grads, 1):
        tw.grad = torch.from_numpy(g[:30].copy())
        tb.grad = torch.from_numpy(g[30:].copy())
        opt.step()
        w, m, v = cnn.adamw_step(w, g, m, v, step, 1e-2, wd=1e-2, decay_mask=mask)
    ref = np.concatenate([tw.detach().numpy(), tb.detach().numpy()])
    np.testing.assert_allclose(w, ref, rtol=1e-12, atol=1e-14)
