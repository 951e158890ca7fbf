"""What the trained warm start gains over plain Gauss-Newton: on held-out
large-motion pairs (<= 10 deg / 15 cm, seeds and scenes disjoint from
training), network + Gauss-Newton reaches the Gauss-Newton optimum next to
the truth at least as often as Gauss-Newton from the identity, with fewer
iterations (both stop early at 1e-6).  Uses the weights that
`python -m paper_1807_08271_amd.warmstart` trained with the library's own
kernels."""
import os

import pytest

pytestmark = pytest.mark.gpu


def test_warm_start_gain(ctx):
    from paper_1807_08271_amd import rgbid as rg
    from paper_1807_08271_amd import warmstart as ws
    assert os.path.exists(ws.DEFAULT_WEIGHTS), "train the warm start first"
    net = rg.rgbid_warmstart_create(ctx, ws.load_weights())
    res = ws.evaluate(ctx, net, n_pairs=128, chunk=64, log=print,
                      schedules={"plain": (False, (10, 10, 10, 10)),
                                 "warm": (True, (10, 10, 10, 10))})
    rg.rgbid_warmstart_free(net)
    plain, warm = res["plain"], res["warm"]
    assert warm["pairs"] >= 100
    assert warm["success_rate"] >= plain["success_rate"]
    assert warm["mean_gn_iters"] < plain["mean_gn_iters"]
