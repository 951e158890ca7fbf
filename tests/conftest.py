import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    oracle.build(force=False)
    yield


@pytest.fixture(scope="session")
def ctx():
    """A library context on cuda:0 (GPU tests only)."""
    import torch
    from paper_1807_08271_amd import rgbid
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = rgbid.rgbid_create(0)
    yield c
    torch.cuda.synchronize()
    rgbid.rgbid_destroy(c)


@pytest.fixture(scope="session")
def c1_pairs():
    import synth
    return [synth.pair_c1(i) for i in range(3)]


@pytest.fixture(scope="session")
def c2_pairs():
    import synth
    return [synth.pair_c2(i, ss=2) for i in range(2)]
