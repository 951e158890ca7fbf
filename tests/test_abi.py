"""The C-ABI library loads and exports every entry point include/rgbid.h
declares (no device calls: runs without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rgbid.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rgbid_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1807_08271_amd import rgbid
    lib = rgbid.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(rgbid.exported_symbols())


def test_default_params():
    from paper_1807_08271_amd import rgbid
    p = rgbid.rgbid_default_params()
    assert p.levels == 4 and list(p.iters)[:4] == [10] * 4
    assert p.weight == rgbid.RGBID_W_HUBER and abs(p.huber_k - 1.345) < 1e-15
    assert p.sample_max == 19200 and p.scale_iters == 20 and p.warp == rgbid.RGBID_WARP_FULLRES
    assert p.scale_warm == 1
    assert rgbid.rgbid_default_params(scale_warm=0).scale_warm == 0
    with pytest.raises(TypeError):
        rgbid.rgbid_default_params(scale_wram=0)


def test_pose_maps_host_functions():
    # the decoupled exp / log of the library's host code against scipy
    import numpy as np
    from scipy.spatial.transform import Rotation
    from paper_1807_08271_amd import rgbid
    rng = np.random.default_rng(0)
    for _ in range(20):
        xi = np.concatenate([rng.normal(size=3), rng.normal(size=3) * 0.5])
        R, t = rgbid.rgbid_pose_exp(xi)
        np.testing.assert_allclose(R, Rotation.from_rotvec(xi[3:]).as_matrix(), atol=1e-14)
        np.testing.assert_array_equal(t, xi[:3])
        np.testing.assert_allclose(rgbid.rgbid_pose_log(R, t), xi, atol=1e-12)


def test_tracker_default_params():
    from paper_1807_08271_amd import rgbid
    p = rgbid.rgbid_tracker_default_params()
    assert p.align.levels == 4 and p.align.weight == rgbid.RGBID_W_HUBER
    assert p.rf_threshold == 0.8 and p.kf_threshold == 0.7
    assert p.covis_level == 2 and p.tol_sigmas == 3.0 and p.buffer == 8 and p.covariance == 1
