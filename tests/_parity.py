"""Shared helpers of the GPU parity tests: tolerances of the normal equations,
pose errors, and device upload of synthetic frames."""
import numpy as np

import oracle


def rot_err(Ra, Rb):
    return float(np.linalg.norm(oracle.log_so3(Ra.T @ Rb)))


def check_normal_equations(gpu, ref, rel=1e-4, flips=20, what=""):
    """|dH_ij| <= rel sqrt(H_ii H_jj), |dg_i| <= rel sqrt(H_ii cost), and the
    valid-pixel counts within `flips` (pixels whose inclusion is decided
    within FP32 rounding of a threshold)."""
    H, Hr = gpu["H"], ref["H"]
    d = np.sqrt(np.abs(np.diag(Hr)))
    bound_H = rel * np.outer(d, d) + 1e-300
    eH = np.abs(H - Hr) / bound_H
    bound_g = rel * d * np.sqrt(abs(ref["cost"])) + 1e-300
    eg = np.abs(gpu["g"] - ref["g"]) / bound_g
    dn = abs(gpu["n_valid_I"] - ref["n_valid_I"]) + abs(gpu["n_valid_W"] - ref["n_valid_W"])
    msg = "%s: max H err %.3g, max g err %.3g (units of the bound), count diff %d" % (
        what, eH.max(), eg.max(), dn)
    assert eH.max() <= 1.0 and eg.max() <= 1.0 and dn <= flips, msg
    return eH.max(), eg.max(), dn


def upload(frame_I, frame_W, device="cuda"):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(frame_I, dtype=np.float32)).to(device),
            torch.from_numpy(np.ascontiguousarray(frame_W, dtype=np.float32)).to(device))
