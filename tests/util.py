"""Shared helpers for the GPU parity tests (comparison rules, device upload)."""
import numpy as np

REL_TOL = 1e-4   # max|dPn| / max(Pn_oracle)


def rel_err(p_gpu, p_orc):
    p_gpu = np.asarray(p_gpu, dtype=np.float64)
    p_orc = np.asarray(p_orc, dtype=np.float64)
    return float(np.max(np.abs(p_gpu - p_orc)) / np.max(p_orc))


def peak_matches(p_gpu, p_orc, tol=REL_TOL):
    """Argmax agrees, or the oracle's own top bins are within tol of each other
    (then any of those bins is a correct answer)."""
    p_gpu = np.asarray(p_gpu, dtype=np.float64)
    p_orc = np.asarray(p_orc, dtype=np.float64)
    kg = int(np.argmax(p_gpu))
    ko = int(np.argmax(p_orc))
    if kg == ko:
        return True
    return p_orc[ko] - p_orc[kg] <= tol * p_orc[ko]


def to_dev(curve, device="cuda"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(curve.t, dtype=np.float64)).to(device)
    x = torch.from_numpy(np.ascontiguousarray(curve.x, dtype=np.float32)).to(device)
    return t, x
