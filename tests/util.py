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


def ls_denominators(t, f, block=1024):
    """D_c = sum cos^2(w(t - tau)) and D_s = sum sin^2(w(t - tau)) per frequency
    in FP64, tau from tan 2 w tau = sum sin 2wt / sum cos 2wt (Eq. 2).  Used
    only to mark bins where Pn is ill-conditioned: a denominator of 1e-7 Nt
    makes Pn change by its full size under a 1e-7 relative change of the
    trigonometric values, which no FP32 path can meet."""
    t = np.asarray(t, dtype=np.float64)
    t = t - 0.5 * (t.min() + t.max())
    f = np.asarray(f, dtype=np.float64)
    Dc = np.empty(f.size)
    Ds = np.empty(f.size)
    for k0 in range(0, f.size, block):
        ph = np.outer(f[k0:k0 + block], t)
        ph -= np.rint(ph)
        th = 4.0 * np.pi * ph
        tau2 = np.arctan2(np.sin(th).sum(1), np.cos(th).sum(1))  # 2 w tau
        a = 2.0 * np.pi * ph - 0.5 * tau2[:, None]
        Dc[k0:k0 + block] = (np.cos(a) ** 2).sum(1)
        Ds[k0:k0 + block] = (np.sin(a) ** 2).sum(1)
    return Dc, Ds
