"""FP64 CPU oracle for the normalized Lomb-Scargle periodogram.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check in
__graft_entry__.py and by the cpu_baseline leg of bench.py -- never by the
package paper_1007_1658_amd.  It shares no code with the HIP path.

The arithmetic lives in lsp_oracle.c (Eqs. (1)-(3) of Section 3, the grid of
Section 4.3); this module only marshals numpy arrays into it, plus the pure
numpy pieces that have no C twin (per-curve maxima of a batch).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        P = ctypes.c_void_p
        lib.oracle_normalize.argtypes = [P, i64, P, P, P]
        lib.oracle_normalize.restype = i32
        lib.oracle_periodogram.argtypes = [P, P, i64, d, d, P, i64, P, i32]
        lib.oracle_periodogram.restype = i32
        lib.oracle_periodogram_ld.argtypes = [P, P, i64, d, d, P, i64, P, i32]
        lib.oracle_periodogram_ld.restype = i32
        lib.oracle_fap.argtypes = [d, i64, i64]
        lib.oracle_fap.restype = d
        lib.oracle_window.argtypes = [P, i64, d, d, i64, P, i32]
        lib.oracle_window.restype = i32
        lib.oracle_gls.argtypes = [P, P, P, i64, d, d, P, i64, P, i32]
        lib.oracle_gls.restype = i32
        lib.oracle_mh.argtypes = [P, P, P, i64, i32, d, d, P, i64, P, i32]
        lib.oracle_mh.restype = i32
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = i32
        lib.oracle_philox4x32_10.argtypes = [P, P, P]
        lib.oracle_philox4x32_10.restype = None
        lib.oracle_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint64, i64, P]
        lib.oracle_normals.restype = None
        _LIB = lib
    return _LIB


class OracleError(RuntimeError):
    pass


ZERO_VARIANCE = -2


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_lib().oracle_max_threads())


def normalize(x):
    """(X, mean, var): zero mean, unit population variance (Section 3)."""
    x = _f64(x)
    X = np.empty_like(x)
    mean = ctypes.c_double()
    var = ctypes.c_double()
    rc = _lib().oracle_normalize(_ptr(x), x.size, _ptr(X), ctypes.byref(mean), ctypes.byref(var))
    if rc != 0:
        raise OracleError(f"oracle_normalize failed ({rc})")
    return X, mean.value, var.value


def periodogram(t, x, f_min, df, Nf=None, k=None, long_double=False, threads=0):
    """Pn(f_k), f_k = f_min + k df, in FP64 by the two-pass Eqs. (1)-(2).

    Either Nf (k = 0..Nf-1) or an explicit integer array k is given.
    """
    t = _f64(t)
    x = _f64(x)
    if t.shape != x.shape or t.ndim != 1:
        raise OracleError("t and x must be 1-D of equal length")
    if k is None:
        if Nf is None:
            raise OracleError("give Nf or k")
        kp = None
        n_out = int(Nf)
    else:
        kk = np.ascontiguousarray(np.asarray(k, dtype=np.int64))
        kp = _ptr(kk)
        n_out = kk.size
    out = np.empty(n_out, dtype=np.float64)
    fn = _lib().oracle_periodogram_ld if long_double else _lib().oracle_periodogram
    rc = fn(_ptr(t), _ptr(x), t.size, float(f_min), float(df), kp, n_out, _ptr(out), int(threads))
    if rc == ZERO_VARIANCE:
        raise OracleError("zero variance")
    if rc != 0:
        raise OracleError(f"oracle_periodogram failed ({rc})")
    return out


def gls(t, y, f_min, df, Nf=None, k=None, w=None, threads=0):
    """Generalized (floating-mean, weighted) periodogram p(f_k) in FP64:
    the weighted least-squares fraction of variance explained by
    a cos + b sin + c at each frequency (w None: equal weights)."""
    t = _f64(t)
    y = _f64(y)
    if t.shape != y.shape or t.ndim != 1:
        raise OracleError("t and y must be 1-D of equal length")
    wp = None
    if w is not None:
        w = _f64(w)
        if w.shape != t.shape:
            raise OracleError("w must match t")
        wp = _ptr(w)
    if k is None:
        if Nf is None:
            raise OracleError("give Nf or k")
        kp, n_out = None, int(Nf)
    else:
        kk = np.ascontiguousarray(np.asarray(k, dtype=np.int64))
        kp, n_out = _ptr(kk), kk.size
    out = np.empty(n_out, dtype=np.float64)
    rc = _lib().oracle_gls(_ptr(t), _ptr(y), wp, t.size, float(f_min), float(df), kp, n_out, _ptr(out),
                           int(threads))
    if rc == ZERO_VARIANCE:
        raise OracleError("zero variance")
    if rc != 0:
        raise OracleError(f"oracle_gls failed ({rc})")
    return out


def multiharmonic(t, y, K, f_min, df, Nf=None, k=None, w=None, threads=0):
    """Multi-harmonic periodogram p_K(f_k) in FP64: the weighted least-squares
    fraction of variance explained by c + sum_{h<=K} (a_h cos h wt + b_h sin h wt)."""
    t = _f64(t)
    y = _f64(y)
    if t.shape != y.shape or t.ndim != 1:
        raise OracleError("t and y must be 1-D of equal length")
    wp = None
    if w is not None:
        w = _f64(w)
        if w.shape != t.shape:
            raise OracleError("w must match t")
        wp = _ptr(w)
    if k is None:
        if Nf is None:
            raise OracleError("give Nf or k")
        kp, n_out = None, int(Nf)
    else:
        kk = np.ascontiguousarray(np.asarray(k, dtype=np.int64))
        kp, n_out = _ptr(kk), kk.size
    out = np.empty(n_out, dtype=np.float64)
    rc = _lib().oracle_mh(_ptr(t), _ptr(y), wp, t.size, int(K), float(f_min), float(df), kp, n_out, _ptr(out),
                          int(threads))
    if rc == ZERO_VARIANCE:
        raise OracleError("zero variance")
    if rc != 0:
        raise OracleError(f"oracle_mh failed ({rc})")
    return out


def fap(Pn, Nt, Nf):
    """Eq. (3) false-alarm probability (vectorised over Pn)."""
    f = _lib().oracle_fap
    arr = np.atleast_1d(np.asarray(Pn, dtype=np.float64))
    out = np.array([f(float(p), int(Nt), int(Nf)) for p in arr.ravel()]).reshape(arr.shape)
    return out if np.ndim(Pn) else float(out[0])


def window(t, f_min, df, Nf, threads=0):
    """Spectral window W(f_k) = |sum_j exp(2 pi i f_k t_j)|^2 in FP64."""
    t = _f64(t)
    out = np.empty(int(Nf), dtype=np.float64)
    rc = _lib().oracle_window(_ptr(t), t.size, float(f_min), float(df), int(Nf), _ptr(out), int(threads))
    if rc != 0:
        raise OracleError(f"oracle_window failed ({rc})")
    return out


def peak(Pn):
    """(max, argmax) with the lowest index on exact ties."""
    Pn = np.asarray(Pn)
    k = int(np.argmax(Pn))  # numpy returns the first maximal index
    return float(Pn[k]), k


def batched_peaks(t, x, off, f_min, df, Nf, curves=None, threads=0):
    """Per-curve (max Pn, argmax k) of a CSR batch, by calling periodogram per curve."""
    off = np.asarray(off, dtype=np.int64)
    n = off.size - 1
    sel = range(n) if curves is None else curves
    res = {}
    for c in sel:
        a, b = int(off[c]), int(off[c + 1])
        P = periodogram(t[a:b], x[a:b], float(f_min[c]), float(df[c]), Nf=int(Nf[c]), threads=threads)
        res[int(c)] = peak(P)
    return res


# ---- Monte Carlo and surrogate inputs -----------------------------------------------

def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: four 32-bit counter words, two key words."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.empty(4, dtype=np.uint32)
    _lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def normals(seed, stream, n):
    """The first n N(0,1) deviates of counter stream `stream` (FP64)."""
    out = np.empty(int(n), dtype=np.float64)
    _lib().oracle_normals(int(seed) & (2**64 - 1), int(stream) & (2**64 - 1), int(n), _ptr(out))
    return out


def mc_maxpower(t, f_min, df, Nf, R, seed, stream_base=0, threads=0):
    """max Pn of R white-noise realizations (draws as the GPU's), one pattern."""
    res = np.empty(int(R))
    for r in range(int(R)):
        x = normals(seed, stream_base + r, len(t))
        res[r] = periodogram(t, x, f_min, df, Nf=Nf, threads=threads).max()
    return res


N_BANDS = 64


def band_limits(Nf):
    """[lo, hi) frequency-index ranges of the 64 log-spaced window bands."""
    Nf = int(Nf)
    out = []
    for b in range(N_BANDS):
        # edges round(Nf^(b/64)) - 1, the outer ones fixed at 0 and Nf
        lo = 0 if b == 0 else int(np.rint(np.exp(np.log(Nf) * b / N_BANDS))) - 1
        hi = Nf if b == N_BANDS - 1 else int(np.rint(np.exp(np.log(Nf) * (b + 1) / N_BANDS))) - 1
        lo = min(max(lo, 0), Nf - 1)
        hi = min(max(hi, lo + 1), Nf)
        out.append((lo, hi))
    return out


def window_features(t, f_min, df, Nf, threads=0):
    """The 68 surrogate inputs of one sorted pattern, from the FP64 window."""
    t = _f64(t)
    W = window(t, f_min, df, Nf, threads=threads)
    Nt = t.size
    f = [np.log10(W[lo:hi].mean() / Nt + 1e-30) for lo, hi in band_limits(Nf)]
    T = t.max() - t.min()
    d = np.diff(t)
    gap = d[d > 5.0 * T / (Nt - 1)].sum() / T
    return np.array(f + [np.log10(Nt), np.log10(T), gap, np.log10(Nf)])
