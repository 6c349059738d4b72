"""mi355lsp -- MI355X (gfx950) direct normalized Lomb-Scargle periodogram.

Thin ctypes binding over the C ABI of libmi355lsp.so (include/lsp.h); the
Python functions carry the C names and only marshal arguments: every step
of the computation runs in the library's HIP kernels.  Torch tensors supply
device memory and streams.  There is no CPU fallback: if the library is not
built, or no gfx950 device is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmi355lsp.so")

LSP_OK = 0
LSP_ERR_INVALID_ARG = -1
LSP_ERR_ZERO_VARIANCE = -2
LSP_ERR_NO_DEVICE = -3
LSP_ERR_HIP = -4
LSP_ERR_MODEL = -5
LSP_ERR_CAPTURE = -6
LSP_ERR_UNSUPPORTED = -7

LSP_PHASE_SPLIT = 0
LSP_PHASE_NAIVE = 1
LSP_PHASE_SPLIT32 = 2

LSP_TRIG_AUTO = 0
LSP_TRIG_DIRECT = 1
LSP_TRIG_RECUR = 2
LSP_TRIG_MFMA = 3

PHASES = {"split": LSP_PHASE_SPLIT, "naive": LSP_PHASE_NAIVE, "split32": LSP_PHASE_SPLIT32}
TRIGS = {"auto": LSP_TRIG_AUTO, "direct": LSP_TRIG_DIRECT, "recur": LSP_TRIG_RECUR, "mfma": LSP_TRIG_MFMA}


class LspError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: {lsp_status_string(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


LSP_SUM_AUTO = 0
LSP_SUM_KAHAN = 1
LSP_SUM_TWO = 2
SUMS = {"auto": LSP_SUM_AUTO, "kahan": LSP_SUM_KAHAN, "two": LSP_SUM_TWO}


class lsp_tile(ctypes.Structure):
    _fields_ = [("trig", ctypes.c_int32), ("m", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("splits", ctypes.c_int32),
                ("unroll", ctypes.c_int32), ("sum", ctypes.c_int32)]

    def as_dict(self):
        return {"trig": self.trig, "m": self.m, "waves": self.waves, "splits": self.splits,
                "unroll": self.unroll, "sum": self.sum}


class lsp_options(ctypes.Structure):
    _fields_ = [("phase", ctypes.c_int32), ("check", ctypes.c_int32), ("tile", lsp_tile)]


_lib = None

# symbol -> (restype, argtypes); the exported surface of include/lsp.h
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double
SIGNATURES = {
    "lsp_periodogram": (_I32, [_P, _P, _I64, _D, _D, _I64, _P, _P]),
    "lsp_periodogram_ex": (_I32, [_P, _P, _I64, _D, _D, _I64, _P, _P, ctypes.POINTER(lsp_options)]),
    "lsp_periodogram_noalloc": (_I32, [_P, _P, _I64, _D, _D, _I64, _P, _P]),
    "lsp_periodogram_batched": (_I32, [_P, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "lsp_mc_maxpower": (_I32, [_P, _P, _I32, _P, _P, _P, _I32, ctypes.c_uint64, ctypes.c_uint64, _P, _P]),
    "lsp_window_features": (_I32, [_P, _P, _I32, _P, _P, _P, _P, _P]),
    "lsp_normals": (_I32, [ctypes.c_uint64, ctypes.c_uint64, _I64, _P, _P]),
    "lsp_model_param_count": (_I64, []),
    "lsp_model_create": (_I32, [_I32, ctypes.c_uint64, ctypes.POINTER(_P)]),
    "lsp_model_destroy": (_I32, [_P]),
    "lsp_model_set_scalers": (_I32, [_P, _P, _P, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    "lsp_model_get_params": (_I32, [_P, _I32, _P, _I64]),
    "lsp_model_set_params": (_I32, [_P, _I32, _P, _I64]),
    "lsp_model_save": (_I32, [_P, ctypes.c_char_p, _I32]),
    "lsp_model_set_law_error": (_I32, [_P, ctypes.c_float, ctypes.c_float]),
    "lsp_model_load": (_I32, [ctypes.c_char_p, ctypes.POINTER(_P)]),
    "lsp_mlp_forward": (_I32, [_P, _P, _I32, _P, _P]),
    "lsp_mlp_grad": (_I32, [_P, _I32, _P, _P, _I32, _I32, _P, _P, _P]),
    "lsp_mlp_adam_step": (_I32, [_P, _I32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]),
    "lsp_mlp_gemm_nt": (_I32, [_P, _P, _P, _I32, _I32, _I32, _P]),
    "lsp_fap_surrogate": (_I32, [_P, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _P, ctypes.c_float, _I32,
                                 ctypes.c_uint64, _P]),
    "lsp_autotune": (_I32, [_I64, _I64, _I32, _P, ctypes.POINTER(lsp_tile), ctypes.POINTER(_D)]),
    "lsp_tune_lookup": (_I32, [_I64, _I64, _I32, ctypes.POINTER(lsp_tile)]),
    "lsp_list_tiles": (_I32, [_I32, ctypes.POINTER(lsp_tile), _I32]),
    "lsp_gls": (_I32, [_P, _P, _P, _I64, _D, _D, _I64, _P, _I32, _I32, _P]),
    "lsp_set_batched_form": (_I32, [_I32]),
    "lsp_periodogram_fast": (_I32, [_P, _P, _I64, _D, _D, _I64, _I32, _P, _P]),
    "lsp_multiharmonic": (_I32, [_P, _P, _P, _I64, _I32, _D, _D, _I64, _P, _I32, _I32, _P]),
    "lsp_get_batched_form": (_I32, []),
    "lsp_tune_cache_save": (_I32, [ctypes.c_char_p]),
    "lsp_tune_cache_load": (_I32, [ctypes.c_char_p]),
    "lsp_microbench": (_I32, [_I32, _I32, _I32, _P, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "lsp_probe_sincos": (_I32, [_P, _I64, _P, _P, _P]),
    "lsp_probe_phase": (_I32, [_P, _P, _I64, _D, _I32, _P, _P]),
    "lsp_probe_recurrence": (_I32, [_P, _I64, _D, _D, _D, _I32, _P, _P, _P]),
    "lsp_probe_cmac": (_I32, [_P, _P, _I32, _P, _P]),
    "lsp_probe_cpair": (_I32, [_P, _P, _I32, _P, _P, _P]),
    "lsp_profile_enable": (_I32, [_I32]),
    "lsp_profile_read": (_I32, [ctypes.POINTER(_D), ctypes.POINTER(_I64), ctypes.c_char_p, _I32]),
    "lsp_profile_read_calls": (_I32, [_P, _I64, ctypes.POINTER(_I64)]),
    "lsp_grid_paper": (_I32, [_D, _D, _I64, _D, _D, _I32, ctypes.POINTER(_D), ctypes.POINTER(_D),
                              ctypes.POINTER(_I64)]),
    "lsp_fap_analytic": (_D, [_D, _I64, _I64]),
    "lsp_status_string": (ctypes.c_char_p, [_I32]),
    "lsp_last_error": (ctypes.c_char_p, []),
    "lsp_version": (ctypes.c_char_p, []),
    "lsp_device_count": (_I32, []),
}


def load_library(path):
    """A libmi355lsp build at `path` with the C signatures declared (e.g. the
    LDS-poisoning debug build, debug/libmi355lsp_poison.so)."""
    # torch first, where it is installed: its HIP runtime is then the one the
    # library binds to (both are libamdhip64.so.7), so tensors and the
    # library's calls share one runtime whichever the caller touched first
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def lib():
    """The loaded libmi355lsp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "(or python paper_1007_1658_amd/build.py)")
        _lib = load_library(LIB_PATH)
    return _lib


def lsp_status_string(status: int) -> str:
    return lib().lsp_status_string(int(status)).decode()


def lsp_last_error() -> str:
    return lib().lsp_last_error().decode()


def lsp_version() -> str:
    return lib().lsp_version().decode()


def lsp_device_count() -> int:
    return int(lib().lsp_device_count())


def _check(status: int, where: str):
    if status != LSP_OK:
        raise LspError(status, where, lsp_last_error())


# ---- host-only helpers --------------------------------------------------------------

def lsp_grid_paper(t_min: float, t_max: float, Nt: int, F_over: float = 4.0, F_high: float = 1.0,
                   round_to: int = 1):
    """(f_min, df, Nf) of the paper's grid, Eqs. (9)-(11)."""
    f_min, df, nf = _D(), _D(), _I64()
    _check(lib().lsp_grid_paper(float(t_min), float(t_max), int(Nt), float(F_over), float(F_high),
                                int(round_to), ctypes.byref(f_min), ctypes.byref(df), ctypes.byref(nf)),
           "lsp_grid_paper")
    return f_min.value, df.value, int(nf.value)


def lsp_fap_analytic(Pn: float, Nt: int, Nf: int) -> float:
    """Eq. (3) false-alarm probability."""
    return float(lib().lsp_fap_analytic(float(Pn), int(Nt), int(Nf)))


# ---- device entry points --------------------------------------------------------------

def _torch():
    import torch
    return torch


def _dev_tensor(a, dtype, name):
    torch = _torch()
    if not isinstance(a, torch.Tensor) or not a.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if a.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {a.dtype}")
    if not a.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return a


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(a):
    return ctypes.c_void_p(a.data_ptr()) if a is not None else None


def lsp_periodogram(t, x, f_min: float, df: float, Nf: int, Pn=None, stream=None):
    """Pn[k] = Pn(f_min + k df), k < Nf, for device t (float64) and x (float32)."""
    return lsp_periodogram_ex(t, x, f_min, df, Nf, Pn=Pn, stream=stream)


# size of the fixed per-GPU scratch array of lsp_periodogram_noalloc (include/lsp.h)
LSP_NOALLOC_SCRATCH_BYTES = 96 * 1024 * 1024


def lsp_periodogram_noalloc(t, x, f_min: float, df: float, Nf: int, Pn, stream=None):
    """lsp_periodogram on the library's fixed scratch array: no device memory is
    allocated by the library (Pn, the output, is the caller's)."""
    torch = _torch()
    _dev_tensor(t, torch.float64, "t")
    _dev_tensor(x, torch.float32, "x")
    _dev_tensor(Pn, torch.float32, "Pn")
    if t.ndim != 1 or x.shape != t.shape:
        raise ValueError("t and x must be 1-D and of equal length")
    if Pn.numel() < int(Nf):
        raise ValueError("Pn is shorter than Nf")
    with torch.cuda.device(t.device):
        st = lib().lsp_periodogram_noalloc(_ptr(t), _ptr(x), t.numel(), float(f_min), float(df), int(Nf),
                                           _ptr(Pn), _stream_ptr(stream))
    _check(st, "lsp_periodogram_noalloc")
    return Pn


def lsp_multiharmonic(t, y, K: int, f_min: float, df: float, Nf: int, w=None, p=None, waves=0, splits=0,
                      stream=None):
    """Multi-harmonic periodogram p_K[Nf] (device float32), K in 1..4."""
    torch = _torch()
    _dev_tensor(t, torch.float64, "t")
    _dev_tensor(y, torch.float32, "y")
    if t.ndim != 1 or y.shape != t.shape:
        raise ValueError("t and y must be 1-D and of equal length")
    if w is not None:
        _dev_tensor(w, torch.float32, "w")
        if w.shape != t.shape:
            raise ValueError("w must match t")
    if p is None:
        p = torch.empty(int(Nf), dtype=torch.float32, device=t.device)
    _dev_tensor(p, torch.float32, "p")
    if p.numel() < int(Nf):
        raise ValueError("p is shorter than Nf")
    _check(lib().lsp_multiharmonic(_ptr(t), _ptr(y), _ptr(w), t.numel(), int(K), float(f_min), float(df), int(Nf),
                                   _ptr(p), int(waves), int(splits), _stream_ptr(stream)), "lsp_multiharmonic")
    return p


def lsp_set_batched_form(trig):
    """Kernel form of the batched / Monte-Carlo / window paths: "mfma" or "recur"."""
    _check(lib().lsp_set_batched_form(TRIGS[trig] if isinstance(trig, str) else int(trig)), "lsp_set_batched_form")


def lsp_get_batched_form() -> str:
    v = int(lib().lsp_get_batched_form())
    return {LSP_TRIG_RECUR: "recur", LSP_TRIG_MFMA: "mfma"}.get(v, str(v))


def lsp_periodogram_fast(t, x, f_min: float, df: float, Nf: int, macc: int = 4, Pn=None, stream=None):
    """Approximate Pn[Nf] by extirpolation + FFT (f_min a whole multiple of df)."""
    torch = _torch()
    _dev_tensor(t, torch.float64, "t")
    _dev_tensor(x, torch.float32, "x")
    if t.ndim != 1 or x.shape != t.shape:
        raise ValueError("t and x must be 1-D and of equal length")
    if Pn is None:
        Pn = torch.empty(int(Nf), dtype=torch.float32, device=t.device)
    _dev_tensor(Pn, torch.float32, "Pn")
    if Pn.numel() < int(Nf):
        raise ValueError("Pn is shorter than Nf")
    _check(lib().lsp_periodogram_fast(_ptr(t), _ptr(x), t.numel(), float(f_min), float(df), int(Nf), int(macc),
                                      _ptr(Pn), _stream_ptr(stream)), "lsp_periodogram_fast")
    return Pn


def lsp_gls(t, y, f_min: float, df: float, Nf: int, w=None, p=None, waves=0, splits=0, stream=None):
    """Generalized (floating-mean, weighted) periodogram p[Nf] (device float32)."""
    torch = _torch()
    _dev_tensor(t, torch.float64, "t")
    _dev_tensor(y, torch.float32, "y")
    if t.ndim != 1 or y.shape != t.shape:
        raise ValueError("t and y must be 1-D and of equal length")
    if w is not None:
        _dev_tensor(w, torch.float32, "w")
        if w.shape != t.shape:
            raise ValueError("w must match t")
    if p is None:
        p = torch.empty(int(Nf), dtype=torch.float32, device=t.device)
    _dev_tensor(p, torch.float32, "p")
    if p.numel() < int(Nf):
        raise ValueError("p is shorter than Nf")
    _check(lib().lsp_gls(_ptr(t), _ptr(y), _ptr(w), t.numel(), float(f_min), float(df), int(Nf), _ptr(p),
                         int(waves), int(splits), _stream_ptr(stream)), "lsp_gls")
    return p


def lsp_periodogram_ex(t, x, f_min: float, df: float, Nf: int, Pn=None, stream=None,
                       phase="split", trig="auto", m=0, waves=0, splits=0, unroll=0, sum="auto",
                       check=False):
    torch = _torch()
    _dev_tensor(t, torch.float64, "t")
    _dev_tensor(x, torch.float32, "x")
    if t.ndim != 1 or x.shape != t.shape:
        raise ValueError("t and x must be 1-D and of equal length")
    if Pn is None:
        Pn = torch.empty(int(Nf), dtype=torch.float32, device=t.device)
    _dev_tensor(Pn, torch.float32, "Pn")
    if Pn.numel() < int(Nf):
        raise ValueError("Pn is shorter than Nf")
    opt = lsp_options()
    opt.phase = PHASES[phase] if isinstance(phase, str) else int(phase)
    opt.check = 1 if check else 0
    opt.tile.trig = TRIGS[trig] if isinstance(trig, str) else int(trig)
    opt.tile.m, opt.tile.waves, opt.tile.splits = int(m), int(waves), int(splits)
    opt.tile.unroll = int(unroll)
    opt.tile.sum = SUMS[sum] if isinstance(sum, str) else int(sum)
    with torch.cuda.device(t.device):
        st = lib().lsp_periodogram_ex(_ptr(t), _ptr(x), t.numel(), float(f_min), float(df), int(Nf),
                                      _ptr(Pn), _stream_ptr(stream), ctypes.byref(opt))
    _check(st, "lsp_periodogram_ex")
    return Pn


def lsp_periodogram_batched(t, x, off, f_min, df, Nf, want_pn=False, want_times=False, stream=None,
                            out=None):
    """Per-curve (pmax, kbest, fbest[, Pn CSR][, t_ns]) of a CSR batch in one persistent launch.

    t, x: device tensors (float64 / float32) holding all curves back to back.
    off, f_min, df, Nf: host arrays (numpy) describing the batch shape.
    out: optional dict of preallocated device outputs (reused across calls so
    that the cached hipGraph is replayed).
    """
    torch = _torch()
    _dev_tensor(t, torch.float64, "t")
    _dev_tensor(x, torch.float32, "x")
    off = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    f_min = np.ascontiguousarray(np.asarray(f_min, dtype=np.float64))
    df = np.ascontiguousarray(np.asarray(df, dtype=np.float64))
    Nf = np.ascontiguousarray(np.asarray(Nf, dtype=np.int64))
    n = off.size - 1
    if n < 1 or f_min.size != n or df.size != n or Nf.size != n:
        raise ValueError("batch arrays disagree in length")
    if int(off[-1]) != t.numel() or x.numel() != t.numel():
        raise ValueError("off[-1] must equal the number of samples")
    dev = t.device
    if out is None:
        out = {}
    if "pmax" not in out:
        out["pmax"] = torch.empty(n, dtype=torch.float32, device=dev)
        out["kbest"] = torch.empty(n, dtype=torch.int64, device=dev)
        out["fbest"] = torch.empty(n, dtype=torch.float64, device=dev)
    if want_pn and "Pn" not in out:
        out["Pn"] = torch.empty(int(Nf.sum()), dtype=torch.float32, device=dev)
    if want_times and "t_ns" not in out:
        out["t_ns"] = torch.empty(2 * n, dtype=torch.int64, device=dev)
    hp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    with torch.cuda.device(dev):
        st = lib().lsp_periodogram_batched(
            _ptr(t), _ptr(x), hp(off), n, hp(f_min), hp(df), hp(Nf),
            _ptr(out.get("Pn")), _ptr(out["pmax"]), _ptr(out["kbest"]), _ptr(out["fbest"]),
            _ptr(out.get("t_ns")), _stream_ptr(stream))
    _check(st, "lsp_periodogram_batched")
    return out


N_FEATURES = 68


def _host_shape(off, f_min, df, Nf):
    off = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    f_min = np.ascontiguousarray(np.asarray(f_min, dtype=np.float64))
    df = np.ascontiguousarray(np.asarray(df, dtype=np.float64))
    Nf = np.ascontiguousarray(np.asarray(Nf, dtype=np.int64))
    n = off.size - 1
    if n < 1 or f_min.size != n or df.size != n or Nf.size != n:
        raise ValueError("pattern arrays disagree in length")
    return off, f_min, df, Nf, n


def lsp_mc_maxpower(t, off, f_min, df, Nf, R: int, seed: int, stream_base: int = 0, out=None, stream=None):
    """max Pn of R white-noise realizations on each pattern: device float32 [n_pat, R]."""
    torch = _torch()
    _dev_tensor(t, torch.float64, "t")
    off, f_min, df, Nf, n = _host_shape(off, f_min, df, Nf)
    if int(off[-1]) != t.numel():
        raise ValueError("off[-1] must equal the number of samples")
    if out is None:
        out = torch.empty((n, int(R)), dtype=torch.float32, device=t.device)
    _dev_tensor(out, torch.float32, "out")
    hp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    with torch.cuda.device(t.device):
        st = lib().lsp_mc_maxpower(_ptr(t), hp(off), n, hp(f_min), hp(df), hp(Nf), int(R),
                                   int(seed) & (2**64 - 1), int(stream_base) & (2**64 - 1), _ptr(out),
                                   _stream_ptr(stream))
    _check(st, "lsp_mc_maxpower")
    return out


def lsp_window_features(t, off, f_min, df, Nf, out=None, stream=None):
    """Spectral-window features of each pattern: device float32 [n_pat, 68]."""
    torch = _torch()
    _dev_tensor(t, torch.float64, "t")
    off, f_min, df, Nf, n = _host_shape(off, f_min, df, Nf)
    if int(off[-1]) != t.numel():
        raise ValueError("off[-1] must equal the number of samples")
    if out is None:
        out = torch.empty((n, N_FEATURES), dtype=torch.float32, device=t.device)
    _dev_tensor(out, torch.float32, "out")
    hp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    with torch.cuda.device(t.device):
        st = lib().lsp_window_features(_ptr(t), hp(off), n, hp(f_min), hp(df), hp(Nf), _ptr(out),
                                       _stream_ptr(stream))
    _check(st, "lsp_window_features")
    return out


def lsp_normals(seed: int, stream_id: int, n: int, device="cuda", stream=None):
    """The first n deviates of counter stream stream_id (as drawn by lsp_mc_maxpower)."""
    torch = _torch()
    out = torch.empty(int(n), dtype=torch.float32, device=device)
    st = lib().lsp_normals(int(seed) & (2**64 - 1), int(stream_id) & (2**64 - 1), int(n), _ptr(out),
                           _stream_ptr(stream))
    _check(st, "lsp_normals")
    return out


def lsp_autotune(Nt: int, Nf: int, phase="split", stream=None):
    """(tile dict, best ms) for (Nt, Nf); also stored in the library's tuner cache."""
    tile = lsp_tile()
    ms = _D()
    ph = PHASES[phase] if isinstance(phase, str) else int(phase)
    _check(lib().lsp_autotune(int(Nt), int(Nf), ph, _stream_ptr(stream), ctypes.byref(tile),
                              ctypes.byref(ms)), "lsp_autotune")
    return tile.as_dict(), ms.value


def lsp_list_tiles(phase="split"):
    """The launch shapes built into the library for a phase mode (list of dicts)."""
    ph = PHASES[phase] if isinstance(phase, str) else int(phase)
    n = lib().lsp_list_tiles(ph, None, 0)
    if n < 0:
        raise LspError(LSP_ERR_INVALID_ARG, "lsp_list_tiles")
    arr = (lsp_tile * max(n, 1))()
    lib().lsp_list_tiles(ph, arr, n)
    return [arr[i].as_dict() for i in range(n)]


def lsp_tune_lookup(Nt: int, Nf: int, phase="split"):
    """The cached launch shape for (Nt, Nf, phase) as a dict, or None."""
    tile = lsp_tile()
    ph = PHASES[phase] if isinstance(phase, str) else int(phase)
    st = lib().lsp_tune_lookup(int(Nt), int(Nf), ph, ctypes.byref(tile))
    if st == LSP_ERR_INVALID_ARG:
        return None
    _check(st, "lsp_tune_lookup")
    return tile.as_dict()


TUNE_CACHE = os.path.join(_HERE, "tune_gfx950.json")


def lsp_tune_cache_save(path=None):
    _check(lib().lsp_tune_cache_save(path.encode() if path else None), "lsp_tune_cache_save")


def lsp_tune_cache_load(path=None):
    _check(lib().lsp_tune_cache_load(path.encode() if path else None), "lsp_tune_cache_load")


def lsp_microbench(kind: int, waves_per_simd: int = 2, iters: int = 4096, stream=None):
    """(lane-ops/s, ms) of one instruction class: 0 FP32 FMA, 1 FP64 FMA, 2 sin+cos, 3 FP64 phase;
    4-7 MFMA FLOP/s with 0, 4, 8, 16 FP32 FMAs per MFMA; 8 the 16-FMA stream alone (FMA/s)."""
    ops, ms = _D(), _D()
    _check(lib().lsp_microbench(int(kind), int(waves_per_simd), int(iters), _stream_ptr(stream),
                                ctypes.byref(ops), ctypes.byref(ms)), "lsp_microbench")
    return ops.value, ms.value


def lsp_probe_sincos(r, stream=None):
    """(sin, cos)(2 pi r) by the hardware instructions the kernels use; r: device float32."""
    torch = _torch()
    _dev_tensor(r, torch.float32, "r")
    s, c = torch.empty_like(r), torch.empty_like(r)
    with torch.cuda.device(r.device):
        _check(lib().lsp_probe_sincos(_ptr(r), r.numel(), _ptr(s), _ptr(c), _stream_ptr(stream)),
               "lsp_probe_sincos")
    return s, c


def lsp_probe_phase(t, f, t_ref: float, phase="split", stream=None):
    """Reduced phase of f[i] at t[i] in the given phase mode (device float64 t, f -> float32)."""
    torch = _torch()
    _dev_tensor(t, torch.float64, "t")
    _dev_tensor(f, torch.float64, "f")
    if f.numel() != t.numel():
        raise ValueError("t and f differ in length")
    phi = torch.empty(t.numel(), dtype=torch.float32, device=t.device)
    with torch.cuda.device(t.device):
        _check(lib().lsp_probe_phase(_ptr(t), _ptr(f), t.numel(), float(t_ref), PHASES[phase], _ptr(phi),
                                     _stream_ptr(stream)), "lsp_probe_phase")
    return phi


def lsp_probe_recurrence(t, t_ref: float, f0: float, step_df: float, M: int, stream=None):
    """(cos, sin)(2 pi (f0 + m step_df)(t - t_ref)), m < M, as the recurrence form makes them:
    two device float32 tensors [n, M]."""
    torch = _torch()
    _dev_tensor(t, torch.float64, "t")
    c = torch.empty((t.numel(), int(M)), dtype=torch.float32, device=t.device)
    s = torch.empty_like(c)
    with torch.cuda.device(t.device):
        _check(lib().lsp_probe_recurrence(_ptr(t), t.numel(), float(t_ref), float(f0), float(step_df), int(M),
                                          _ptr(c), _ptr(s), _stream_ptr(stream)), "lsp_probe_recurrence")
    return c, s


def lsp_probe_cmac(L, R, stream=None):
    """P[a][b] = sum_j L[a][j] R[b][j] by the matrix-core form's complex product
    (device complex64 L, R of shape [32, K], K a multiple of 16): complex64 [32, 32]."""
    torch = _torch()
    _dev_tensor(L, torch.complex64, "L")
    _dev_tensor(R, torch.complex64, "R")
    if L.ndim != 2 or L.shape[0] != 32 or R.shape != L.shape:
        raise ValueError("L and R must both be [32, K]")
    P = torch.empty((32, 32), dtype=torch.complex64, device=L.device)
    _check(lib().lsp_probe_cmac(_ptr(L), _ptr(R), int(L.shape[1]), _ptr(P), _stream_ptr(stream)),
           "lsp_probe_cmac")
    return P


def lsp_probe_cpair(L, R, stream=None):
    """(sum_j L[a][j] R[b][j], sum_j L[a][j] conj(R[b][j])) by the conjugate-pair
    products (device complex64 L, R of shape [32, K], K a multiple of 16):
    two complex64 [32, 32]."""
    torch = _torch()
    _dev_tensor(L, torch.complex64, "L")
    _dev_tensor(R, torch.complex64, "R")
    if L.ndim != 2 or L.shape[0] != 32 or R.shape != L.shape:
        raise ValueError("L and R must both be [32, K]")
    Pp = torch.empty((32, 32), dtype=torch.complex64, device=L.device)
    Pm = torch.empty((32, 32), dtype=torch.complex64, device=L.device)
    _check(lib().lsp_probe_cpair(_ptr(L), _ptr(R), int(L.shape[1]), _ptr(Pp), _ptr(Pm), _stream_ptr(stream)),
           "lsp_probe_cpair")
    return Pp, Pm


PROFILE_KERNEL = 1   # events on the main kernel's launches
PROFILE_CALLS = 2    # events on each single-curve call's first and last kernels


def lsp_profile_enable(on=True):
    """on: False/0 off, True = PROFILE_KERNEL, or a mask of PROFILE_KERNEL | PROFILE_CALLS."""
    mode = PROFILE_KERNEL if on is True else int(on)
    _check(lib().lsp_profile_enable(mode), "lsp_profile_enable")


def lsp_profile_read():
    """(total ms, launches, kernel name) of the main kernel since lsp_profile_enable."""
    tot, n = _D(), _I64()
    buf = ctypes.create_string_buffer(256)
    _check(lib().lsp_profile_read(ctypes.byref(tot), ctypes.byref(n), buf, 256), "lsp_profile_read")
    return tot.value, int(n.value), buf.value.decode()


def lsp_profile_read_calls():
    """Device ms of each single-curve call since lsp_profile_enable (first kernel's start to last kernel's end)."""
    n = _I64()
    _check(lib().lsp_profile_read_calls(None, 0, ctypes.byref(n)), "lsp_profile_read_calls")
    out = np.zeros(int(n.value), dtype=np.float64)
    if out.size:
        _check(lib().lsp_profile_read_calls(out.ctypes.data, out.size, ctypes.byref(n)), "lsp_profile_read_calls")
    return out


# ---- false-alarm surrogate ------------------------------------------------------------

N_QUANTILES = 9
TAU = (0.5, 0.75, 0.9, 0.95, 0.975, 0.99, 0.995, 0.998, 0.999)


def lsp_model_param_count() -> int:
    return int(lib().lsp_model_param_count())


def lsp_mlp_gemm_nt(A, B, out=None, stream=None):
    """C = A B^T for device bfloat16 A [M, K], B [N, K] (multiples of 32); returns float32 C."""
    torch = _torch()
    _dev_tensor(A, torch.bfloat16, "A")
    _dev_tensor(B, torch.bfloat16, "B")
    M, K = A.shape
    N = B.shape[0]
    if out is None:
        out = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(lib().lsp_mlp_gemm_nt(_ptr(A), _ptr(B), _ptr(out), M, N, K, _stream_ptr(stream)), "lsp_mlp_gemm_nt")
    return out


class Model:
    """An ensemble of surrogate networks living on the current device (lsp_model)."""

    def __init__(self, members: int = 4, seed: int = 0, path: str = None):
        h = ctypes.c_void_p()
        if path is not None:
            _check(lib().lsp_model_load(path.encode(), ctypes.byref(h)), "lsp_model_load")
        else:
            _check(lib().lsp_model_create(int(members), int(seed) & (2**64 - 1), ctypes.byref(h)),
                   "lsp_model_create")
        self.h = h
        self._members = None

    def close(self):
        if self.h:
            lib().lsp_model_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    @property
    def members(self) -> int:
        if self._members is None:
            n = 0
            buf = np.empty(lsp_model_param_count(), dtype=np.float32)
            while lib().lsp_model_get_params(self.h, n, buf.ctypes.data_as(ctypes.c_void_p), buf.size) == LSP_OK:
                n += 1
            self._members = n
        return self._members

    def get_params(self, member: int) -> np.ndarray:
        out = np.empty(lsp_model_param_count(), dtype=np.float32)
        _check(lib().lsp_model_get_params(self.h, int(member), out.ctypes.data_as(ctypes.c_void_p), out.size),
               "lsp_model_get_params")
        return out

    def set_params(self, member: int, params):
        a = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        _check(lib().lsp_model_set_params(self.h, int(member), a.ctypes.data_as(ctypes.c_void_p), a.size),
               "lsp_model_set_params")

    def set_scalers(self, feat_mean, feat_std, feat_zmax: float, q_mu: float, q_sigma: float):
        m = np.ascontiguousarray(np.asarray(feat_mean, dtype=np.float32))
        sd = np.ascontiguousarray(np.asarray(feat_std, dtype=np.float32))
        _check(lib().lsp_model_set_scalers(self.h, m.ctypes.data_as(ctypes.c_void_p),
                                           sd.ctypes.data_as(ctypes.c_void_p), float(feat_zmax), float(q_mu),
                                           float(q_sigma)), "lsp_model_set_scalers")

    def set_law_error(self, err_m: float, err_beta: float):
        """Calibrated standard errors of the law's location and scale (lsp_model_set_law_error)."""
        _check(lib().lsp_model_set_law_error(self.h, float(err_m), float(err_beta)), "lsp_model_set_law_error")

    def save(self, path: str, with_optimizer: bool = False):
        _check(lib().lsp_model_save(self.h, path.encode(), 1 if with_optimizer else 0), "lsp_model_save")

    def forward(self, feat, stream=None):
        """Quantiles [members, B, 9] (device float32) of device features [B, 68]."""
        torch = _torch()
        _dev_tensor(feat, torch.float32, "feat")
        B = feat.shape[0]
        q = torch.empty((self.members, B, N_QUANTILES), dtype=torch.float32, device=feat.device)
        _check(lib().lsp_mlp_forward(self.h, _ptr(feat), B, _ptr(q), _stream_ptr(stream)), "lsp_mlp_forward")
        return q

    def grad(self, member: int, feat, samples, want_grad=True, stream=None):
        """(flat gradient or None, loss) of one member on a minibatch (device tensors)."""
        torch = _torch()
        _dev_tensor(feat, torch.float32, "feat")
        _dev_tensor(samples, torch.float32, "samples")
        B, R = samples.shape
        g = torch.empty(lsp_model_param_count(), dtype=torch.float32, device=feat.device) if want_grad else None
        loss = torch.empty(1, dtype=torch.float32, device=feat.device)
        _check(lib().lsp_mlp_grad(self.h, int(member), _ptr(feat), _ptr(samples), int(R), int(B), _ptr(g),
                                  _ptr(loss), _stream_ptr(stream)), "lsp_mlp_grad")
        return g, loss

    def adam_step(self, member: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(lib().lsp_mlp_adam_step(self.h, int(member), float(lr), float(beta1), float(beta2), float(eps),
                                       _stream_ptr(stream)), "lsp_mlp_adam_step")

    def fap(self, t, off, f_min, df, Nf, p_obs, max_err=0.005, mc_realizations=10000, seed=0, stream=None):
        """(fap, err, used_mc) device tensors for observed maxima p_obs [n_pat]: the
        mean FAP, its 99 % error bound, and where Monte Carlo answered instead
        (the bound above max_err, or features out of range)."""
        torch = _torch()
        _dev_tensor(t, torch.float64, "t")
        _dev_tensor(p_obs, torch.float32, "p_obs")
        off, f_min, df, Nf, n = _host_shape(off, f_min, df, Nf)
        fap = torch.empty(n, dtype=torch.float32, device=t.device)
        err = torch.empty(n, dtype=torch.float32, device=t.device)
        used = torch.zeros(n, dtype=torch.int32, device=t.device)
        hp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(lib().lsp_fap_surrogate(self.h, _ptr(t), hp(off), n, hp(f_min), hp(df), hp(Nf), _ptr(p_obs),
                                       _ptr(fap), _ptr(err), _ptr(used), float(max_err), int(mc_realizations),
                                       int(seed) & (2**64 - 1), _stream_ptr(stream)), "lsp_fap_surrogate")
        return fap, err, used
