"""Host-side checks of the C ABI (CPU only: no kernel is launched)."""
import ctypes
import math
import re
import os

import numpy as np
import pytest
from scipy import stats

import oracle
import paper_1007_1658_amd as lsp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lsp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lsp_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "lsp_periodogram" in names and "lsp_periodogram_batched" in names
    L = lsp.lib()
    for n in names:
        assert hasattr(L, n), n
    # and the binding covers the same surface
    assert set(names) <= set(lsp.SIGNATURES)


def test_status_strings():
    for s in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lsp.lsp_status_string(s)
    assert lsp.lsp_version().startswith("mi355lsp")


def test_grid_helper_reproduces_paper_nf():
    # CoRoT series of Section 5.2: Nt = 382,003; with oversampling 4, high factor 2 and the
    # kernel's 256-thread blocks the printed Nf = 1,528,064 follows.
    f_min, df, nf = lsp.lsp_grid_paper(0.0, 150.0, 382003, 4.0, 2.0, 256)
    assert nf == 1528064
    assert df == pytest.approx(1.0 / 600.0)
    assert f_min == df
    # no rounding: Nf = F_high F_over Nt / 2 exactly (Eq. (11)), c0 grid
    f_min, df, nf = lsp.lsp_grid_paper(0.3, 99.8, 1000, 4.0, 1.0, 1)
    assert nf == 2000 and df == pytest.approx(1.0 / (4 * 99.5))
    # odd products round up
    assert lsp.lsp_grid_paper(0, 1, 1001, 1.0, 1.0, 1)[2] == 501


@pytest.mark.parametrize("bad", [
    (1.0, 1.0, 10, 4, 1, 1), (0, 1, 1, 4, 1, 1), (0, 1, 10, 0, 1, 1), (0, 1, 10, 4, -1, 1),
    (0, 1, 10, 4, 1, 0), (0, float("inf"), 10, 4, 1, 1),
])
def test_grid_helper_rejects(bad):
    with pytest.raises(lsp.LspError) as ei:
        lsp.lsp_grid_paper(*bad)
    assert ei.value.status == lsp.LSP_ERR_INVALID_ARG


def test_fap_analytic_against_oracle_and_beta():
    for Nt in (4, 10, 1000, 65536):
        for Nf in (1, 2000, 131072):
            for P in np.linspace(0, Nt / 2, 9):
                a = lsp.lsp_fap_analytic(P, Nt, Nf)
                b = oracle.fap(P, Nt, Nf)
                assert a == pytest.approx(b, rel=1e-12, abs=1e-300)
    assert lsp.lsp_fap_analytic(2.0, 100, 1) == pytest.approx(stats.beta(1, 48.5).sf(0.04), rel=1e-10)
    assert math.isnan(lsp.lsp_fap_analytic(1.0, 3, 5))
    assert math.isnan(lsp.lsp_fap_analytic(-1.0, 30, 5))
    assert math.isnan(lsp.lsp_fap_analytic(16.0, 30, 5))


def test_validation_happens_before_any_gpu_work():
    L = lsp.lib()
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    cases = [
        (null, fake, 10, 0.1, 0.1, 10, fake),     # null t
        (fake, fake, 1, 0.1, 0.1, 10, fake),      # Nt < 2
        (fake, fake, 10, 0.1, 0.0, 10, fake),     # df = 0
        (fake, fake, 10, -0.1, 0.1, 10, fake),    # f_min < 0
        (fake, fake, 10, 0.1, 0.1, 0, fake),      # Nf = 0
        (fake, fake, 10, float("nan"), 0.1, 10, fake),
        (fake, fake, 10, 0.1, float("inf"), 10, fake),
        (fake, fake, 10, 0.1, 0.1, 10, null),     # null Pn
    ]
    for c in cases:
        assert L.lsp_periodogram(*c, null) == lsp.LSP_ERR_INVALID_ARG
    # an unknown phase mode is rejected too
    opt = lsp.lsp_options()
    opt.phase = 9
    assert L.lsp_periodogram_ex(fake, fake, 10, 0.1, 0.1, 10, fake, null, ctypes.byref(opt)) == \
        lsp.LSP_ERR_INVALID_ARG
    opt.phase = lsp.LSP_PHASE_NAIVE
    opt.tile.trig = lsp.LSP_TRIG_RECUR
    assert L.lsp_periodogram_ex(fake, fake, 10, 0.1, 0.1, 10, fake, null, ctypes.byref(opt)) == \
        lsp.LSP_ERR_UNSUPPORTED


def test_matrix_core_probe_validation_on_host():
    L = lsp.lib()
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(16)
    for args in ((null, fake, 16, fake), (fake, fake, 8, fake), (fake, fake, 24, fake), (fake, fake, 8192, fake),
                 (fake, fake, 16, null)):
        assert L.lsp_probe_cmac(*args, null) == lsp.LSP_ERR_INVALID_ARG, args
    for args in ((null, fake, 16, fake, fake), (fake, fake, 8, fake, fake), (fake, fake, 16, fake, null),
                 (fake, fake, 8192, fake, fake)):
        assert L.lsp_probe_cpair(*args, null) == lsp.LSP_ERR_INVALID_ARG, args


def test_generalized_periodogram_validation_on_host():
    L = lsp.lib()
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(16)
    cases = [
        (null, fake, null, 10, 0.1, 0.1, 10, fake, 0, 0),   # null t
        (fake, null, null, 10, 0.1, 0.1, 10, fake, 0, 0),   # null y
        (fake, fake, null, 2, 0.1, 0.1, 10, fake, 0, 0),    # Nt < 3
        (fake, fake, null, 10, 0.1, 0.0, 10, fake, 0, 0),   # df = 0
        (fake, fake, null, 10, 0.1, 0.1, 0, fake, 0, 0),    # Nf = 0
        (fake, fake, null, 10, 0.1, 0.1, 10, null, 0, 0),   # null p
        (fake, fake, null, 10, 0.1, 0.1, 10, fake, 3, 0),   # waves = 3
        (fake, fake, null, 10, 0.1, 0.1, 10, fake, 4, -1),  # negative splits
    ]
    for c in cases:
        assert L.lsp_gls(*c, null) == lsp.LSP_ERR_INVALID_ARG, c
    # 8-wave workgroups: the generalized periodogram only (K = 1), not K = 2
    assert L.lsp_multiharmonic(fake, fake, null, 10, 2, 0.1, 0.1, 10, fake, 8, 0, null) == lsp.LSP_ERR_INVALID_ARG
    # K beyond what is built; Nt below 2K + 1 for K = 4
    assert L.lsp_multiharmonic(fake, fake, null, 20, 5, 0.1, 0.1, 10, fake, 0, 0, null) == lsp.LSP_ERR_UNSUPPORTED
    assert L.lsp_multiharmonic(fake, fake, null, 8, 4, 0.1, 0.1, 10, fake, 0, 0, null) == lsp.LSP_ERR_INVALID_ARG


def test_batched_validation_on_host():
    L = lsp.lib()
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(16)
    hp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    off = np.array([0, 5, 6], dtype=np.int64)      # second curve has Nt = 1
    fm = np.array([0.1, 0.1])
    df = np.array([0.1, 0.1])
    nf = np.array([10, 10], dtype=np.int64)
    assert L.lsp_periodogram_batched(fake, fake, hp(off), 2, hp(fm), hp(df), hp(nf), null, fake, null, null,
                                     null, null) == lsp.LSP_ERR_INVALID_ARG
    off = np.array([1, 5, 9], dtype=np.int64)      # off[0] != 0
    assert L.lsp_periodogram_batched(fake, fake, hp(off), 2, hp(fm), hp(df), hp(nf), null, fake, null, null,
                                     null, null) == lsp.LSP_ERR_INVALID_ARG


def test_no_device_reported_without_gpu():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    assert lsp.lsp_device_count() == 0
    L = lsp.lib()
    fake = ctypes.c_void_p(16)
    st = L.lsp_periodogram(fake, fake, 10, 0.1, 0.1, 10, fake, ctypes.c_void_p(0))
    assert st == lsp.LSP_ERR_NO_DEVICE


def test_batched_form_switch_on_host():
    L = lsp.lib()
    assert L.lsp_set_batched_form(7) == lsp.LSP_ERR_INVALID_ARG
    assert L.lsp_set_batched_form(lsp.LSP_TRIG_DIRECT) == lsp.LSP_ERR_INVALID_ARG
    lsp.lsp_set_batched_form("recur")
    assert lsp.lsp_get_batched_form() == "recur"
    lsp.lsp_set_batched_form("mfma")
    assert lsp.lsp_get_batched_form() == "mfma"


def test_fast_periodogram_validation_on_host():
    L = lsp.lib()
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(16)
    cases = [
        (null, fake, 10, 0.1, 0.1, 10, 4, fake),     # null t
        (fake, fake, 1, 0.1, 0.1, 10, 4, fake),      # Nt < 2
        (fake, fake, 10, 0.1, 0.1, 10, 5, fake),     # macc not 4, 6, 8
        (fake, fake, 10, 0.15, 0.1, 10, 4, fake),    # f_min not a multiple of df
        (fake, fake, 10, 0.1, 0.0, 10, 4, fake),     # df = 0
        (fake, fake, 10, 0.0, 1e-9, 1 << 26, 8, fake),  # grid beyond 2^28
    ]
    for c in cases:
        assert L.lsp_periodogram_fast(*c, null) == lsp.LSP_ERR_INVALID_ARG, c


def test_profile_call_read_validation_on_host():
    L = lsp.lib()
    n = ctypes.c_int64(-1)
    assert L.lsp_profile_read_calls(None, -1, ctypes.byref(n)) == lsp.LSP_ERR_INVALID_ARG
    assert L.lsp_profile_read_calls(None, 4, ctypes.byref(n)) == lsp.LSP_ERR_INVALID_ARG
    assert L.lsp_profile_enable(0) == lsp.LSP_OK
    assert L.lsp_profile_read_calls(None, 0, ctypes.byref(n)) == lsp.LSP_OK and n.value == 0


def test_microbench_validation_on_host():
    L = lsp.lib()
    ops = ctypes.c_double()
    null = ctypes.c_void_p(0)
    for kind, waves, iters in ((-1, 2, 10), (9, 2, 10), (4, 0, 10), (4, 9, 10), (4, 2, 0)):
        assert L.lsp_microbench(kind, waves, iters, null, ctypes.byref(ops), None) == lsp.LSP_ERR_INVALID_ARG
    assert L.lsp_microbench(4, 2, 10, null, None, None) == lsp.LSP_ERR_INVALID_ARG


def test_probe_validation_on_host():
    L = lsp.lib()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation rejects first
    null = ctypes.c_void_p(0)
    assert L.lsp_probe_sincos(fake, -1, fake, fake, null) == lsp.LSP_ERR_INVALID_ARG
    assert L.lsp_probe_sincos(null, 5, fake, fake, null) == lsp.LSP_ERR_INVALID_ARG
    assert L.lsp_probe_sincos(null, 0, null, null, null) == lsp.LSP_OK           # empty: nothing to do
    assert L.lsp_probe_phase(fake, fake, 4, 0.0, 9, fake, null) == lsp.LSP_ERR_INVALID_ARG
    assert L.lsp_probe_phase(fake, fake, 4, float("inf"), 0, fake, null) == lsp.LSP_ERR_INVALID_ARG
    assert L.lsp_probe_phase(fake, null, 4, 0.0, 0, fake, null) == lsp.LSP_ERR_INVALID_ARG
    for M in (0, 33):
        assert L.lsp_probe_recurrence(fake, 4, 0.0, 1.0, 0.1, M, fake, fake, null) == lsp.LSP_ERR_INVALID_ARG
    assert L.lsp_probe_recurrence(fake, 4, 0.0, float("nan"), 0.1, 8, fake, fake, null) == lsp.LSP_ERR_INVALID_ARG
    assert L.lsp_probe_recurrence(fake, 4, 0.0, 1.0, 0.1, 8, null, fake, null) == lsp.LSP_ERR_INVALID_ARG

