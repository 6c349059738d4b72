"""GPU parity: the HIP periodogram against the FP64 oracle (needs a gfx950 GPU).

Bar: max|dPn| / max(Pn_oracle) <= 1e-4 and the same peak bin (or an oracle
near-tie within that tolerance), on the same seeded inputs.
"""
import numpy as np
import pytest

import oracle
from paper_1007_1658_amd import synth
from util import REL_TOL, peak_matches, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1007_1658_amd as lsp  # noqa: E402

TRIG_NAME = {lsp.LSP_TRIG_DIRECT: "direct", lsp.LSP_TRIG_RECUR: "recur", lsp.LSP_TRIG_MFMA: "mfma"}
SUM_NAME = {lsp.LSP_SUM_KAHAN: "kahan", lsp.LSP_SUM_TWO: "two"}

# every launch shape built into the library, per phase mode
ALL = [(ph, TRIG_NAME[t["trig"]], t["m"], t["unroll"], SUM_NAME[t["sum"]])
       for ph in ("split", "split32", "naive") for t in lsp.lsp_list_tiles(ph)]


@pytest.fixture(scope="module")
def c0_case():
    c = synth.c0()
    P = oracle.periodogram(c.t, c.x, c.f_min, c.df, Nf=c.Nf)
    return c, P


@pytest.mark.parametrize("phase,trig,m,unroll,summ", ALL)
@pytest.mark.parametrize("waves,splits", [(4, 1), (2, 3)])
def test_c0_all_shapes(c0_case, phase, trig, m, unroll, summ, waves, splits):
    c, P = c0_case
    print(f"c0 phase={phase} trig={trig} m={m} unroll={unroll} sum={summ} waves={waves} splits={splits}",
          flush=True)
    t, x = to_dev(c)
    Pg = lsp.lsp_periodogram_ex(t, x, c.f_min, c.df, c.Nf, phase=phase, trig=trig, m=m, unroll=unroll,
                                sum=summ, waves=waves, splits=splits).cpu().numpy()
    assert rel_err(Pg, P) <= REL_TOL
    assert peak_matches(Pg, P)


@pytest.mark.parametrize("waves", [1, 2, 4, 8])
@pytest.mark.parametrize("Nt,Nf,splits", [(1000, 2000, 1), (1000, 2000, 7), (4097, 3001, 3), (300, 129, 2)])
def test_matrix_core_every_workgroup_size(waves, Nt, Nf, splits):
    """The matrix-core kernel merges the curve's partial moments inside every
    workgroup (any of its 1-8 waves) and converts the raw samples itself:
    parity at each workgroup size, on ragged sizes and a shifted epoch."""
    print(f"mfma waves={waves} Nt={Nt} Nf={Nf} splits={splits}", flush=True)
    g = np.random.default_rng([13, Nt, Nf, splits])
    tt = np.sort(g.uniform(0.0, 40.0, Nt)) + 5.0e4
    xx = (3.0 * np.sin(2 * np.pi * 0.7 * tt) + g.normal(0, 1.0, Nt) + 20.0).astype(np.float32)
    df = 1.0 / (4.0 * (tt[-1] - tt[0]))
    f_min = 0.5 * df
    P = oracle.periodogram(tt, xx, f_min, df, Nf=Nf)
    t = torch.from_numpy(tt).cuda()
    x = torch.from_numpy(xx).cuda()
    Pg = lsp.lsp_periodogram_ex(t, x, f_min, df, Nf, trig="mfma", m=32, waves=waves, splits=splits).cpu().numpy()
    assert rel_err(Pg, P) <= REL_TOL
    assert peak_matches(Pg, P)


@pytest.mark.parametrize("Nt,Nf,splits", [
    (2, 1, 1), (3, 7, 1), (63, 100, 1), (64, 64, 1), (65, 513, 2), (130, 1025, 3),
    (1000, 511, 4), (4097, 3000, 5), (257, 8193, 1), (5000, 20, 64),
])
@pytest.mark.parametrize("phase,trig,m", [("split", "recur", 8), ("split", "recur", 16), ("split", "recur", 14),
                                          ("split", "direct", 1), ("split32", "recur", 8),
                                          ("naive", "direct", 4), ("split", "mfma", 32)])
def test_ragged_sizes(Nt, Nf, splits, phase, trig, m):
    print(f"ragged Nt={Nt} Nf={Nf} splits={splits} {phase}/{trig}/{m}", flush=True)
    g = np.random.default_rng([11, Nt, Nf])
    tt = np.sort(g.uniform(0.0, 30.0, Nt))
    xx = (np.sin(2 * np.pi * 1.3 * tt) + g.normal(0, 1.0, Nt)).astype(np.float32)
    T = tt.max() - tt.min()
    df = 1.0 / (4 * T)
    c = synth.Curve(tt, xx, df, df, Nf)
    P = oracle.periodogram(c.t, c.x, c.f_min, c.df, Nf=Nf)
    t, x = to_dev(c)
    Pg = lsp.lsp_periodogram_ex(t, x, c.f_min, c.df, Nf, phase=phase, trig=trig, m=m,
                                waves=4, splits=splits).cpu().numpy()
    assert Pg.shape == (Nf,)
    assert rel_err(Pg, P) <= REL_TOL
    assert peak_matches(Pg, P)


@pytest.mark.parametrize("Nt,Nf,splits", [(3, 7, 1), (65, 513, 2), (1000, 511, 4), (4097, 30000, 5), (5000, 20, 64)])
def test_matrix_core_form_eight_waves_ragged(Nt, Nf, splits):
    """8-wave workgroups (the tuned matrix-core shape) on ragged sizes: partial
    workgroups in frequency, ragged sample chunks."""
    print(f"ragged mfma w8 Nt={Nt} Nf={Nf} splits={splits}", flush=True)
    g = np.random.default_rng([12, Nt, Nf])
    tt = np.sort(g.uniform(0.0, 30.0, Nt))
    xx = (np.sin(2 * np.pi * 1.3 * tt) + g.normal(0, 1.0, Nt)).astype(np.float32)
    df = 1.0 / (4 * (tt.max() - tt.min()))
    c = synth.Curve(tt, xx, df, df, Nf)
    P = oracle.periodogram(c.t, c.x, c.f_min, c.df, Nf=Nf)
    t, x = to_dev(c)
    Pg = lsp.lsp_periodogram_ex(t, x, c.f_min, c.df, Nf, trig="mfma", m=32, waves=8, splits=splits).cpu().numpy()
    assert rel_err(Pg, P) <= REL_TOL
    assert peak_matches(Pg, P)


def test_default_call_and_output_fully_written(c0_case):
    c, P = c0_case
    t, x = to_dev(c)
    Pn = torch.full((c.Nf + 7,), -1.0, dtype=torch.float32, device="cuda")
    lsp.lsp_periodogram(t, x, c.f_min, c.df, c.Nf, Pn=Pn)
    Pg = Pn.cpu().numpy()
    assert np.all(Pg[:c.Nf] >= 0.0)
    assert np.all(Pg[c.Nf:] == -1.0)  # nothing past Nf is touched
    assert rel_err(Pg[:c.Nf], P) <= REL_TOL


def test_c1_full_size_sampled():
    """Full c1 size in the benchmark's default launch; oracle on sampled bins."""
    c = synth.c1()
    t, x = to_dev(c)
    print(f"c1 Nt={c.Nt} Nf={c.Nf}", flush=True)
    Pg = lsp.lsp_periodogram(t, x, c.f_min, c.df, c.Nf).cpu().numpy()
    g = np.random.default_rng(1)
    kpk = int(np.argmax(Pg))
    k = np.unique(np.concatenate([g.integers(0, c.Nf, 600), np.arange(max(0, kpk - 8), min(c.Nf, kpk + 9)),
                                  np.arange(0, 64), np.arange(c.Nf - 64, c.Nf)]))
    P = oracle.periodogram(c.t, c.x, c.f_min, c.df, k=k)
    err = float(np.max(np.abs(Pg[k] - P)) / P.max())
    print(f"c1 sampled rel err {err:.3e}", flush=True)
    assert err <= REL_TOL
    assert np.all(Pg >= 0) and np.all(Pg <= c.Nt / 2 * (1 + 1e-5))
    # the global peak is one of the injected frequencies (within one bin)
    f_pk = c.f_min + kpk * c.df
    assert np.min(np.abs(c.injected - f_pk)) <= 1.5 * c.df


def test_c2_precision_split_vs_naive():
    """Epoch-offset times (2455000 d + 3650 d): the split path meets the bar, the naive one does not."""
    c = synth.c2()
    t, x = to_dev(c)
    print(f"c2 Nt={c.Nt} Nf={c.Nf}", flush=True)
    Ps = lsp.lsp_periodogram_ex(t, x, c.f_min, c.df, c.Nf, phase="split").cpu().numpy()
    k0 = int(round((13.7 - c.f_min) / c.df))
    g = np.random.default_rng(2)
    k = np.unique(np.concatenate([g.integers(0, c.Nf, 300), np.arange(k0 - 6, k0 + 7)]))
    P = oracle.periodogram(c.t, c.x, c.f_min, c.df, k=k)
    err_s = float(np.max(np.abs(Ps[k] - P)) / P.max())
    assert abs(int(np.argmax(Ps)) - k0) <= 1
    Pn = lsp.lsp_periodogram_ex(t, x, c.f_min, c.df, c.Nf, phase="naive", trig="direct", m=4).cpu().numpy()
    err_n = float(np.max(np.abs(Pn[k] - P)) / P.max())
    print(f"c2 sampled rel err split {err_s:.3e} naive {err_n:.3e}", flush=True)
    assert err_s <= REL_TOL
    assert err_n > 10 * err_s


@pytest.mark.parametrize("config", ["c1", "c2"])
@pytest.mark.parametrize("waves", [8, 4, 2])
def test_matrix_core_form_full_size_sampled(config, waves):
    """The matrix-core form at full size (c1: small amplitudes; c2: epoch-offset
    times), oracle on sampled bins and around the peak."""
    c = getattr(synth, config)()
    t, x = to_dev(c)
    print(f"{config} mfma waves={waves} Nt={c.Nt} Nf={c.Nf}", flush=True)
    Pg = lsp.lsp_periodogram_ex(t, x, c.f_min, c.df, c.Nf, trig="mfma", m=32, waves=waves).cpu().numpy()
    g = np.random.default_rng(3)
    kpk = int(np.argmax(Pg))
    k = np.unique(np.concatenate([g.integers(0, c.Nf, 400), np.arange(max(0, kpk - 8), min(c.Nf, kpk + 9)),
                                  np.arange(0, 64), np.arange(c.Nf - 64, c.Nf)]))
    P = oracle.periodogram(c.t, c.x, c.f_min, c.df, k=k)
    err = float(np.max(np.abs(Pg[k] - P)) / P.max())
    print(f"{config} mfma sampled rel err {err:.3e}", flush=True)
    assert err <= REL_TOL
    assert int(k[np.argmax(P)]) == kpk or abs(P.max() - P[np.searchsorted(k, kpk)]) <= REL_TOL * P.max()


def test_matrix_core_form_outlier_and_dynamic_range():
    """A 1000-sigma spike among unit noise, and a 1e-6 sinusoid in 1e-7 noise:
    the per-chunk power-of-two scaling keeps both within the bar."""
    g = np.random.default_rng(17)
    Nt, Nf = 3000, 6000
    tt = np.sort(g.uniform(0, 50, Nt))
    df = 1.0 / (4 * (tt[-1] - tt[0]))
    spike = g.normal(0, 1, Nt)
    spike[1234] = 1000.0
    tiny = 1e-6 * np.sin(2 * np.pi * 2.2 * tt) + 1e-7 * g.normal(0, 1, Nt)
    for xx in (spike, tiny):
        c = synth.Curve(tt, xx.astype(np.float32), df, df, Nf)
        P = oracle.periodogram(c.t, c.x, c.f_min, c.df, Nf=Nf)
        t, x = to_dev(c)
        for splits in (1, 7):
            Pg = lsp.lsp_periodogram_ex(t, x, df, df, Nf, trig="mfma", m=32, waves=4, splits=splits).cpu().numpy()
            assert rel_err(Pg, P) <= REL_TOL
            assert peak_matches(Pg, P)


def test_deterministic_rerun():
    c = synth.c1(Nt=20000, Nf=40000)
    t, x = to_dev(c)
    a = lsp.lsp_periodogram(t, x, c.f_min, c.df, c.Nf).cpu().numpy()
    b = lsp.lsp_periodogram(t, x, c.f_min, c.df, c.Nf).cpu().numpy()
    assert np.array_equal(a, b)


def test_invariances_on_gpu():
    c = synth.c0(Nt=3000, Nf=6000)
    t, x = to_dev(c)
    base = lsp.lsp_periodogram(t, x, c.f_min, c.df, c.Nf).cpu().numpy()
    m = base.max()
    shifted = lsp.lsp_periodogram(t + 2455000.0, x, c.f_min, c.df, c.Nf).cpu().numpy()
    assert np.max(np.abs(shifted - base)) <= REL_TOL * m
    scaled = lsp.lsp_periodogram(t, (x * -4.5 + 3.0).contiguous(), c.f_min, c.df, c.Nf).cpu().numpy()
    assert np.max(np.abs(scaled - base)) <= REL_TOL * m
    p = torch.randperm(c.Nt, generator=torch.Generator().manual_seed(3)).cuda()
    perm = lsp.lsp_periodogram(t[p].contiguous(), x[p].contiguous(), c.f_min, c.df, c.Nf).cpu().numpy()
    assert np.max(np.abs(perm - base)) <= REL_TOL * m


def test_zero_frequency_and_constant_series():
    c = synth.c0(Nt=500, Nf=50)
    t, x = to_dev(c)
    Pg = lsp.lsp_periodogram(t, x, 0.0, c.df, c.Nf).cpu().numpy()   # k = 0 is f = 0
    P = oracle.periodogram(c.t, c.x, 0.0, c.df, Nf=c.Nf)
    assert abs(Pg[0]) <= REL_TOL * P.max()
    assert rel_err(Pg, P) <= REL_TOL
    xc = torch.full_like(x, 2.5)
    Pc = lsp.lsp_periodogram(t, xc, c.f_min, c.df, c.Nf).cpu().numpy()
    assert np.all(Pc == 0.0)
    with pytest.raises(lsp.LspError) as ei:
        lsp.lsp_periodogram_ex(t, xc, c.f_min, c.df, c.Nf, check=True)
    assert ei.value.status == lsp.LSP_ERR_ZERO_VARIANCE


def test_profile_hook_counts_launches():
    c = synth.c0()
    t, x = to_dev(c)
    lsp.lsp_profile_enable(lsp.PROFILE_KERNEL | lsp.PROFILE_CALLS)
    for _ in range(3):
        lsp.lsp_periodogram(t, x, c.f_min, c.df, c.Nf)
    ms, n, name = lsp.lsp_profile_read()
    calls = lsp.lsp_profile_read_calls()
    lsp.lsp_profile_enable(False)
    assert n == 3 and ms > 0 and name.startswith(("pgram_kernel<", "pgram_mfma_kernel<"))
    # each call's span (first kernel's start to last kernel's end) holds its main kernel
    assert calls.shape == (3,) and np.all(calls > 0) and calls.sum() >= ms
    assert lsp.lsp_profile_read_calls().size == 0   # disabling clears the records
    lsp.lsp_profile_enable(lsp.PROFILE_CALLS)        # calls alone: no kernel records
    lsp.lsp_periodogram(t, x, c.f_min, c.df, c.Nf)
    ms, n, name = lsp.lsp_profile_read()
    calls = lsp.lsp_profile_read_calls()
    lsp.lsp_profile_enable(False)
    assert n == 0 and calls.size == 1 and calls[0] > 0


@pytest.mark.parametrize("K", [1, 3])
def test_profile_hook_on_weighted_passes(K):
    """The hook's events on the generalized (one launch) and multi-harmonic
    (first pass's start to last pass's end) kernels."""
    c = synth.c0()
    t, x = to_dev(c)
    lsp.lsp_profile_enable(True)
    if K == 1:
        lsp.lsp_gls(t, x, c.f_min, c.df, c.Nf)
    else:
        lsp.lsp_multiharmonic(t, x, K, c.f_min, c.df, c.Nf)
    ms, n, name = lsp.lsp_profile_read()
    calls = lsp.lsp_profile_read_calls()
    lsp.lsp_profile_enable(False)
    assert n == 1 and ms > 0 and name.startswith("gls_" if K == 1 else "mh_mfma_kernel")
    assert calls.size == 0   # per-call spans are recorded for single-curve calls only


def test_autotune_and_cache_roundtrip(tmp_path):
    tile, ms = lsp.lsp_autotune(4096, 8192)
    assert tile["m"] > 0 and ms > 0
    c = synth.c0(Nt=4096, Nf=8192)
    t, x = to_dev(c)
    P = oracle.periodogram(c.t, c.x, c.f_min, c.df, k=np.arange(0, 8192, 37))
    Pg = lsp.lsp_periodogram(t, x, c.f_min, c.df, c.Nf).cpu().numpy()  # uses the tuned shape
    assert float(np.max(np.abs(Pg[::37] - P)) / P.max()) <= REL_TOL
    f = tmp_path / "tune.json"
    lsp.lsp_tune_cache_save(str(f))
    lsp.lsp_tune_cache_load(str(f))
    assert "mi355lsp-tune-2" in f.read_text()


def test_invalid_arguments_raise():
    c = synth.c0(Nt=100, Nf=10)
    t, x = to_dev(c)
    for bad in [dict(df=0.0), dict(df=-1.0), dict(Nf=0), dict(f_min=float("nan"))]:
        kw = dict(f_min=c.f_min, df=c.df, Nf=c.Nf)
        kw.update(bad)
        with pytest.raises((lsp.LspError, RuntimeError)):
            lsp.lsp_periodogram(t, x, kw["f_min"], kw["df"], kw["Nf"])
