"""GPU parity of the multi-harmonic periodogram (K = 2, 3, 4) against the FP64 oracle
(the least-squares definition; Section 6.3's pointer to Schwarzenberg-Czerny).
Bar: max|dp| / max(p_oracle) <= 1e-4 and the same peak bin."""
import numpy as np
import pytest

import oracle
from paper_1007_1658_amd import synth
from util import REL_TOL, peak_matches, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1007_1658_amd as lsp  # noqa: E402


def _dev(*arrs):
    return [None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def _case(Nt, seed, weighted):
    g = np.random.default_rng([29, Nt, seed])
    t = np.sort(g.uniform(0.0, 30.0, Nt))
    sig = g.uniform(0.3, 2.0, Nt)
    ph = 2 * np.pi * 0.9 * t
    y = (4.0 + 0.8 * np.sin(ph) + 0.5 * np.cos(2 * ph + 0.3) + sig * g.normal(0, 1, Nt)).astype(np.float32)
    w = (1.0 / sig ** 2).astype(np.float32) if weighted else None
    return t, y, w


@pytest.mark.parametrize("Nt,Nf,splits", [(9, 7, 1), (63, 100, 1), (64, 1025, 2), (130, 513, 3),
                                          (1000, 2000, 4), (4097, 3000, 7), (5000, 20, 64)])
@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("K", [2, 3, 4])
def test_multiharmonic_matches_oracle(Nt, Nf, splits, weighted, K):
    """Every bin, including the lowest (less than a cycle over the baseline,
    where the centred normal equations are ill-conditioned and the merge hands
    the bin to the FP64 recomputation) and Nt = 2K + 1 (as many samples as
    parameters: the fit interpolates)."""
    print(f"mh K={K} Nt={Nt} Nf={Nf} splits={splits} weighted={weighted}", flush=True)
    t, y, w = _case(Nt, 1, weighted)
    df = 1.0 / (4 * (t[-1] - t[0]))
    P = oracle.multiharmonic(t, y.astype(np.float64), K, df, df, Nf=Nf,
                             w=None if w is None else w.astype(np.float64))
    td, yd, wd = _dev(t, y, w)
    Pg = lsp.lsp_multiharmonic(td, yd, K, df, df, Nf, w=wd, splits=splits).cpu().numpy()
    err = rel_err(Pg, P)
    print(f"mh K={K} Nt={Nt}: every-bin rel err {err:.3e}", flush=True)
    assert err <= REL_TOL
    assert peak_matches(Pg, P)
    assert np.all(Pg >= -1e-5) and np.all(Pg <= 1 + 1e-5)


@pytest.mark.parametrize("K", [2, 4])
def test_multiharmonic_full_size_sampled(K):
    """c1's sampling (Nt 65,536, Nf 131,072) with weights; oracle on sampled bins."""
    c = synth.c1()
    g = np.random.default_rng(5)
    w = g.uniform(0.5, 2.0, c.Nt).astype(np.float32)
    td, yd, wd = _dev(c.t, c.x, w)
    Pg = lsp.lsp_multiharmonic(td, yd, K, c.f_min, c.df, c.Nf, w=wd).cpu().numpy()
    kpk = int(np.argmax(Pg))
    k = np.unique(np.concatenate([g.integers(0, c.Nf, 150), np.arange(max(0, kpk - 6), min(c.Nf, kpk + 7)),
                                  np.arange(0, 16), np.arange(c.Nf - 16, c.Nf)]))
    P = oracle.multiharmonic(c.t, c.x.astype(np.float64), K, c.f_min, c.df, k=k, w=w.astype(np.float64))
    err = float(np.max(np.abs(Pg[k] - P)) / P.max())
    low = float(np.max(np.abs(Pg[:16] - P[:16])) / P.max())
    print(f"mh K={K} c1 sampled rel err {err:.3e} (first 16 bins {low:.3e})", flush=True)
    assert err <= REL_TOL


def test_multiharmonic_long_series_sampled():
    """K = 2 on 2^20 weighted samples: the records kernel (bounded grid, each
    block merging the moments itself) strides over them; oracle on sampled
    bins and the lowest eight."""
    Nt, Nf, K = 1 << 20, 2048, 2
    t, y, w = _case(Nt, 3, True)
    df = 1.0 / (4 * (t[-1] - t[0]))
    print(f"mh long Nt={Nt} Nf={Nf} K={K}", flush=True)
    td, yd, wd = _dev(t, y, w)
    Pg = lsp.lsp_multiharmonic(td, yd, K, df, df, Nf, w=wd).cpu().numpy()
    g = np.random.default_rng(12)
    kpk = int(np.argmax(Pg))
    k = np.unique(np.concatenate([g.integers(0, Nf, 32), np.arange(max(0, kpk - 3), min(Nf, kpk + 4)),
                                  np.arange(0, 8)]))
    P = oracle.multiharmonic(t, y.astype(np.float64), K, df, df, k=k, w=w.astype(np.float64))
    err = float(np.max(np.abs(Pg[k] - P)) / P.max())
    print(f"mh long sampled rel err {err:.3e}", flush=True)
    assert err <= REL_TOL
    assert abs((kpk + 1) * df - 0.9) <= 1.5 * df


def test_one_harmonic_is_lsp_gls_and_bad_K_raises():
    t, y, w = _case(900, 2, True)
    df = 1.0 / (4 * (t[-1] - t[0]))
    td, yd, wd = _dev(t, y, w)
    p1 = lsp.lsp_multiharmonic(td, yd, 1, df, df, 1500, w=wd)
    pg = lsp.lsp_gls(td, yd, df, df, 1500, w=wd)
    assert torch.equal(p1, pg)
    with pytest.raises(lsp.LspError) as ei:
        lsp.lsp_multiharmonic(td, yd, 5, df, df, 1500, w=wd)
    assert ei.value.status == lsp.LSP_ERR_UNSUPPORTED
    with pytest.raises(lsp.LspError) as ei:
        lsp.lsp_multiharmonic(td, yd, 0, df, df, 1500, w=wd)
    assert ei.value.status == lsp.LSP_ERR_INVALID_ARG
