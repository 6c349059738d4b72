"""Race check of the matrix-core kernels, whose waves share LDS operands across
barriers: the debug build (LSP_POISON_LDS) fills the shared staging area with
NaN bits after every block's reads, so any read that a barrier does not order
after its write returns NaN.  The same parity bar as the normal build must
hold: max|dPn| / max(Pn_oracle) <= 1e-4 (and finite output)."""
import os

import numpy as np
import pytest

import oracle
from paper_1007_1658_amd import synth
from util import REL_TOL, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1007_1658_amd as lsp  # noqa: E402
from paper_1007_1658_amd import build as pkg_build  # noqa: E402

if not os.path.exists(pkg_build.POISON_LIB):  # pragma: no cover
    pytest.skip("LDS-poison build missing (run build())", allow_module_level=True)


@pytest.fixture
def poisoned(monkeypatch):
    monkeypatch.setattr(lsp, "_lib", lsp.load_library(pkg_build.POISON_LIB))
    lsp.lsp_set_batched_form("mfma")
    yield
    lsp.lsp_set_batched_form("mfma")


def _series(Nt, Nf, seed):
    g = np.random.default_rng([77, Nt, seed])
    t = np.sort(g.uniform(0.0, 40.0, Nt))
    x = (np.sin(2 * np.pi * 1.1 * t) + g.normal(0, 1.0, Nt)).astype(np.float32)
    df = 1.0 / (4 * (t[-1] - t[0]))
    return synth.Curve(t, x, df, df, Nf)


@pytest.mark.parametrize("Nt,Nf,waves,splits", [(1000, 2000, 4, 1), (1000, 2000, 8, 3), (4097, 20000, 8, 5),
                                                (65, 513, 4, 2)])
def test_poisoned_periodogram(poisoned, Nt, Nf, waves, splits):
    c = _series(Nt, Nf, 1)
    print(f"poison mfma Nt={Nt} Nf={Nf} waves={waves} splits={splits}", flush=True)
    t, x = to_dev(c)
    Pg = lsp.lsp_periodogram_ex(t, x, c.f_min, c.df, Nf, trig="mfma", m=32, waves=waves, splits=splits)
    Pg = Pg.cpu().numpy()
    P = oracle.periodogram(c.t, c.x, c.f_min, c.df, Nf=Nf)
    assert np.isfinite(Pg).all()
    assert rel_err(Pg, P) <= REL_TOL


def test_poisoned_gls_and_multiharmonic(poisoned):
    c = _series(3000, 4000, 2)
    w = np.random.default_rng(3).uniform(0.5, 2.0, c.Nt).astype(np.float32)
    t, x = to_dev(c)
    wd = torch.from_numpy(w).cuda()
    pg = lsp.lsp_gls(t, x, c.f_min, c.df, c.Nf, w=wd, waves=8, splits=3).cpu().numpy()
    P = oracle.gls(c.t, c.x.astype(np.float64), c.f_min, c.df, Nf=c.Nf, w=w.astype(np.float64))
    assert np.isfinite(pg).all() and rel_err(pg, P) <= REL_TOL
    for K in (2, 4):
        pk = lsp.lsp_multiharmonic(t, x, K, c.f_min, c.df, c.Nf, w=wd, splits=3).cpu().numpy()
        Pk = oracle.multiharmonic(c.t, c.x.astype(np.float64), K, c.f_min, c.df, Nf=c.Nf,
                                  w=w.astype(np.float64))
        k = np.arange(8, c.Nf)   # a few cycles per baseline: well-conditioned normal equations
        assert np.isfinite(pk).all()
        assert np.max(np.abs(pk[k] - Pk[k])) <= REL_TOL * Pk.max(), K


def test_poisoned_batched(poisoned):
    b = synth.c3(seed_sub=1, n_curves=48, nt_range=(2, 3000), T_range=(5.0, 200.0))  # as tests/test_batched.py
    t = torch.from_numpy(b.t).cuda()
    x = torch.from_numpy(b.x).cuda()
    out = lsp.lsp_periodogram_batched(t, x, b.off, b.f_min, b.df, b.Nf, want_pn=True)
    torch.cuda.synchronize()
    Pn = out["Pn"].cpu().numpy()
    assert np.isfinite(Pn).all()
    pn_off = np.concatenate([[0], np.cumsum(b.Nf)])
    for c in range(b.n):
        cv = b.curve(c)
        P = oracle.periodogram(cv.t, cv.x, cv.f_min, cv.df, Nf=cv.Nf)
        assert rel_err(Pn[pn_off[c]:pn_off[c + 1]], P) <= REL_TOL, c
