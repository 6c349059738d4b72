"""GPU parity at extreme aspect ratios, on sampled bins against the FP64 oracle:
a very long series with few frequencies (2^25 samples: many sample
splits, 64-bit offsets), a short series with a very long grid (2^24
frequencies: a large frequency grid and 64 MB of output), and a 2^22-sample
series on 4096 frequencies.  Bar: max|dPn| / max(Pn_oracle) <= 1e-4 over the
sampled bins (which include the peak and its neighbours)."""
import numpy as np
import pytest

import oracle
from paper_1007_1658_amd import synth
from util import REL_TOL, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1007_1658_amd as lsp  # noqa: E402


def _series(Nt, seed, f0):
    g = np.random.default_rng([1007, seed])
    t = np.cumsum(g.exponential(1.0 / 720.0, Nt))          # sorted, ~2-min mean cadence
    x = (np.sin(2 * np.pi * f0 * t) + g.normal(0, 2.0, Nt)).astype(np.float32)
    return t, x


def _check(c, Pg, n_sample, seed):
    g = np.random.default_rng(seed)
    kpk = int(np.argmax(Pg))
    k = np.unique(np.concatenate([g.integers(0, c.Nf, n_sample),
                                  np.arange(max(0, kpk - 3), min(c.Nf, kpk + 4))]))
    P = oracle.periodogram(c.t, c.x, c.f_min, c.df, k=k)
    err = float(np.max(np.abs(Pg[k].astype(np.float64) - P)) / P.max())
    return err, k, P


@pytest.mark.parametrize("Nt,Nf,n_sample", [(1 << 25, 16, 4), (1 << 22, 4096, 64), (1000, 1 << 24, 256)])
def test_extreme_aspect_ratios(Nt, Nf, n_sample):
    t, x = _series(Nt, Nt % 97, 3.1)
    span = float(t[-1] - t[0])
    df = 1.0 / (4.0 * span)
    if Nf <= 4096:
        f_min = 3.1 - (Nf // 2) * df                     # a window around the signal
        f_min = max(df, f_min)
    else:
        f_min = df
    c = synth.Curve(t, x, f_min, df, Nf)
    print(f"extreme Nt={Nt} Nf={Nf}", flush=True)
    td, xd = to_dev(c)
    for name, kw in (("default", None), ("mfma", dict(trig="mfma", m=32, waves=8)),
                     ("recur", dict(trig="recur", m=8, waves=4))):
        if kw is None:
            Pg = lsp.lsp_periodogram(td, xd, c.f_min, c.df, c.Nf)
        else:
            Pg = lsp.lsp_periodogram_ex(td, xd, c.f_min, c.df, c.Nf, **kw)
        Pg = Pg.cpu().numpy()
        assert np.all(np.isfinite(Pg)) and Pg.min() >= 0.0
        err, k, P = _check(c, Pg, n_sample, 5)
        print(f"  {name}: sampled rel err {err:.2e} over {k.size} bins", flush=True)
        assert err <= REL_TOL, name
    del td, xd
    torch.cuda.empty_cache()
