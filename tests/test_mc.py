"""GPU parity of the Monte-Carlo generator, noise max power and window features."""
import numpy as np
import pytest

import oracle
from paper_1007_1658_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1007_1658_amd as lsp  # noqa: E402


@pytest.fixture(params=["mfma", "recur"], autouse=True)
def batched_form(request):
    """Every test here runs on both kernel forms of the batched path."""
    print(f"batched form {request.param}", flush=True)
    lsp.lsp_set_batched_form(request.param)
    yield request.param
    lsp.lsp_set_batched_form("mfma")


def _patterns(n, seed, nt_range=(40, 600)):
    g = np.random.default_rng(seed)
    ts, off, fm, dfs, nfs = [], [0], [], [], []
    for p in range(n):
        nt = int(g.integers(*nt_range))
        t = np.sort(g.uniform(0, g.uniform(5, 80), nt))
        df = 1.0 / (4 * (t[-1] - t[0]))
        ts.append(t); off.append(off[-1] + nt); fm.append(df); dfs.append(df); nfs.append(2 * nt)
    return np.concatenate(ts), np.array(off), np.array(fm), np.array(dfs), np.array(nfs)


@pytest.mark.parametrize("seed,stream", [(0, 0), (12345, 7), (2**63 + 11, 2**40 + 3)])
def test_normals_match_oracle(seed, stream):
    z = lsp.lsp_normals(seed, stream, 5000).cpu().numpy().astype(np.float64)
    zo = oracle.normals(seed, stream, 5000)
    assert np.max(np.abs(z - zo) / (1 + np.abs(zo))) < 2e-6


def test_mc_maxpower_matches_oracle_and_is_batch_invariant():
    t, off, fm, df, nf = _patterns(5, 1)
    td = torch.from_numpy(t).cuda()
    R = 6
    pm = lsp.lsp_mc_maxpower(td, off, fm, df, nf, R, seed=99).cpu().numpy()
    for p in range(5):
        tp = t[off[p]:off[p + 1]]
        ref = oracle.mc_maxpower(tp, fm[p], df[p], nf[p], R, seed=99, stream_base=p * R)
        assert np.max(np.abs(pm[p] - ref) / ref.max()) <= 1e-4, p
    # the same draws when the batch is split: stream ids, not batch layout, pick the deviates
    pm2 = lsp.lsp_mc_maxpower(td[off[2]:off[3]].contiguous(), off[2:4] - off[2], fm[2:3], df[2:3], nf[2:3], R,
                              seed=99, stream_base=2 * R).cpu().numpy()
    assert np.array_equal(pm2[0], pm[2])


def test_window_features_match_oracle():
    t, off, fm, df, nf = _patterns(6, 2, (30, 3000))
    td = torch.from_numpy(t).cuda()
    F = lsp.lsp_window_features(td, off, fm, df, nf).cpu().numpy().astype(np.float64)
    for p in range(6):
        ref = oracle.window_features(t[off[p]:off[p + 1]], fm[p], df[p], nf[p])
        assert np.max(np.abs(F[p, :64] - ref[:64])) < 1e-4, p
        assert np.allclose(F[p, 64:], ref[64:], rtol=1e-6, atol=1e-6)


def test_batched_groups_regression():
    """The regrouped batched launch still matches single-curve calls bit for bit."""
    b = synth.c3(seed_sub=4, n_curves=12, nt_range=(100, 2000))
    t = torch.from_numpy(b.t).cuda()
    x = torch.from_numpy(b.x).cuda()
    out = lsp.lsp_periodogram_batched(t, x, b.off, b.f_min, b.df, b.Nf, want_pn=True)
    Pn = out["Pn"].cpu().numpy()
    pn_off = np.concatenate([[0], np.cumsum(b.Nf)])
    for c in range(b.n):
        cv = b.curve(c)
        P = oracle.periodogram(cv.t, cv.x, cv.f_min, cv.df, Nf=cv.Nf)
        assert np.max(np.abs(Pn[pn_off[c]:pn_off[c + 1]] - P)) <= 1e-4 * P.max()
