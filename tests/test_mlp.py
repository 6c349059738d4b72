"""GPU parity of the surrogate network (BF16 MFMA) against the CPU reference."""
import numpy as np
import pytest
from scipy import stats

from oracle import mlp_ref as R
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1007_1658_amd as lsp  # noqa: E402


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("M,N,K", [(32, 32, 32), (64, 96, 256), (256, 32, 96)])
def test_gemm_nt_layout(M, N, K):
    g = torch.Generator().manual_seed(M + N + K)
    A = torch.randn(M, K, generator=g).to(torch.bfloat16)
    B = torch.randn(N, K, generator=g).to(torch.bfloat16)
    C = lsp.lsp_mlp_gemm_nt(A.cuda(), B.cuda()).cpu().numpy().astype(np.float64)
    ref = A.double().numpy() @ B.double().numpy().T
    assert np.max(np.abs(C - ref)) <= 1e-5 * np.abs(ref).max()


def _model_and_data(B=48, nR=64, seed=5):
    g = np.random.default_rng(seed)
    m = lsp.Model(members=2, seed=seed)
    params = [g.normal(0, 0.06, R.N_PARAMS).astype(np.float32) for _ in range(2)]
    for e in range(2):
        m.set_params(e, params[e])
    mean = g.normal(0, 0.3, 68).astype(np.float32)
    std = g.uniform(0.5, 2.0, 68).astype(np.float32)
    m.set_scalers(mean, std, 50.0, MU, SIGMA)
    feat = g.normal(0, 1, (B, 68)) * std + mean
    nt = np.rint(10 ** g.uniform(np.log10(200), np.log10(20000), B))
    feat[:, 64] = np.log10(nt)        # the slots the head reads Nt and Nf from
    feat[:, 67] = np.log10(2 * nt)
    feat = feat.astype(np.float32)
    y = g.normal(9.0, 1.3, (B, nR)).astype(np.float32)
    return m, params, feat, y, mean.astype(np.float64), std.astype(np.float64)


MU, SIGMA = -0.5, 0.3
Z99 = 2.5758293035489   # the bound's standard errors (two-sided 99 % point)


def test_param_roundtrip_and_count():
    m = lsp.Model(members=3, seed=1)
    assert lsp.lsp_model_param_count() == R.N_PARAMS == 149762
    assert m.members == 3
    p = np.random.default_rng(0).normal(0, 1, R.N_PARAMS).astype(np.float32)
    m.set_params(2, p)
    assert np.array_equal(m.get_params(2), p)
    m.close()


def max_elem_rel(a, b, scale):
    """max_i |a_i - b_i| / scale_i (element by element)"""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / scale))


# Element-wise bars.  Both sides round the matrix-product operands to BF16 at
# the same points; they differ by FP32 against FP64 accumulation, which can
# flip the BF16 rounding of an activation (a 2^-8 relative step) and carry it
# forward.  Quantiles: |dq| <= 2e-3 |q|.  Gradients: |dg| <= 2e-2 of the
# largest |g| of the same layer's weights or biases (a per-layer scale, so a
# wrong layout in one product cannot hide behind a large gradient elsewhere).
Q_ELEM_TOL = 2e-3
G_ELEM_TOL = 2e-2


def test_forward_matches_reference():
    m, params, feat, y, mean, std = _model_and_data()
    q = m.forward(torch.from_numpy(feat).cuda()).cpu().numpy()
    for e in range(2):
        ref = R.forward(params[e].astype(np.float64), feat, mean, std, MU, SIGMA, bf=True)["q"]
        err = max_elem_rel(q[e], ref, np.abs(ref))
        print(f"member {e}: quantiles max element rel err {err:.3e}, rel L2 {rel_l2(q[e], ref):.3e}", flush=True)
        assert err <= Q_ELEM_TOL
        assert np.all(np.diff(q[e], axis=1) > 0)
    m.close()


def test_gradient_matches_reference():
    m, params, feat, y, mean, std = _model_and_data()
    g, loss = m.grad(1, torch.from_numpy(feat).cuda(), torch.from_numpy(y).cuda())
    Lr, gr, _ = R.loss_and_grad(params[1].astype(np.float64), feat, y, mean, std, MU, SIGMA, bf=True)
    assert abs(loss.item() - Lr) <= 1e-4 * abs(Lr)
    gg = g.cpu().numpy()
    assert rel_l2(gg, gr) <= 1e-3
    # element by element, per layer's weights and biases
    o = 0
    for li, (n_out, n_in) in enumerate(R.SHAPES):
        for what, sz in (("W", n_out * n_in), ("b", n_out)):
            seg, ref = gg[o:o + sz], gr[o:o + sz]
            err = max_elem_rel(seg, ref, np.abs(ref).max())
            print(f"layer {li} {what}: max |dg| / max |g| = {err:.3e}", flush=True)
            assert err <= G_ELEM_TOL
            o += sz
    m.close()


def test_adam_step_matches_reference():
    m, params, feat, y, mean, std = _model_and_data()
    g, _ = m.grad(0, torch.from_numpy(feat).cuda(), torch.from_numpy(y).cuda())
    gh = g.cpu().numpy().astype(np.float64)
    w0 = m.get_params(0).astype(np.float64)
    m.adam_step(0, 1e-3)
    w1 = m.get_params(0).astype(np.float64)
    ref, mm, vv = R.adam_step(w0, gh, np.zeros_like(w0), np.zeros_like(w0), 1, lr=1e-3)
    assert np.max(np.abs(w1 - ref)) <= 1e-6
    # second step with the same minibatch
    g2, _ = m.grad(0, torch.from_numpy(feat).cuda(), torch.from_numpy(y).cuda())
    m.adam_step(0, 1e-3)
    ref2, _, _ = R.adam_step(ref, g2.cpu().numpy().astype(np.float64), mm, vv, 2, lr=1e-3)
    assert np.max(np.abs(m.get_params(0) - ref2)) <= 2e-6
    m.close()


def test_save_load_roundtrip(tmp_path):
    m, params, feat, y, mean, std = _model_and_data()
    f = str(tmp_path / "m.bin")
    m.save(f)
    m2 = lsp.Model(path=f)
    for e in range(2):
        assert np.array_equal(m2.get_params(e), m.get_params(e))
    fd = torch.from_numpy(feat).cuda()
    assert torch.equal(m.forward(fd), m2.forward(fd))
    with pytest.raises(lsp.LspError) as ei:
        lsp.Model(path=str(tmp_path / "missing.bin"))
    assert ei.value.status == lsp.LSP_ERR_MODEL
    m.close(); m2.close()


def _patterns(n, seed):
    g = np.random.default_rng(seed)
    ts, off, fm, dfs, nfs = [], [0], [], [], []
    for p in range(n):
        nt = int(g.integers(60, 400))
        t = np.sort(g.uniform(0, g.uniform(5, 60), nt))
        df = 1.0 / (4 * (t[-1] - t[0]))
        ts.append(t); off.append(off[-1] + nt); fm.append(df); dfs.append(df); nfs.append(2 * nt)
    return np.concatenate(ts), np.array(off), np.array(fm), np.array(dfs), np.array(nfs)


def test_fap_surrogate_and_fallback():
    t, off, fm, df, nf = _patterns(8, 3)
    td = torch.from_numpy(t).cuda()
    feat = lsp.lsp_window_features(td, off, fm, df, nf)
    m = lsp.Model(members=3, seed=2)
    F = feat.cpu().numpy()
    mean, std = F.mean(0), F.std(0) + 1e-3
    m.set_scalers(mean, std, 1e6, -0.4, 0.5)
    p_obs = torch.linspace(6.0, 12.0, 8).cuda()
    fap, err, used = m.fap(td, off, fm, df, nf, p_obs, max_err=10.0, mc_realizations=0)
    fe = []
    for e in range(3):
        raw = R.forward(m.get_params(e).astype(np.float64), F, mean.astype(np.float32).astype(np.float64),
                        std.astype(np.float32).astype(np.float64), -0.4, 0.5, bf=True)["raw"]
        fe.append(R.fap(raw, F, -0.4, 0.5, p_obs.cpu().numpy()))
    fe = np.array(fe)
    assert np.max(np.abs(fap.cpu().numpy() - fe.mean(0))) <= 1e-3
    # no law errors set: the bound is 2.576 times the members' spread
    assert np.max(np.abs(err.cpu().numpy() - Z99 * fe.std(0))) <= 3e-3
    assert used.sum().item() == 0
    # forced fallback: every pattern answered by Monte Carlo with the same draws as lsp_mc_maxpower
    Rn = 256
    fap2, sig2, used2 = m.fap(td, off, fm, df, nf, p_obs, max_err=0.0, mc_realizations=Rn, seed=77)
    pm = lsp.lsp_mc_maxpower(td, off, fm, df, nf, Rn, seed=77).cpu().numpy()
    assert used2.sum().item() == 8
    expect = (pm >= p_obs.cpu().numpy()[:, None]).mean(axis=1)
    assert np.allclose(fap2.cpu().numpy(), expect, atol=1e-7)
    m.close()


def test_reported_quantiles_and_fap_agree():
    # one member: the FAP at its own tau-quantile is 1 - tau
    t, off, fm, df, nf = _patterns(8, 6)
    td = torch.from_numpy(t).cuda()
    feat = lsp.lsp_window_features(td, off, fm, df, nf)
    F = feat.cpu().numpy()
    m = lsp.Model(members=1, seed=3)
    m.set_scalers(F.mean(0), F.std(0) + 1e-3, 1e6, -0.4, 0.5)
    q = m.forward(feat)[0]
    assert torch.all(q[:, 1:] > q[:, :-1])
    for i, tau in enumerate(R.TAU):
        fap, _, _ = m.fap(td, off, fm, df, nf, q[:, i].contiguous(), max_err=10.0, mc_realizations=0)
        assert np.allclose(fap.cpu().numpy(), 1 - tau, atol=2e-5), tau
    m.close()


def test_short_training_reduces_loss():
    t, off, fm, df, nf = _patterns(64, 4)
    td = torch.from_numpy(t).cuda()
    feat = lsp.lsp_window_features(td, off, fm, df, nf)
    y = lsp.lsp_mc_maxpower(td, off, fm, df, nf, 64, seed=5)
    F = feat.cpu().numpy()
    Y = y.cpu().numpy()
    nt, nfr = R.nt_nf(F)
    W = R.w_of(Y, nt[:, None]) - np.log(nfr)[:, None]
    m = lsp.Model(members=1, seed=9)
    m.set_scalers(F.mean(0), F.std(0) + 1e-3, 1e6, float(W.mean()), float(W.std()))
    losses = []
    for step in range(300):
        _, loss = m.grad(0, feat, y, want_grad=False)
        m.adam_step(0, 3e-3)
        losses.append(loss.item())
    # every pattern's own maximum-likelihood law bounds the in-sample loss from below
    fits = [stats.gumbel_r.fit(W[b]) for b in range(W.shape[0])]
    floor = np.mean([-np.mean(stats.gumbel_r.logpdf(W[b], *fits[b])) for b in range(W.shape[0])])
    assert losses[-1] >= floor - 1e-4
    assert losses[-1] - floor < 0.5 * (losses[0] - floor)
    m.close()


def test_truncated_or_foreign_model_file_is_rejected(tmp_path):
    m, params, feat, y, mean, std = _model_and_data()
    f = tmp_path / "m.bin"
    m.save(str(f))
    data = f.read_bytes()
    (tmp_path / "short.bin").write_bytes(data[: len(data) // 2])
    (tmp_path / "foreign.bin").write_bytes(b"NOT-A-MODEL-FILE" + data[16:])
    for name in ("short.bin", "foreign.bin"):
        with pytest.raises(lsp.LspError) as ei:
            lsp.Model(path=str(tmp_path / name))
        assert ei.value.status == lsp.LSP_ERR_MODEL, name
    m.close()


def test_out_of_range_features_route_to_monte_carlo():
    t, off, fm, df, nf = _patterns(6, 8)
    td = torch.from_numpy(t).cuda()
    feat = lsp.lsp_window_features(td, off, fm, df, nf)
    F = feat.cpu().numpy()
    m = lsp.Model(members=2, seed=4)
    # a feature range narrower than the patterns' own spread: every pattern is out of range
    m.set_scalers(F.mean(0), F.std(0) + 1e-3, 1e-3, -0.4, 0.5)
    p_obs = torch.full((6,), 8.0, device="cuda")
    fap, sig, used = m.fap(td, off, fm, df, nf, p_obs, max_err=10.0, mc_realizations=64, seed=5)
    assert used.sum().item() == 6
    pm = lsp.lsp_mc_maxpower(td, off, fm, df, nf, 64, seed=5).cpu().numpy()
    assert np.allclose(fap.cpu().numpy(), (pm >= 8.0).mean(axis=1), atol=1e-7)
    m.close()


def test_law_errors_enter_bound_fallback_and_model_file(tmp_path):
    """bound = 2.576 sqrt(spread^2 + (err_m dFAP/dm)^2 + (err_beta dFAP/dbeta)^2),
    with the derivatives of each pattern's law at its p_obs; the bound decides
    the fallback and the law errors survive save/load."""
    t, off, fm, df, nf = _patterns(12, 6)
    td = torch.from_numpy(t).cuda()
    feat = lsp.lsp_window_features(td, off, fm, df, nf)
    F = feat.cpu().numpy()
    m = lsp.Model(members=3, seed=7)
    mean, std = F.mean(0), F.std(0) + 1e-3
    m.set_scalers(mean, std, 1e6, -0.4, 0.5)
    p_obs = torch.linspace(5.0, 9.0, 12, device="cuda")
    pn = p_obs.cpu().numpy().astype(np.float64)
    f0, b0, _ = m.fap(td, off, fm, df, nf, p_obs, max_err=1e9, mc_realizations=0)
    err_m, err_b = 0.06, 0.03
    m.set_law_error(err_m, err_b)
    f1, b1, _ = m.fap(td, off, fm, df, nf, p_obs, max_err=1e9, mc_realizations=0)
    f0, b0, f1, b1 = (a.cpu().numpy().astype(np.float64) for a in (f0, b0, f1, b1))
    assert np.array_equal(f0, f1)
    dms, dbs, fs = [], [], []
    for e in range(3):
        raw = R.forward(m.get_params(e).astype(np.float64), F, mean.astype(np.float32).astype(np.float64),
                        std.astype(np.float32).astype(np.float64), -0.4, 0.5, bf=True)["raw"]
        dm, db = R.fap_sensitivity(raw, F, -0.4, 0.5, pn)
        dms.append(dm); dbs.append(db); fs.append(R.fap(raw, F, -0.4, 0.5, pn))
    dm, db, spread = np.mean(dms, 0), np.mean(dbs, 0), np.std(fs, 0)
    expect = Z99 * np.sqrt(spread ** 2 + (err_m * dm) ** 2 + (err_b * db) ** 2)
    print("bound", b1, "expected", expect, flush=True)
    assert np.max(np.abs(b1 - expect)) <= 3e-3 * max(1.0, expect.max())
    # the law terms are what the errors added: against the spread-only bound
    law = np.sqrt(np.maximum((b1 / Z99) ** 2 - (b0 / Z99) ** 2, 0.0))
    assert np.max(np.abs(law - np.sqrt((err_m * dm) ** 2 + (err_b * db) ** 2))) <= 2e-3
    # a tolerance below every bound sends every pattern to Monte Carlo
    _, _, used = m.fap(td, off, fm, df, nf, p_obs, max_err=float(b1.min()) * 0.5, mc_realizations=32, seed=3)
    assert used.sum().item() == 12
    path = str(tmp_path / "m.bin")
    m.save(path)
    m2 = lsp.Model(path=path)
    _, b2, _ = m2.fap(td, off, fm, df, nf, p_obs, max_err=1e9, mc_realizations=0)
    assert np.allclose(b2.cpu().numpy(), b1, rtol=1e-6)
    for bad in ((-0.1, 0.0), (0.0, float("nan")), (20.0, 0.0)):
        with pytest.raises(lsp.LspError) as ei:
            m.set_law_error(*bad)
        assert ei.value.status == lsp.LSP_ERR_INVALID_ARG
    m.close(); m2.close()
