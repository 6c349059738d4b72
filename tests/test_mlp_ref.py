"""Pins of the CPU reference of the surrogate network (CPU only)."""
import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import mlp_ref as R


def _feat(g, B):
    """Random features with valid Nt (feat[64]) and Nf = 2 Nt (feat[67])."""
    feat = g.normal(0, 1, (B, 68))
    nt = np.rint(10 ** g.uniform(np.log10(200), np.log10(20000), B))
    feat[:, 64] = np.log10(nt)
    feat[:, 67] = np.log10(2 * nt)
    return feat


def _setup(seed=0, B=16, nR=40, scale=0.05):
    g = np.random.default_rng(seed)
    p = g.normal(0, scale, R.N_PARAMS)
    feat = _feat(g, B)
    y = g.normal(9.0, 1.5, (B, nR))
    return p, feat, y, np.zeros(68), np.ones(68), -0.5, 0.3


def test_bf16_rounding_known_values():
    # 1 + 2^-8 is halfway between BF16 neighbours 1 and 1 + 2^-7: ties to even -> 1
    assert R.bf16(1.0 + 2 ** -8) == 1.0
    assert R.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6     # halfway, rounds to the even 1 + 2^-6
    assert R.bf16(1.0 + 2 ** -8 + 2 ** -12) == 1.0 + 2 ** -7
    assert R.bf16(-2.5) == -2.5 and R.bf16(0.0) == 0.0


def test_gradient_matches_finite_differences():
    p, feat, y, mean, std, mu, sigma = _setup()
    L, g, _ = R.loss_and_grad(p, feat, y, mean, std, mu, sigma, bf=False)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.integers(0, R.N_PARAMS, 40), [R.N_PARAMS - 1, R.N_PARAMS - 9, 0]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        Lp = R.loss_and_grad(pp, feat, y, mean, std, mu, sigma, bf=False)[0]
        Lm = R.loss_and_grad(pm, feat, y, mean, std, mu, sigma, bf=False)[0]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g).max()), i


def test_gumbel_nll_matches_library_and_vanishes_at_its_fit():
    # the loss is the Gumbel (maximum) negative log-likelihood: scipy's density,
    # and zero gradient at scipy's maximum-likelihood fit
    w = stats.gumbel_r.rvs(loc=-0.4, scale=1.07, size=(1, 4000), random_state=5)
    loc, scale = stats.gumbel_r.fit(w[0])
    L, dm, db = R.gumbel_nll(np.array([loc]), np.array([scale]), w)
    assert L == pytest.approx(-np.mean(stats.gumbel_r.logpdf(w[0], loc, scale)), rel=1e-12)
    _, dm1, db1 = R.gumbel_nll(np.array([loc + 0.05]), np.array([scale * 1.05]), w)
    assert abs(dm[0]) < 1e-3 * abs(dm1[0]) + 1e-9 and abs(db[0]) < 1e-3 * abs(db1[0]) + 1e-9


def test_unit_law_is_eq3_with_all_frequencies_independent():
    # m = 0, beta = 1: P(max >= p) = 1 - exp(-Nf e^-w) against Eq. (3),
    # 1 - (1 - e^-w)^Nf; they differ by about (Nf e^-w)^2 / (2 Nf)
    feat = _feat(np.random.default_rng(2), 8)
    nt, nf = R.nt_nf(feat)
    mu, sigma = 0.7, 1.3
    raw = np.zeros((8, 2))
    raw[:, 0] = -mu / sigma
    for fap_target in (0.2, 0.05, 0.01, 0.001):
        w = np.log(nf) - np.log(-np.log1p(-fap_target))
        p = R.z_of(w, nt)
        got = R.fap(raw, feat, mu, sigma, p)
        eq3 = np.array([oracle.fap(float(p[i]), int(nt[i]), int(nf[i])) for i in range(8)])
        lam = nf * np.exp(-w)
        assert np.all(np.abs(got - eq3) <= lam ** 2 / nf), fap_target
        assert np.allclose(got, fap_target, rtol=1e-12)


def test_quantiles_hit_their_levels():
    g = np.random.default_rng(4)
    feat = _feat(g, 12)
    raw = g.normal(0, 1.5, (12, 2))
    q = R.quantiles(raw, feat, 0.3, 0.8)
    assert np.all(np.diff(q, axis=1) > 0)
    for i, t in enumerate(R.TAU):
        assert np.allclose(R.fap(raw, feat, 0.3, 0.8, q[:, i]), 1 - t, rtol=1e-10)


def test_adam_first_step_is_signed_lr():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 2.0])
    w1, m, v = R.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    assert np.allclose(w1, w - 0.01 * np.sign(g), atol=1e-9)


def test_head_scale_is_positive_and_gelu_grad_matches():
    raw = np.random.default_rng(3).normal(0, 3, (20, 2))
    m, b = R.head(raw, 9.0, 1.5)
    assert np.all(b > 0) and np.allclose(R.head(np.zeros((1, 2)), 9.0, 1.5)[1], 1.0)
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    assert np.allclose(R.gelu_grad(z), (R.gelu(z + h) - R.gelu(z - h)) / (2 * h), atol=1e-8)


def test_gelu_matches_torch_tanh_form_and_erf_form():
    """The tanh-form GELU against an independent implementation (torch's
    approximate='tanh' on the CPU, in FP64), and against the exact erf form
    it approximates (Hendrycks & Gimpel's tanh form is within 5e-4 of it): a
    wrong constant in either the sqrt(2/pi) factor or the cubic coefficient
    fails the first comparison."""
    torch = pytest.importorskip("torch")
    from scipy.special import erf
    z = np.linspace(-8.0, 8.0, 4001)
    ref = torch.nn.functional.gelu(torch.from_numpy(z), approximate="tanh").numpy()
    assert np.max(np.abs(R.gelu(z) - ref)) <= 1e-14
    exact = 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))
    assert np.max(np.abs(R.gelu(z) - exact)) <= 5e-4


def test_fap_sensitivity_matches_finite_differences():
    """The law's derivatives that carry the calibrated location and scale
    errors to a pattern's FAP, against central differences of R.fap in m
    (through mu) and in beta (through the scale output)."""
    g = np.random.default_rng(11)
    B = 12
    feat = _feat(g, B)
    raw = g.normal(0, 0.5, (B, 2))
    nt, nf = R.nt_nf(feat)
    p = R.z_of(np.log(nf) + g.uniform(-1.0, 4.0, B), nt)
    mu, sigma = -0.4, 0.5
    dm, db = R.fap_sensitivity(raw, feat, mu, sigma, p)
    h = 1e-6
    fd_m = (R.fap(raw, feat, mu + h, sigma, p) - R.fap(raw, feat, mu - h, sigma, p)) / (2 * h)
    assert np.allclose(dm, fd_m, rtol=1e-6, atol=1e-10)
    # beta = softplus(r1 + shift): d beta / d r1 = sigmoid(r1 + shift)
    _, beta = R.head(raw, mu, sigma)
    rp, rm = raw.copy(), raw.copy()
    rp[:, 1] += h
    rm[:, 1] -= h
    fd_r = (R.fap(rp, feat, mu, sigma, p) - R.fap(rm, feat, mu, sigma, p)) / (2 * h)
    dbeta_dr = 1.0 / (1.0 + np.exp(-(raw[:, 1] + R.BETA_SHIFT)))
    assert np.allclose(db * dbeta_dr, fd_r, rtol=1e-6, atol=1e-10)
