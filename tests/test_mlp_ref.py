"""Pins of the CPU reference of the surrogate network (CPU only)."""
import numpy as np
import pytest

from oracle import mlp_ref as R


def _setup(seed=0, B=16, nR=40, scale=0.05):
    g = np.random.default_rng(seed)
    p = g.normal(0, scale, R.N_PARAMS)
    feat = g.normal(0, 1, (B, 68))
    y = g.normal(9.0, 1.5, (B, nR))
    return p, feat, y, np.zeros(68), np.ones(68), 9.0, 1.5


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


def test_pinball_closed_form():
    # one pattern, samples 1..10: at q = 5.5 the tau-quantile loss is the mean of rho
    y = np.arange(1.0, 11.0)[None, :]
    q = np.full((1, 9), 5.5)
    L, dq = R.pinball(q, y)
    # L = 1/9 sum_tau mean_r rho_tau(y_r - q), written out sample by sample
    expect = np.mean([np.mean([(v - 5.5) * (t - (v < 5.5)) for v in y[0]]) for t in R.TAU])
    assert L == pytest.approx(expect, rel=1e-12)
    assert np.allclose(dq, (0.5 - R.TAU[None, :]) / 9)


def test_adam_first_step_is_signed_lr():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 2.0])
    w1, m, v = R.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    assert np.allclose(w1, w - 0.01 * np.sign(g), atol=1e-9)


def test_fap_interpolation_hits_the_levels():
    q = np.array([5.0, 5.6, 6.3, 6.9, 7.4, 8.0, 8.5, 9.1, 9.6])
    for i, t in enumerate(R.TAU):
        assert R.fap_from_quantiles(q, q[i]) == pytest.approx(1 - t, rel=1e-12)
    # monotone in p, and beyond the ends it follows the end segments
    ps = np.linspace(3, 12, 50)
    f = [R.fap_from_quantiles(q, p) for p in ps]
    assert np.all(np.diff(f) < 0)


def test_head_is_monotone_and_gelu_grad_matches():
    raw = np.random.default_rng(3).normal(0, 3, (20, 9))
    q = R.head(raw, 9.0, 1.5)
    assert np.all(np.diff(q, axis=1) > 0)
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    assert np.allclose(R.gelu_grad(z), (R.gelu(z + h) - R.gelu(z - h)) / (2 * h), atol=1e-8)
