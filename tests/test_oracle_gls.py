"""Pins of the oracle's generalized (floating-mean, weighted) periodogram (CPU).

The definition: the weighted least-squares fraction of variance explained by
a cos wt + b sin wt + c (Zechmeister & Kuerster 2009, named in Section 6.3).
"""
import numpy as np
import pytest

import oracle


def _lstsq_power(t, y, w, f):
    """Brute force: weighted least squares with numpy, p = 1 - chi2_min / chi2_0."""
    sw = np.sqrt(w)
    A = np.stack([np.cos(2 * np.pi * f * t), np.sin(2 * np.pi * f * t), np.ones_like(t)], axis=1)
    coef, *_ = np.linalg.lstsq(A * sw[:, None], y * sw, rcond=None)
    chi2 = np.sum(w * (y - A @ coef) ** 2)
    Y = np.sum(w * y) / np.sum(w)
    chi0 = np.sum(w * (y - Y) ** 2)
    return 1.0 - chi2 / chi0


@pytest.mark.parametrize("Nt", [5, 17, 200])
@pytest.mark.parametrize("weighted", [False, True])
def test_gls_matches_brute_force_least_squares(Nt, weighted):
    g = np.random.default_rng([5, Nt, weighted])
    t = np.sort(g.uniform(0, 20, Nt))
    y = 3.0 + np.sin(2 * np.pi * 0.41 * t) + g.normal(0, 0.7, Nt)
    w = g.uniform(0.2, 3.0, Nt) if weighted else np.ones(Nt)
    df = 1.0 / (4 * (t[-1] - t[0]))
    k = np.arange(1, 60)
    p = oracle.gls(t, y, df * 0.5, df, k=k, w=w if weighted else None)
    for i, kk in enumerate(k):
        assert p[i] == pytest.approx(_lstsq_power(t, y, w, df * 0.5 + kk * df), rel=1e-8, abs=1e-12)


def test_gls_is_lomb_scargle_at_fourier_frequencies_of_even_sampling():
    # there sum cos = sum sin = 0: fitting the mean changes nothing and
    # p = 2 Pn / N with Pn the paper's normalized periodogram (Eq. 1)
    N = 64
    t = np.arange(N) * 0.5
    g = np.random.default_rng(1)
    y = g.normal(0, 1, N) + 2.0
    df = 1.0 / (N * 0.5)
    k = np.arange(1, N // 2)
    p = oracle.gls(t, y, 0.0, df, k=k)
    Pn = oracle.periodogram(t, y, 0.0, df, k=k)
    assert np.allclose(p, 2 * Pn / N, rtol=1e-10, atol=1e-13)


def test_gls_invariances_and_range():
    g = np.random.default_rng(2)
    t = np.sort(g.uniform(0, 40, 300))
    y = np.cos(2 * np.pi * 1.7 * t + 0.3) + g.normal(0, 1, 300)
    w = g.uniform(0.5, 2, 300)
    df = 1.0 / (4 * 40.0)
    p = oracle.gls(t, y, df, df, Nf=400, w=w)
    assert np.all(p >= -1e-12) and np.all(p <= 1 + 1e-12)
    # floating mean: an added constant changes nothing; neither does a scale of y or of w
    assert np.allclose(oracle.gls(t, y + 50.0, df, df, Nf=400, w=w), p, rtol=1e-9, atol=1e-12)
    assert np.allclose(oracle.gls(t, -3.5 * y, df, df, Nf=400, w=w), p, rtol=1e-12, atol=1e-14)
    assert np.allclose(oracle.gls(t, y, df, df, Nf=400, w=7 * w), p, rtol=1e-12, atol=1e-14)
    # a sample given twice is the same sample with twice the weight
    i = 123
    t2, y2, w2 = np.insert(t, i, t[i]), np.insert(y, i, y[i]), np.insert(w, i, w[i])
    w3 = w.copy()
    w3[i] *= 2
    assert np.allclose(oracle.gls(t2, y2, df, df, Nf=400, w=w2), oracle.gls(t, y, df, df, Nf=400, w=w3),
                       rtol=1e-11, atol=1e-14)


def test_gls_of_an_exact_sinusoid_with_offset_is_one():
    g = np.random.default_rng(3)
    t = np.sort(g.uniform(0, 10, 40))
    df = 0.01
    f = 0.37
    y = 1.3 * np.cos(2 * np.pi * f * t) - 0.4 * np.sin(2 * np.pi * f * t) + 12.0
    p = oracle.gls(t, y, f, df, Nf=1)
    assert p[0] == pytest.approx(1.0, abs=1e-12)
    # the fixed-mean periodogram does not reach its maximum there in general
    assert 2 * oracle.periodogram(t, y, f, df, Nf=1)[0] / t.size < 1 - 1e-6
