"""Pins of the oracle's multi-harmonic periodogram (CPU).

The definition: the weighted least-squares fraction of variance explained by
c + sum_{h<=K} (a_h cos h wt + b_h sin h wt) (Schwarzenberg-Czerny 1996,
named in Section 6.3)."""
import numpy as np
import pytest

import oracle


def _lstsq_power(t, y, w, f, K):
    sw = np.sqrt(w)
    cols = [np.ones_like(t)]
    for h in range(1, K + 1):
        cols += [np.cos(2 * np.pi * h * f * t), np.sin(2 * np.pi * h * f * t)]
    A = np.stack(cols, axis=1)
    coef, *_ = np.linalg.lstsq(A * sw[:, None], y * sw, rcond=None)
    chi2 = np.sum(w * (y - A @ coef) ** 2)
    Y = np.sum(w * y) / np.sum(w)
    return 1.0 - chi2 / np.sum(w * (y - Y) ** 2)


@pytest.mark.parametrize("K", [1, 2, 3, 4])
@pytest.mark.parametrize("weighted", [False, True])
def test_mh_matches_brute_force_least_squares(K, weighted):
    g = np.random.default_rng([8, K, weighted])
    Nt = 120
    t = np.sort(g.uniform(0, 25, Nt))
    y = 2.0 + np.sin(2 * np.pi * 0.33 * t) + 0.5 * np.cos(4 * np.pi * 0.33 * t + 1) + g.normal(0, 0.8, Nt)
    w = g.uniform(0.3, 3.0, Nt) if weighted else np.ones(Nt)
    df = 1.0 / (4 * (t[-1] - t[0]))
    k = np.arange(1, 50)
    p = oracle.multiharmonic(t, y, K, df, df, k=k, w=w if weighted else None)
    for i, kk in enumerate(k):
        assert p[i] == pytest.approx(_lstsq_power(t, y, w, df + kk * df, K), rel=1e-8, abs=1e-12)


def test_one_harmonic_is_the_generalized_periodogram():
    g = np.random.default_rng(9)
    t = np.sort(g.uniform(0, 40, 400))
    y = np.cos(2 * np.pi * 1.1 * t) + g.normal(0, 1, 400)
    w = g.uniform(0.5, 2, 400)
    df = 1.0 / 160
    assert np.allclose(oracle.multiharmonic(t, y, 1, df, df, Nf=300, w=w), oracle.gls(t, y, df, df, Nf=300, w=w),
                       rtol=1e-10, atol=1e-13)


def test_mh_exact_harmonic_signal_monotone_in_K_and_invariances():
    g = np.random.default_rng(10)
    t = np.sort(g.uniform(0, 10, 80))
    f = 0.7
    y = 3 + np.cos(2 * np.pi * f * t) + 0.4 * np.sin(4 * np.pi * f * t) - 0.2 * np.cos(6 * np.pi * f * t)
    assert oracle.multiharmonic(t, y, 3, f, 0.01, Nf=1)[0] == pytest.approx(1.0, abs=1e-10)
    assert oracle.multiharmonic(t, y, 2, f, 0.01, Nf=1)[0] < 1 - 1e-3
    # more harmonics never explain less (nested least-squares fits)
    yn = y + g.normal(0, 0.5, 80)
    ps = [oracle.multiharmonic(t, yn, K, 0.05, 0.05, Nf=60) for K in (1, 2, 3, 4)]
    for a, b in zip(ps, ps[1:]):
        assert np.all(b >= a - 1e-12)
    # an offset or scale of y changes nothing; p in [0, 1]
    assert np.allclose(oracle.multiharmonic(t, -2 * yn + 7, 2, 0.05, 0.05, Nf=60), ps[1], rtol=1e-9, atol=1e-12)
    assert np.all(ps[3] >= -1e-12) and np.all(ps[3] <= 1 + 1e-12)


def test_mh_degenerate_zero_frequency_is_zero():
    g = np.random.default_rng(11)
    t = np.sort(g.uniform(0, 5, 30))
    y = g.normal(0, 1, 30)
    # f = 0: every harmonic column is the constant or zero; nothing beyond the mean is explained
    assert oracle.multiharmonic(t, y, 2, 0.0, 0.1, Nf=1)[0] == pytest.approx(0.0, abs=1e-12)


def _reduced_lstsq_power(t, y, w, cols):
    """Brute-force weighted fit of the constant plus the given columns."""
    sw = np.sqrt(w)
    A = np.stack([np.ones_like(t)] + cols, axis=1)
    coef, *_ = np.linalg.lstsq(A * sw[:, None], y * sw, rcond=None)
    chi2 = np.sum(w * (y - A @ coef) ** 2)
    Y = np.sum(w * y) / np.sum(w)
    return 1.0 - chi2 / np.sum(w * (y - Y) ** 2)


@pytest.mark.parametrize("K", [2, 3])
def test_mh_vanishing_columns_at_nyquist_drop_out(K):
    """Even sampling at the Nyquist frequency: sin(w t_j) is zero up to the
    rounding of the phase, and cos(2 w t_j) is the constant.  Such columns
    carry no information and drop out (pivot <= 1e-12 of the total weight, the
    rule of the generalized periodogram), so the power is the brute-force fit
    of the columns that remain (cos w t, and for K = 3 cos 3wt = cos wt: only
    one).  A rule relative to each column's own size would keep the rounding
    noise of the sine column and fit it."""
    g = np.random.default_rng([12, K])
    N, dt = 200, 0.01
    t = np.arange(N) * dt + 3.0
    y = 1.5 + np.sin(2 * np.pi * 7.3 * t) + g.normal(0, 0.7, N)
    w = g.uniform(0.5, 2.0, N)
    fn = 0.5 / dt
    p = oracle.multiharmonic(t, y, K, fn, 1.0, Nf=1, w=w)[0]
    ref = _reduced_lstsq_power(t, y, w, [np.cos(np.pi * np.arange(N))])
    assert p == pytest.approx(ref, rel=1e-9)
    # one harmonic is the generalized periodogram on every bin of an even grid
    # from f = 0 through the Nyquist frequency (degenerate bins included)
    df = fn / 64
    assert np.allclose(oracle.multiharmonic(t, y, 1, 0.0, df, Nf=70, w=w), oracle.gls(t, y, 0.0, df, Nf=70, w=w),
                       rtol=1e-9, atol=1e-13)
