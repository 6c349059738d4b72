"""Pins of the oracle's extirpolation + FFT periodogram (Press & Rybicki 1989,
cited in Section 1).  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import extirp as E


@pytest.mark.parametrize("macc", [4, 6, 8])
def test_lagrange_weights_partition_unity_and_reproduce_polynomials(macc):
    u = np.random.default_rng(1).uniform(10, 1000, 500)
    n0, W = E.lagrange_weights(u, macc)
    assert np.allclose(W.sum(axis=1), 1.0, atol=1e-12)
    for p in range(1, macc):           # degree < macc polynomials are reproduced exactly
        pts = n0[:, None] + np.arange(macc)[None, :]
        assert np.allclose((W * (pts - 500.0) ** p).sum(axis=1), (u - 500.0) ** p, rtol=1e-9, atol=1e-6)


def test_on_grid_times_are_exact():
    # times on the grid: every sample lands on one point, the FFT is the exact sum
    N = 4096
    df = 1.0 / 50.0
    g = np.random.default_rng(2)
    n = np.sort(g.choice(N // 5, 300, replace=False))
    t = 3.0 + n / (df * N)
    x = np.sin(2 * np.pi * 0.37 * t) + g.normal(0, 0.5, t.size)
    P = E.periodogram_fast(t, x, df, df, 100, macc=4, N=N)
    ref = oracle.periodogram(t, x, df, df, Nf=100)
    assert np.allclose(P, ref, rtol=1e-9, atol=1e-9 * ref.max())


def test_single_sample_spreading_error_falls_with_order():
    # |FFT(spread)[k] - e^{-2 pi i k u / N}| shrinks as macc grows, for k well below N
    N, u = 1 << 12, 1234.37
    errs = []
    for macc in (4, 6, 8):
        F = np.fft.fft(E.extirpolate(np.array([u]), np.array([1.0]), N, macc))
        k = np.arange(1, N // (4 * 8))
        errs.append(np.max(np.abs(F[k] - np.exp(-2j * np.pi * k * u / N))))
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
    assert errs[0] < 1e-4


@pytest.mark.parametrize("macc,tol", [(4, 1e-4), (6, 1e-7), (8, 1e-9)])
def test_approximation_error_against_direct_sums(macc, tol):
    g = np.random.default_rng(3)
    t = np.sort(g.uniform(0, 100, 2000))
    x = np.sin(2 * np.pi * 1.7 * t) + g.normal(0, 1, t.size)
    df = 1.0 / (4 * (t[-1] - t[0]))
    P = E.periodogram_fast(t, x, df, df, 4000, macc=macc)
    ref = oracle.periodogram(t, x, df, df, Nf=4000)
    err = np.max(np.abs(P - ref)) / ref.max()
    assert err < tol
    assert np.argmax(P) == np.argmax(ref)
