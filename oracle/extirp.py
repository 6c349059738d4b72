"""Fast approximate Lomb-Scargle periodogram by extirpolation and FFT
(Press & Rybicki 1989, the approach Section 1 cites) -- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy, written from the method's definition, not from any GPU code:
  1. centre x (x - mean) and take the population variance (Section 3);
  2. map every time onto a periodic grid of N points whose period is 1/df:
     u_j = (t_j - t_min) df N (grid units), so that e^{2 pi i k df (t_j - t_min)}
     = e^{2 pi i k u_j / N};
  3. extirpolate: add x_j to the `macc` grid points nearest u_j, weighted by
     those points' Lagrange basis polynomials evaluated at u_j (the transpose
     of Lagrange interpolation, so sum_n g_n phi(n) ~ sum_j x_j phi(u_j) for
     any smooth periodic phi); add 1 likewise at 2 u_j (mod N), for the sums
     at twice the angle;
  4. forward FFT of both grids: bin k gives sum_j x_j e^{-2 pi i k u_j / N}
     = XC - i XS and sum_j e^{-4 pi i k u_j / N} = C2 - i S2 at f = k df;
  5. Pn by Eqs. (5)-(7) with CC = (Nt + C2) / 2, CS = S2 / 2, SS = Nt - CC.
The approximation error comes from step 3 only; it falls as the grid gets
finer relative to the highest frequency (N >= 4 macc k_max here).
"""
import numpy as np


def grid_size(k_max: int, macc: int) -> int:
    """Smallest power of two >= 4 macc k_max (k_max >= 1): 2 macc grid points
    per period of the highest frequency the double-angle sums need, 2 k_max df,
    as Press & Rybicki size the grid."""
    need = 4 * macc * max(int(k_max), 1)
    n = 1
    while n < need:
        n <<= 1
    return n


def lagrange_weights(u, macc):
    """First grid point and the macc Lagrange weights of the points
    n0, ..., n0 + macc - 1 around each u (n0 = floor(u) - macc/2 + 1)."""
    u = np.asarray(u, dtype=np.float64)
    fl = np.floor(u)
    n0 = fl.astype(np.int64) - (macc // 2 - 1)
    s = u - n0  # position relative to n0, in [macc/2 - 1, macc/2)
    W = np.ones((u.size, macc))
    for m in range(macc):
        for l in range(macc):
            if l != m:
                W[:, m] *= (s - l) / (m - l)
    return n0, W


def extirpolate(u, v, N, macc):
    """Grid of N points with each value v_j spread around u_j (periodic)."""
    g = np.zeros(N)
    n0, W = lagrange_weights(u, macc)
    idx = (n0[:, None] + np.arange(macc)[None, :]) % N
    np.add.at(g, idx.ravel(), (W * np.asarray(v, dtype=np.float64)[:, None]).ravel())
    return g


def periodogram_fast(t, x, f_min, df, Nf, macc=4, N=None):
    """Pn at f_k = f_min + k df, k < Nf; f_min must be a whole multiple of df."""
    t = np.asarray(t, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    m0 = int(round(f_min / df))
    if abs(m0 * df - f_min) > 1e-9 * max(df, abs(f_min)):
        raise ValueError("f_min must be a whole multiple of df")
    k_max = m0 + int(Nf) - 1
    if N is None:
        N = grid_size(k_max, macc)
    Nt = t.size
    xc = x - x.mean()
    var = np.mean(xc * xc)
    u = (t - t.min()) * df * N
    gx = extirpolate(u, xc, N, macc)
    g1 = extirpolate(np.mod(2.0 * u, N), np.ones(Nt), N, macc)
    Fx = np.fft.fft(gx)[m0:m0 + Nf]
    F1 = np.fft.fft(g1)[m0:m0 + Nf]
    XC, XS = Fx.real, -Fx.imag
    C2, S2 = F1.real, -F1.imag
    CC = 0.5 * (Nt + C2)
    CS = 0.5 * S2
    SS = Nt - CC
    two_wt = np.where((CS == 0) & (CC - SS == 0), 0.0, np.arctan2(2 * CS, CC - SS))
    st, ct = np.sin(0.5 * two_wt), np.cos(0.5 * two_wt)
    Dc = ct * ct * CC + 2 * ct * st * CS + st * st * SS
    Ds = ct * ct * SS - 2 * ct * st * CS + st * st * CC
    a = ct * XC + st * XS
    b = ct * XS - st * XC
    fl = 1e-12 * Nt
    P = 0.5 * (np.where(Dc > fl, a * a / np.where(Dc > fl, Dc, 1), 0) + np.where(Ds > fl, b * b / np.where(Ds > fl, Ds, 1), 0))
    return P / var
