"""Seeded synthetic light curves and frequency grids.

This module only draws inputs: sampling times, values and grid parameters.
It contains none of the periodogram arithmetic and is shared by the HIP
path's tests and benchmark and by the oracle's tests.  Every generator is
deterministic in its seed (numpy default_rng([10071658, config, sub])).

Workloads (times in days, frequencies in cycles per day):

  c0  plain method, one short curve: Nt = 1000 times uniform in [0, 100],
      sorted; x = sin(2 pi 0.37 t) + N(0, 0.5^2); df = 1/(4 T) with
      T = t_max - t_min (oversampling 4, high factor 1); f_min = df;
      Nf = 2000 (= 4 * 1 * Nt / 2, the grid rule of Section 4.3).
  c1  one long curve: 65,536 samples at 2-min cadence in on-segments of
      U[2, 12] d separated by gaps of U[0.5, 3] d (about 20 % gap duty),
      with N(0, (10 s)^2) timing jitter; x = sum of 5 sinusoids with
      frequencies U[1, 20] and amplitudes log-uniform in [1e-3, 1e-1], plus
      N(0, 1e-3^2) noise; df = 1/(4 T), f_min = df, Nf = 131,072.
  c2  precision stress: Nt = 100,000 times uniform over 3650 d after the
      epoch 2455000; x = sin(2 pi 13.7 (t - 2455000)) + N(0, 1);
      df = 50 / 2^20, f_min = df, Nf = 2^20 (up to 50 c/d).
  c3  Monte-Carlo batch: 4096 white-noise curves N(0, 1), Nt log-uniform in
      [200, 20000], own sorted times uniform over a baseline U[10, 1000] d,
      own grid df = 1/(4 T), f_min = df, Nf = 2 Nt.
  c4  sampling patterns for the false-alarm surrogate: Nt log-uniform in
      [200, 20000], baseline U[10, 1000] d, and one of three gap structures
      (none; random gaps covering a fraction U[0, 0.5] of the baseline with
      lengths log-uniform in [0.01 T, 0.2 T]; daily gaps with an observing
      fraction U[0.3, 0.7] of each day); grid df = 1/(4 T), f_min = df,
      Nf = 2 Nt.
  P   stand-in shaped like the paper's 150-d CoRoT series: Nt = 382,003 on a
      32-s grid with short random gaps, a dominant 0.18-d mode plus weaker
      terms plus noise; oversampling 4, high factor 2, Nf rounded up to a
      multiple of 256 (1,528,064).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED = 10071658


def rng(config: int, sub: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED, int(config), int(sub)])


@dataclasses.dataclass
class Curve:
    t: np.ndarray          # float64 [Nt]
    x: np.ndarray          # float32 [Nt]
    f_min: float
    df: float
    Nf: int
    name: str = ""

    @property
    def Nt(self) -> int:
        return int(self.t.size)

    @property
    def terms(self) -> int:
        return self.Nt * self.Nf


@dataclasses.dataclass
class Batch:
    t: np.ndarray          # float64 [sum Nt], CSR by off
    x: np.ndarray          # float32 [sum Nt]
    off: np.ndarray        # int64 [n+1]
    f_min: np.ndarray      # float64 [n]
    df: np.ndarray         # float64 [n]
    Nf: np.ndarray         # int64 [n]
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.off.size - 1)

    @property
    def Nt(self) -> np.ndarray:
        return np.diff(self.off)

    @property
    def terms(self) -> int:
        return int(np.sum(self.Nt * self.Nf))

    def curve(self, c: int) -> Curve:
        a, b = int(self.off[c]), int(self.off[c + 1])
        return Curve(self.t[a:b], self.x[a:b], float(self.f_min[c]), float(self.df[c]),
                     int(self.Nf[c]), f"{self.name}[{c}]")


def _baseline(t: np.ndarray) -> float:
    return float(t.max() - t.min())


def c0(seed_sub: int = 0, Nt: int = 1000, Nf: int | None = None) -> Curve:
    g = rng(0, seed_sub)
    t = np.sort(g.uniform(0.0, 100.0, Nt))
    x = (np.sin(2 * np.pi * 0.37 * t) + g.normal(0.0, 0.5, Nt)).astype(np.float32)
    df = 1.0 / (4.0 * _baseline(t))
    if Nf is None:
        Nf = 2 * Nt
    return Curve(t, x, df, df, int(Nf), "c0")


def gapped_cadence(g: np.random.Generator, Nt: int, cadence_d: float,
                   on_range=(2.0, 12.0), gap_range=(0.5, 3.0), jitter_d: float = 0.0) -> np.ndarray:
    """Regular cadence inside on-segments separated by random gaps, plus jitter."""
    out = []
    t0 = 0.0
    n = 0
    while n < Nt:
        on = g.uniform(*on_range)
        k = min(int(on / cadence_d), Nt - n)
        out.append(t0 + cadence_d * np.arange(k))
        n += k
        t0 += k * cadence_d + g.uniform(*gap_range)
    t = np.concatenate(out)[:Nt]
    if jitter_d > 0:
        t = t + g.normal(0.0, jitter_d, t.size)
    return np.sort(t)


def c1(seed_sub: int = 0, Nt: int = 65536, Nf: int = 131072) -> Curve:
    g = rng(1, seed_sub)
    t = gapped_cadence(g, Nt, 2.0 / 1440.0, jitter_d=10.0 / 86400.0)
    f = g.uniform(1.0, 20.0, 5)
    A = 10.0 ** g.uniform(-3.0, -1.0, 5)
    ph = g.uniform(0.0, 2 * np.pi, 5)
    x = np.zeros(Nt)
    for i in range(5):
        x += A[i] * np.sin(2 * np.pi * f[i] * t + ph[i])
    x = (x + g.normal(0.0, 1e-3, Nt)).astype(np.float32)
    df = 1.0 / (4.0 * _baseline(t))
    c = Curve(t, x, df, df, int(Nf), "c1")
    c.injected = f  # type: ignore[attr-defined]
    c.amplitudes = A  # type: ignore[attr-defined]
    return c


EPOCH = 2455000.0


def c2(seed_sub: int = 0, Nt: int = 100_000, Nf: int = 1 << 20, f_max: float = 50.0) -> Curve:
    g = rng(2, seed_sub)
    t = EPOCH + np.sort(g.uniform(0.0, 3650.0, Nt))
    x = (np.sin(2 * np.pi * 13.7 * (t - EPOCH)) + g.normal(0.0, 1.0, Nt)).astype(np.float32)
    df = f_max / Nf
    return Curve(t, x, df, df, int(Nf), "c2")


def c3(seed_sub: int = 0, n_curves: int = 4096, nt_range=(200, 20000),
       T_range=(10.0, 1000.0), f_over: float = 4.0) -> Batch:
    g = rng(3, seed_sub)
    Nt = np.rint(np.exp(g.uniform(math.log(nt_range[0]), math.log(nt_range[1]), n_curves))).astype(np.int64)
    T = g.uniform(T_range[0], T_range[1], n_curves)
    off = np.zeros(n_curves + 1, dtype=np.int64)
    off[1:] = np.cumsum(Nt)
    t = np.empty(int(off[-1]))
    x = np.empty(int(off[-1]), dtype=np.float32)
    df = np.empty(n_curves)
    for c in range(n_curves):
        a, b = off[c], off[c + 1]
        tc = np.sort(g.uniform(0.0, T[c], Nt[c]))
        t[a:b] = tc
        x[a:b] = g.normal(0.0, 1.0, Nt[c]).astype(np.float32)
        df[c] = 1.0 / (f_over * _baseline(tc))
    return Batch(t, x, off, df.copy(), df, 2 * Nt, "c3")


def _pattern_times(g: np.random.Generator, Nt: int, T: float, kind: int) -> np.ndarray:
    """Nt sorted times over [0, T] with gap structure `kind` (0 none, 1 random, 2 daily)."""
    if kind == 0:
        return np.sort(g.uniform(0.0, T, Nt))
    if kind == 1:
        duty = g.uniform(0.0, 0.5)
        # gap intervals until they cover about duty * T
        gaps = []
        covered = 0.0
        while covered < duty * T:
            L = math.exp(g.uniform(math.log(0.01 * T), math.log(0.2 * T)))
            a = g.uniform(0.0, T)
            gaps.append((a, a + L))
            covered += L
        keep = []
        while sum(len(k) for k in keep) < Nt:
            c = g.uniform(0.0, T, 2 * Nt)
            ok = np.ones(c.size, dtype=bool)
            for a, b in gaps:
                ok &= ~((c >= a) & (c < b))
            keep.append(c[ok])
        t = np.concatenate(keep)[:Nt]
        return np.sort(t)
    frac = g.uniform(0.3, 0.7)
    days = max(1, int(math.ceil(T)))
    d = g.integers(0, days, Nt)
    return np.sort(np.minimum(d + g.uniform(0.0, frac, Nt), T))


def c4_patterns(n: int = 2200, seed_sub: int = 0, nt_range=(200, 20000), T_range=(10.0, 1000.0)) -> Batch:
    """Sampling patterns of the surrogate workload (values are not used: zeros)."""
    g = rng(4, seed_sub)
    Nt = np.rint(np.exp(g.uniform(math.log(nt_range[0]), math.log(nt_range[1]), n))).astype(np.int64)
    T = g.uniform(T_range[0], T_range[1], n)
    kind = g.integers(0, 3, n)
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(Nt)
    t = np.empty(int(off[-1]))
    df = np.empty(n)
    for p in range(n):
        tp = _pattern_times(g, int(Nt[p]), float(T[p]), int(kind[p]))
        t[off[p]:off[p + 1]] = tp
        df[p] = 1.0 / (4.0 * _baseline(tp))
    b = Batch(t, np.zeros(t.size, dtype=np.float32), off, df.copy(), df, 2 * Nt, "c4")
    b.kind = kind  # type: ignore[attr-defined]
    return b


def subset(b: Batch, idx) -> Batch:
    """The curves idx of a batch, as a batch of their own (CSR rebuilt)."""
    idx = np.asarray(idx, dtype=np.int64)
    Nt = b.off[idx + 1] - b.off[idx]
    off = np.zeros(idx.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(Nt)
    t = np.concatenate([b.t[b.off[i]:b.off[i + 1]] for i in idx]) if idx.size else np.zeros(0)
    x = np.concatenate([b.x[b.off[i]:b.off[i + 1]] for i in idx]) if idx.size else np.zeros(0, np.float32)
    return Batch(t, x, off, b.f_min[idx].copy(), b.df[idx].copy(), b.Nf[idx].copy(), b.name + "-sub")


def paper_standin(seed_sub: int = 0) -> Curve:
    """Shape of the paper's CoRoT validation series (Section 5.2), synthetic."""
    g = rng(9, seed_sub)
    slots = 405_000
    cad = 32.0 / 86400.0
    keep = np.ones(slots, dtype=bool)
    removed = 0
    target = slots - 382_003
    while removed < target:
        a = int(g.integers(0, slots))
        L = int(min(g.integers(1, 200), target - removed))
        seg = keep[a:a + L]
        removed += int(seg.sum())
        keep[a:a + L] = False
    idx = np.nonzero(keep)[0]
    # trim any overshoot (gaps may overlap the end)
    idx = idx[:382_003]
    t = idx * cad + g.normal(0.0, 1.0 / 86400.0, idx.size)
    t = np.sort(t)
    f0 = 1.0 / 0.18
    x = np.sin(2 * np.pi * f0 * t)
    for f, a in ((7.1, 0.3), (3.2, 0.1), (11.3, 0.05)):
        x = x + a * np.sin(2 * np.pi * f * t + g.uniform(0, 2 * np.pi))
    x = (x + g.normal(0.0, 0.5, t.size)).astype(np.float32)
    T = _baseline(t)
    df = 1.0 / (4.0 * T)
    Nt = t.size
    Nf = int(math.ceil(2.0 * 4.0 * Nt / 2.0 / 256.0) * 256)
    return Curve(t, x, df, df, Nf, "paper_standin")


def even(N: int, dt: float = 1.0, t0: float = 0.0) -> np.ndarray:
    return t0 + dt * np.arange(N, dtype=np.float64)
