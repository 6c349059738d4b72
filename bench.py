"""Throughput benchmark of the direct Lomb-Scargle periodogram on one MI355X.

One step = one full call of the hot path (normalization prep, the
periodogram kernel, split-axis reduction and FP64 epilogue) on one
synthetic light curve already resident in HBM.  Prints one JSON line.

Default workload: one long light curve, Nt = 65,536 samples at 2-min cadence
with gaps and jitter, 5 sinusoids + noise, Nf = 131,072 frequencies
(oversampling 4).  The split-precision path is the headline value; the plain
(naive FP32 phase) path is timed beside it.  The CPU baseline is the FP64
oracle on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Nt·Nf terms/s (split-FP32 vs plain) at max|ΔPn|≤1e-4; % FP32 VALU peak"
# The method's work per term, fixed before optimizing and the same for every
# kernel form: phase multiply, round and subtract (3), sin and cos (2), four
# multiply-adds into XC, XS, CC, CS (8).  Every roofline fraction below divides
# this work by the peak of the arithmetic the kernel actually runs on.
FLOP_PER_TERM = 13
PEAK_FP32_TFLOPS = 157.3    # MI355X FP32 vector peak (256 CU x 2.4 GHz)
PEAK_FP16_TFLOPS = 2500.0   # MI355X dense FP16 matrix peak
# what the matrix-core form issues per term (a secondary figure, not the
# method's work): per (a-row, b-column, sample) two complex products (XC + i XS
# and the double-angle sum), each four real products in three FP16 hi/lo
# passes, 24 multiply-adds, which serve the two frequencies F_a +- beta_b
MFMA_ISSUED_FLOP_PER_TERM = 24
REL_TOL = 1e-4

WORKLOADS = {
    "c1": ("single long light curve: Nt=65536 at 2-min cadence with 20% gaps and 10-s jitter, "
           "5 sinusoids (1-20 c/d, amplitudes 1e-3..1e-1) + 1e-3 noise, Nf=131072, oversampling 4"),
    "c0": "plain single light curve: Nt=1000 uniform in [0,100] d, 0.37 c/d sinusoid + noise, Nf=2000",
    "c2": ("precision stress: Nt=100000 over 3650 d after epoch 2455000 d, 13.7 c/d sinusoid + N(0,1), "
           "Nf=1048576 up to 50 c/d"),
    "paper": "paper-shaped stand-in: Nt=382003 on a 32-s grid over 150 d, Nf=1528064",
    "c3": ("batched Monte Carlo: 4096 white-noise curves, Nt log-uniform in [200, 20000], baselines "
           "U[10, 1000] d, Nf = 2 Nt each, one persistent launch (hipGraph), max Pn + argmax per curve"),
    "gls": ("generalized (floating-mean, weighted) periodogram on c1's sampling: Nt=65536, Nf=131072, "
            "weights U[0.5, 2]"),
    "mh": ("multi-harmonic periodogram, K = 2, on c1's sampling: Nt=65536, Nf=131072, weights U[0.5, 2]"),
    "mh4": ("multi-harmonic periodogram, K = 4 (two passes over the samples), on c1's sampling: Nt=65536, "
            "Nf=131072, weights U[0.5, 2]"),
    "fast": ("extirpolation + FFT approximation (Press & Rybicki), macc 4, on c1: Nt=65536, Nf=131072; "
             "Nt*Nf terms/s of the direct sums it replaces"),
}
# The weighted periodograms' work per term, by the same rule as FLOP_PER_TERM.
# Generalized: phase 3, sin and cos 2, w cos and w sin 4, (w y) cos and (w y) sin 4,
# w c then (w c) c and (w c) s 5: 18.  K harmonics: phase 3, sin and cos 2,
# 2K - 1 complex products by e^{i w t} (6 each), 2K weighted harmonic sums (4 each),
# K value sums (4 each): 24 K - 1.
GLS_FLOP_PER_TERM = 18
def MH_FLOP_PER_TERM(K):
    return 24 * K - 1
# what the matrix pipe issues per term: three complex products in three FP16
# passes (36 multiply-adds) per harmonic; half that per term for the
# conjugate-pair kernels (the multi-harmonic ones and the generalized
# periodogram's default), whose products serve two frequencies each
ISSUED_FLOP_PER_HARMONIC = 72


def make_curve(name):
    from paper_1007_1658_amd import synth
    return {"c0": synth.c0, "c1": synth.c1, "c2": synth.c2, "paper": synth.paper_standin}[name]()


def kernel_source_hash(kernel_name=""):
    in_mfma = "mfma" in kernel_name or kernel_name.startswith("gls_")
    name = "pgram_mfma.hip" if in_mfma else "pgram_kernels.hip"
    p = os.path.join(ROOT, "paper_1007_1658_amd", "csrc", name)
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def profile_entry(kernel_name, workload):
    """The committed rocprofv3 PMC summary entry for this kernel and workload,
    if it was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        with open(p) as f:
            d = json.load(f)
        e = d.get(f"{kernel_name}|{workload}")
        if not e or e.get("source_sha") != kernel_source_hash(kernel_name):
            return None
        return e
    except Exception:
        return None


def traffic_from_profiles(kernel_name, workload):
    """HBM bytes per launch (PMC FETCH_SIZE/WRITE_SIZE, copy-calibrated), or None."""
    e = profile_entry(kernel_name, workload)
    return float(e["bytes_per_launch"]) if e and "bytes_per_launch" in e else None


def warm(fn, warmup, min_seconds=0.3):
    """W untimed steps, continued until the GPU has been busy min_seconds (clocks settle)."""
    import torch
    t0 = time.perf_counter()
    n = 0
    while n < warmup or time.perf_counter() - t0 < min_seconds:
        fn()
        n += 1
        if n % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()


def time_steps(fn, steps, warmup, on_start=None):
    """Seconds per step over exactly `steps` steps after `warmup` untimed ones
    (host clock, the stream synchronized on both sides; nothing is recorded
    on the stream between the steps).  on_start runs after the warm-up, e.g.
    to enable the library's profiling hook for the pass."""
    import torch
    warm(fn, warmup)
    if on_start:
        on_start()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


KERNEL_TIMING = ("HIP events attached to the kernel's launches, in a second pass of the same steps "
                 "(the value's pass records none)")


def profiled_passes(fn, steps, calls=True):
    """After the value's timed pass: one more pass of `steps` steps with the
    main kernel's events (its average duration, symbol name) and, for
    single-curve calls, one with each call's events (its device span).
    Events attached to the launches add no commands to the stream but still
    delay each call (about 5 us per pair on a c1 call), so every figure comes
    from a pass that carries only its own events."""
    import paper_1007_1658_amd as lsp
    time_steps(fn, steps, 0, on_start=lambda: lsp.lsp_profile_enable(lsp.PROFILE_KERNEL))
    k_ms, k_n, k_name = lsp.lsp_profile_read()
    span = None
    if calls:
        time_steps(fn, steps, 0, on_start=lambda: lsp.lsp_profile_enable(lsp.PROFILE_CALLS))
        span = lsp.lsp_profile_read_calls()
    lsp.lsp_profile_enable(False)
    return k_ms / 1e3 / max(k_n, 1), k_name, span


def step_stats(ms, what=None):
    a = np.asarray(ms, dtype=np.float64)
    out = {"n": int(a.size), "median_ms": float(np.median(a)), "mean_ms": float(a.mean()),
           "std_ms": float(a.std(ddof=1)) if a.size > 1 else 0.0,
           "min_ms": float(a.min()), "max_ms": float(a.max())}
    if what:
        out["of"] = what
    return out


CALL_TIME = ("device time of each call, its first kernel's start to its last kernel's end (HIP events on "
             "those launches, in a third pass of the same steps)")


def sampled_error(curve, Pg, n=256, seed=0):
    import oracle
    g = np.random.default_rng(seed)
    kpk = int(np.argmax(Pg))
    k = np.unique(np.concatenate([g.integers(0, curve.Nf, n),
                                  np.arange(max(0, kpk - 4), min(curve.Nf, kpk + 5))]))
    P = oracle.periodogram(curve.t, curve.x, curve.f_min, curve.df, k=k)
    return float(np.max(np.abs(Pg[k].astype(np.float64) - P)) / P.max())


def cpu_baseline(curve, target_s):
    """The oracle as it stands, on all host cores, over a frequency subset."""
    import oracle
    cores = oracle.max_threads()
    g = np.random.default_rng(7)
    # two calibration probes (the first, 64 frequencies, is dominated by start-up;
    # the second is at most 16x larger), then the timed subset sized to target_s
    nb = min(curve.Nf, 64)
    for growth_cap in (16.0, None):
        k = np.sort(g.choice(curve.Nf, size=nb, replace=False))
        t0 = time.perf_counter()
        oracle.periodogram(curve.t, curve.x, curve.f_min, curve.df, k=k)
        scale = target_s / max(time.perf_counter() - t0, 1e-3)
        if growth_cap is not None:
            scale = min(scale, growth_cap)
        nb = int(min(curve.Nf, max(64, nb * scale)))
    k = np.sort(g.choice(curve.Nf, size=nb, replace=False))
    t0 = time.perf_counter()
    oracle.periodogram(curve.t, curve.x, curve.f_min, curve.df, k=k)
    el = time.perf_counter() - t0
    return {
        "value": curve.Nt * nb / el,
        "unit": "terms/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"FP64 two-pass oracle over all Nt={curve.Nt} samples at {nb} of the {curve.Nf} "
                   f"frequencies (random subset), {el:.1f} s on {cores} threads"),
        "one_thread": one_thread_baseline(curve),
    }


def one_thread_baseline(curve):
    """The oracle on one host thread: c0 in full (5 runs, mean and sigma, as the
    paper averages five runs) and 128 random frequencies of this workload."""
    import oracle
    from paper_1007_1658_amd import synth
    c0 = synth.c0()
    runs = []
    for _ in range(5):
        t0 = time.perf_counter()
        oracle.periodogram(c0.t, c0.x, c0.f_min, c0.df, Nf=c0.Nf, threads=1)
        runs.append(time.perf_counter() - t0)
    r = np.asarray(runs)
    k = np.sort(np.random.default_rng(8).choice(curve.Nf, size=min(128, curve.Nf), replace=False))
    t0 = time.perf_counter()
    oracle.periodogram(curve.t, curve.x, curve.f_min, curve.df, k=k, threads=1)
    el = time.perf_counter() - t0
    return {"c0_terms_per_s": c0.Nt * c0.Nf / r.mean(), "c0_seconds_mean": float(r.mean()),
            "c0_seconds_std": float(r.std(ddof=1)),
            "subset_terms_per_s": curve.Nt * k.size / el,
            "subset": f"{k.size} random frequencies x all {curve.Nt} samples, {el:.2f} s"}


def calib_copy(mib):
    """A plain copy of known size: reads and writes mib MiB once per launch (5 launches)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": n * 4, "launches": 5}), flush=True)


def microbench():
    """Lane-operation rates of the instruction classes that bound the kernel."""
    import torch
    import paper_1007_1658_amd as lsp
    torch.cuda.init()
    torch.empty(1, device="cuda")
    names = ["fp32_fma", "fp64_fma", "sin+cos pair", "fp64 phase reduction"]
    res = {}
    for kind, name in enumerate(names):
        for w in (1, 2, 4, 8):
            ops, ms = lsp.lsp_microbench(kind, w, 2048)
            res[f"{name}@{w}"] = ops
    # matrix pipe alone and with 4 / 8 / 16 vector FMAs per MFMA, at 1 and 2 waves per
    # SIMD (MFMA FLOP/s), and the 16-FMA stream alone (FMA/s)
    co = {}
    for w in (1, 2):
        for kind, name in ((4, "mfma"), (5, "mfma+4fma"), (6, "mfma+8fma"), (7, "mfma+16fma"), (8, "16fma")):
            ops, ms = lsp.lsp_microbench(kind, w, 1024)
            co[f"{name}@{w}"] = {"ops_per_s": ops, "ms": ms}
    print(json.dumps({"microbench_lane_ops_per_s": res, "mfma_coissue": co}), flush=True)


def run_batched(args):
    """c3: throughput and per-curve latency of the batched persistent launch."""
    import torch
    import paper_1007_1658_amd as lsp
    from paper_1007_1658_amd import synth
    if args.batched_form:
        lsp.lsp_set_batched_form(args.batched_form)
    mfma = lsp.lsp_get_batched_form() == "mfma"
    b = synth.c3()
    t = torch.from_numpy(b.t).cuda()
    x = torch.from_numpy(b.x).cuda()
    out = lsp.lsp_periodogram_batched(t, x, b.off, b.f_min, b.df, b.Nf, want_times=True)
    torch.cuda.synchronize()

    def step():
        lsp.lsp_periodogram_batched(t, x, b.off, b.f_min, b.df, b.Nf, want_times=True, out=out)

    sec = time_steps(step, args.steps, args.warmup)
    tns = out["t_ns"].cpu().numpy().reshape(-1, 2).astype(np.float64)
    lat_run = (tns[:, 1] - tns[:, 0]) * 1e-6          # first item start -> last item end, ms
    lat_done = tns[:, 1] * 1e-6                        # launch start -> curve complete, ms
    terms = b.terms
    # parity on a stratified subset of curves (argmax and peak power vs the oracle)
    import oracle
    pmax = out["pmax"].cpu().numpy()
    kbest = out["kbest"].cpu().numpy()
    order = np.argsort(b.Nt)
    worst = 0.0
    for c in order[np.linspace(0, b.n - 1, 8).astype(int)]:
        cv = b.curve(int(c))
        k = np.unique(np.clip(np.arange(kbest[c] - 1, kbest[c] + 2), 0, cv.Nf - 1))
        P = oracle.periodogram(cv.t, cv.x, cv.f_min, cv.df, k=k)
        i = int(np.nonzero(k == kbest[c])[0][0])
        worst = max(worst, abs(pmax[c] - P[i]) / P.max())
    line = {
        "metric": METRIC + " [batched]", "value": terms / sec, "unit": "terms/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f16x3/f32" if mfma else "f32", "data": "synthetic",
        "config": {"workload": WORKLOADS["c3"], "name": "c3", "curves": b.n, "terms": terms,
                   "form": lsp.lsp_get_batched_form()},
        "latency_ms": {"run_p50": float(np.percentile(lat_run, 50)), "run_p99": float(np.percentile(lat_run, 99)),
                       "done_p50": float(np.percentile(lat_done, 50)), "done_p99": float(np.percentile(lat_done, 99))},
        "peak_rel_err_sampled": worst,
        "roofline": ({"bound": "mfma", "achieved": FLOP_PER_TERM * terms / sec / 1e12, "peak": PEAK_FP16_TFLOPS,
                      "unit": "TFLOP/s", "frac": FLOP_PER_TERM * terms / sec / 1e12 / PEAK_FP16_TFLOPS,
                      "flop_per_term": FLOP_PER_TERM, "traffic": None, "kernel": "batch_mfma_kernel (whole graph)",
                      "mfma_issued_frac": MFMA_ISSUED_FLOP_PER_TERM * terms / sec / 1e12 / PEAK_FP16_TFLOPS}
                     if mfma else
                     {"bound": "alu", "achieved": FLOP_PER_TERM * terms / sec / 1e12, "peak": PEAK_FP32_TFLOPS,
                      "unit": "TFLOP/s", "frac": FLOP_PER_TERM * terms / sec / 1e12 / PEAK_FP32_TFLOPS,
                      "flop_per_term": FLOP_PER_TERM, "traffic": None,
                      "kernel": "batch_pgram_kernel (whole graph)"}),
    }
    print(json.dumps(line), flush=True)


def run_gls(args):
    """The generalized periodogram (lsp_gls, or lsp_multiharmonic with K = 2 for
    --config mh) on c1's sampling with weights; not the headline."""
    import torch
    import oracle
    import paper_1007_1658_amd as lsp
    from paper_1007_1658_amd import synth
    c = synth.c1()
    w = np.random.default_rng(4).uniform(0.5, 2.0, c.Nt).astype(np.float32)
    t = torch.from_numpy(c.t).cuda()
    y = torch.from_numpy(c.x).cuda()
    wd = torch.from_numpy(w).cuda()
    p = torch.empty(c.Nf, dtype=torch.float32, device="cuda")

    mh = args.config in ("mh", "mh4")
    K = 4 if args.config == "mh4" else 2

    def step():
        if mh:
            lsp.lsp_multiharmonic(t, y, K, c.f_min, c.df, c.Nf, w=wd, p=p)
        else:
            lsp.lsp_gls(t, y, c.f_min, c.df, c.Nf, w=wd, p=p)

    step()
    torch.cuda.synchronize()
    pg = p.cpu().numpy()
    g = np.random.default_rng(0)
    kpk = int(np.argmax(pg))
    k = np.unique(np.concatenate([g.integers(0, c.Nf, 256), np.arange(max(0, kpk - 4), min(c.Nf, kpk + 5)),
                                  np.arange(0, 8)]))
    if mh:
        P = oracle.multiharmonic(c.t, c.x.astype(np.float64), K, c.f_min, c.df, k=k, w=w.astype(np.float64))
    else:
        P = oracle.gls(c.t, c.x.astype(np.float64), c.f_min, c.df, k=k, w=w.astype(np.float64))
    err = float(np.max(np.abs(pg[k] - P)) / P.max())
    sec = time_steps(step, args.steps, args.warmup)
    k_avg_s, k_name, _ = profiled_passes(step, args.steps, calls=False)
    terms = c.Nt * c.Nf
    flop = MH_FLOP_PER_TERM(K) if mh else GLS_FLOP_PER_TERM
    issued = ISSUED_FLOP_PER_HARMONIC * (K if mh else 1) // (2 if (mh or k_name == "gls_pm_kernel") else 1)
    achieved = flop * terms / k_avg_s / 1e12
    line = {
        "metric": (f"Nt·Nf terms/s of the multi-harmonic (K={K}) periodogram at max|Δp|≤1e-4" if mh else
                   "Nt·Nf terms/s of the generalized periodogram at max|Δp|≤1e-4"), "value": terms / sec,
        "unit": "terms/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16x3/f32", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "name": args.config, "Nt": c.Nt, "Nf": c.Nf},
        "max_rel_err": err, "meets_1e-4": bool(err <= REL_TOL),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP16_TFLOPS, "traffic": traffic_from_profiles(k_name, args.config),
                     "kernel": k_name, "kernel_avg_ms": k_avg_s * 1e3, "kernel_timing": KERNEL_TIMING,
                     "flop_per_term": flop,
                     "mfma_issued": {"flop_per_term": issued,
                                     "frac": issued * terms / k_avg_s / 1e12 / PEAK_FP16_TFLOPS}},
    }
    print(json.dumps(line), flush=True)


def run_fast(args):
    """The extirpolation + FFT approximation on c1 (not the headline): time per
    call, its error against the direct GPU path and against the FP64 oracle."""
    import torch
    import paper_1007_1658_amd as lsp
    from paper_1007_1658_amd import synth
    c = synth.c1()
    t = torch.from_numpy(c.t).cuda()
    x = torch.from_numpy(c.x).cuda()
    p = torch.empty(c.Nf, dtype=torch.float32, device="cuda")

    def step():
        lsp.lsp_periodogram_fast(t, x, c.f_min, c.df, c.Nf, macc=4, Pn=p)

    step()
    torch.cuda.synchronize()
    err = sampled_error(c, p.cpu().numpy())
    sec = time_steps(step, args.steps, args.warmup)
    line = {
        "metric": "Nt·Nf terms/s (equivalent) of the extirpolation+FFT approximation, macc 4",
        "value": c.Nt * c.Nf / sec, "unit": "terms/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic", "config": {"workload": WORKLOADS["fast"], "name": "fast", "Nt": c.Nt, "Nf": c.Nf},
        "max_rel_err_vs_direct_oracle": err, "meets_1e-4": bool(err <= REL_TOL),
        "roofline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c1", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-tune", action="store_true", help="use the heuristic launch shape")
    ap.add_argument("--form", default="auto", choices=["auto", "valu"],
                    help="auto: the library's (tuned) choice, the matrix-core form on MI355X; "
                         "valu: time the FP32-VALU form (frequency recurrence) instead")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--batched-form", default="", choices=["", "mfma", "recur"],
                    help="c3: kernel form of the batched path (default: the library's, matrix cores)")
    ap.add_argument("--save-tune", default="", help="write the tuner cache to this JSON file")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (HBM counter calibration)")
    ap.add_argument("--microbench", action="store_true",
                    help="only print the gfx950 instruction-throughput table (FP32/FP64 FMA, sin+cos, FP64 phase)")
    args = ap.parse_args()
    if args.calib_copy:
        calib_copy(args.calib_copy)
        return
    if args.microbench:
        microbench()
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the periodogram would shard by frequency, each GPU taking Nf/G bins after a "
              "broadcast of t and x)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1007_1658_amd as lsp

    assert torch.cuda.is_available(), "no GPU"
    if args.config == "c3":
        run_batched(args)
        return
    if args.config in ("gls", "mh", "mh4"):
        run_gls(args)
        return
    if args.config == "fast":
        run_fast(args)
        return
    curve = make_curve(args.config)
    t = torch.from_numpy(curve.t).cuda()
    x = torch.from_numpy(curve.x).cuda()
    Pn = torch.empty(curve.Nf, dtype=torch.float32, device="cuda")

    # launch shapes: the committed tuner cache, else tune now (outside the timed region)
    if os.path.exists(lsp.TUNE_CACHE):
        lsp.lsp_tune_cache_load(lsp.TUNE_CACHE)
    tile = None
    if not args.no_tune:
        for ph in ("split", "naive"):
            if lsp.lsp_tune_lookup(curve.Nt, curve.Nf, ph) is None:
                lsp.lsp_autotune(curve.Nt, curve.Nf, ph)
        tile = lsp.lsp_tune_lookup(curve.Nt, curve.Nf, "split")
        if args.save_tune:
            lsp.lsp_tune_cache_save(args.save_tune)

    # the VALU form's fastest whole call on c1 in sweeps of the built recurrence
    # shapes (M, unroll, summation, waves, splits in steps of 4): two-level FP32
    # sums, whose error on c1 matches the compensated ones (both ~2e-6 of the
    # sampled max); 72 splits of 37 frequency tiles fill the CUs in whole rounds
    valu_kw = dict(trig="recur", m=14, unroll=2, sum="two", waves=4, splits=72 if curve.Nt >= 1 << 15 else 0)
    if args.form == "valu":
        # the FP32-VALU form as the timed line (frequency recurrence)
        tile = {"trig": lsp.LSP_TRIG_RECUR, "m": 14, "waves": 4, "splits": valu_kw["splits"], "unroll": 2,
                "sum": lsp.LSP_SUM_TWO}

        def run_split():
            lsp.lsp_periodogram_ex(t, x, curve.f_min, curve.df, curve.Nf, Pn=Pn, **valu_kw)
    else:
        def run_split():
            lsp.lsp_periodogram(t, x, curve.f_min, curve.df, curve.Nf, Pn=Pn)

    # accuracy of the exact configuration that is timed
    run_split()
    torch.cuda.synchronize()
    err_split = sampled_error(curve, Pn.cpu().numpy())

    # the value's pass records nothing on the stream; the main kernel's
    # duration and each call's span come from passes of the same steps
    sec = time_steps(run_split, args.steps, args.warmup)
    k_avg_s, k_name, steps_ms = profiled_passes(run_split, args.steps)
    terms = curve.Nt * curve.Nf
    value = terms / sec

    plain = None
    if not args.no_plain:
        Pp = torch.empty_like(Pn)

        def run_plain():
            lsp.lsp_periodogram_ex(t, x, curve.f_min, curve.df, curve.Nf, Pn=Pp, phase="naive")

        run_plain()
        torch.cuda.synchronize()
        err_plain = sampled_error(curve, Pp.cpu().numpy())
        sec_p = time_steps(run_plain, max(5, args.steps // 2), 2)
        plain = {"value": terms / sec_p, "ms_per_step": sec_p * 1e3, "max_rel_err": err_plain,
                 "meets_1e-4": bool(err_plain <= REL_TOL)}

    # the FP32-VALU form beside it (frequency recurrence, two-level sums; the
    # shape the sweeps found best on c1), priced against the FP32 vector peak
    valu = None
    if not args.no_plain and args.form != "valu":
        Pv = torch.empty_like(Pn)

        def run_valu():
            lsp.lsp_periodogram_ex(t, x, curve.f_min, curve.df, curve.Nf, Pn=Pv, **valu_kw)

        run_valu()
        torch.cuda.synchronize()
        err_v = sampled_error(curve, Pv.cpu().numpy())
        v_steps = max(40, args.steps)
        sec_v = time_steps(run_valu, v_steps, 2)
        kv_s, kv_name, v_ms = profiled_passes(run_valu, v_steps)
        ach_v = FLOP_PER_TERM * terms / kv_s / 1e12
        valu = {"value": terms / sec_v, "ms_per_step": sec_v * 1e3, "step_stats": step_stats(v_ms, CALL_TIME),
                "kernel": kv_name, "kernel_avg_ms": kv_s * 1e3,
                "frac_fp32_valu_peak": ach_v / PEAK_FP32_TFLOPS,
                "frac_fp32_valu_peak_whole_call": FLOP_PER_TERM * terms / sec_v / 1e12 / PEAK_FP32_TFLOPS,
                "roofline": {"bound": "alu", "achieved": ach_v, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                             "frac": ach_v / PEAK_FP32_TFLOPS, "flop_per_term": FLOP_PER_TERM,
                             "kernel_timing": KERNEL_TIMING,
                             "traffic": traffic_from_profiles(kv_name, args.config)},
                "max_rel_err": err_v, "meets_1e-4": bool(err_v <= REL_TOL)}

    # latency of one small call (c0: Nt 1000, Nf 2000), host to host: the launch-
    # bound end of the range, where the paper's GPUs also paid a fixed cost
    c0_latency = None
    if args.config == "c1" and not args.no_plain:
        from paper_1007_1658_amd import synth
        c0 = synth.c0()
        t0d, x0d = torch.from_numpy(c0.t).cuda(), torch.from_numpy(c0.x).cuda()
        P0 = torch.empty(c0.Nf, dtype=torch.float32, device="cuda")
        lat = []
        for i in range(60):
            torch.cuda.synchronize()
            h0 = time.perf_counter()
            lsp.lsp_periodogram(t0d, x0d, c0.f_min, c0.df, c0.Nf, Pn=P0)
            torch.cuda.synchronize()
            if i >= 10:
                lat.append((time.perf_counter() - h0) * 1e3)
        c0_latency = step_stats(lat)

    mfma = "mfma" in k_name
    peak = PEAK_FP16_TFLOPS if mfma else PEAK_FP32_TFLOPS
    # the method's 13 FLOP per term over the kernel's time, against the peak of
    # the arithmetic the kernel runs on (FP16 matrix cores or FP32 vector)
    achieved = FLOP_PER_TERM * terms / k_avg_s / 1e12
    traffic = traffic_from_profiles(k_name, args.config)
    roof = {
        "bound": "mfma" if mfma else "alu",
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": traffic,
        "kernel": k_name,
        "kernel_avg_ms": k_avg_s * 1e3,
        "kernel_timing": KERNEL_TIMING,
        "flop_per_term": FLOP_PER_TERM,
    }
    if mfma:
        # what the matrix pipe issues per term (MFMA_ISSUED_FLOP_PER_TERM)
        issued = MFMA_ISSUED_FLOP_PER_TERM * terms / k_avg_s / 1e12
        roof["mfma_issued"] = {"flop_per_term": MFMA_ISSUED_FLOP_PER_TERM, "achieved": issued,
                               "frac": issued / PEAK_FP16_TFLOPS}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "step_stats": step_stats(steps_ms, CALL_TIME),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # matrix-core form: FP16 hi/lo products (three passes) with FP32 accumulation
        "dtype": "f16x3/f32" if mfma else "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "name": args.config, "Nt": curve.Nt, "Nf": curve.Nf,
                   "phase": "split", "tile": tile},
        "max_rel_err": err_split,
        "meets_1e-4": bool(err_split <= REL_TOL),
        "plain": plain,
        "valu_form": valu,
        "roofline": roof,
        "cpu_baseline": None if args.no_cpu else cpu_baseline(curve, args.cpu_seconds),
        "c0_call_latency_ms": c0_latency,
    }
    if args.config == "paper":
        # the paper's own timing of this shape (Table 2: 20.3 s on a Tesla C1060, FP32,
        # the V1449 Aql series this synthetic stand-in imitates); context only
        line["paper_context"] = {"hardware": "Tesla C1060 (GT200)", "seconds": 20.3,
                                 "terms_per_s": 382003 * 1528064 / 20.3, "speedup_here": 20.3 / sec}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
