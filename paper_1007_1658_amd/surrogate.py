"""Training and validation of the false-alarm surrogate (the training driver).

Every step of serving a FAP runs in the library (lsp_fap_surrogate: window
features, the network, the law, the per-pattern error bound and the
Monte-Carlo fallback), and so does every step of training that touches the
data at scale: Monte-Carlo maxima (lsp_mc_maxpower), window features
(lsp_window_features), the network's forward, loss, backward and Adam
(lsp_mlp_grad, lsp_mlp_adam_step).  This module chooses minibatches,
learning rates and chunk sizes, and it computes, once per trained model, a
few numbers that the model file then carries: the feature standardization
and the head's location scale (fit_scalers, moments of the training data),
and the calibrated law error (calibrate, set by coverage of held-out
residuals).  These are model-building arithmetic of the driver;
none of it runs when a FAP is served.

    python -m paper_1007_1658_amd.surrogate --out model.bin --report report.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import Model, lsp_fap_analytic, lsp_mc_maxpower, lsp_window_features
from . import synth

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(_HERE, "fap_model", "fap_surrogate_gfx950.bin")
FAP_LEVELS = (0.001, 0.01, 0.05, 0.1)


def _torch():
    import torch
    return torch


def _device_t(b: synth.Batch):
    return _torch().from_numpy(np.ascontiguousarray(b.t)).cuda()


def monte_carlo(b: synth.Batch, R: int, seed: int, stream_base: int = 0, max_values: int = 1 << 28):
    """max Pn of R white-noise realizations on each pattern of b: device [n, R].

    Patterns are processed in chunks holding at most max_values drawn values;
    pattern p uses counter streams stream_base + p R + r whatever the chunking.
    """
    torch = _torch()
    out = torch.empty((b.n, R), dtype=torch.float32, device="cuda")
    p0 = 0
    while p0 < b.n:
        p1 = p0 + 1
        while p1 < b.n and (b.off[p1 + 1] - b.off[p0]) * R <= max_values:
            p1 += 1
        sub = synth.subset(b, np.arange(p0, p1))
        lsp_mc_maxpower(_device_t(sub), sub.off, sub.f_min, sub.df, sub.Nf, R, seed,
                        stream_base=stream_base + p0 * R, out=out[p0:p1])
        p0 = p1
    return out


def features(b: synth.Batch):
    return lsp_window_features(_device_t(b), b.off, b.f_min, b.df, b.Nf)


def law_targets(F: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """w(y) - ln Nf of every Monte-Carlo maximum, w(z) = -((Nt-3)/2) ln(1 - 2z/Nt),
    with Nt and Nf read from the raw features as the library reads them."""
    F = np.asarray(F, dtype=np.float64)
    nt = np.rint(10.0 ** F[:, 64])[:, None]
    nf = np.rint(10.0 ** F[:, 67])[:, None]
    return -((nt - 3.0) / 2.0) * np.log1p(-2.0 * np.asarray(Y, dtype=np.float64) / nt) - np.log(nf)


def fit_scalers(F: np.ndarray, Y: np.ndarray):
    """Feature standardization, the accepted feature range and the head's
    location scale (moment estimates of the Gumbel location and of the spread
    of the targets)."""
    mean = F.mean(axis=0)
    std = np.maximum(F.std(axis=0), 1e-3)
    zmax = float(np.abs((F - mean) / std).max()) * 1.25
    W = law_targets(F, Y)
    beta = W.std() * np.sqrt(6.0) / np.pi
    return mean, std, zmax, float(W.mean() - 0.5772156649 * beta), float(W.std())


def train(F, Y, members=4, steps=1500, batch=256, lr=2e-3, seed=0, holdout=0.1, eval_every=50, log=None):
    """Fits an ensemble on device features F [n, 68] and maxima Y [n, R].

    A seeded `holdout` fraction of the patterns is kept out of the minibatches;
    every `eval_every` steps its loss is measured and each member keeps the
    parameters of its best held-out loss (early stopping)."""
    torch = _torch()
    n = F.shape[0]
    perm = np.random.default_rng([seed, 99]).permutation(n)
    n_ho = int(round(holdout * n)) if holdout > 0 else 0
    tr_idx, ho_idx = perm[n_ho:], perm[:n_ho]
    Fh, Yh = F.cpu().numpy().astype(np.float64), Y.cpu().numpy()
    mean, std, zmax, mu, sig = fit_scalers(Fh[tr_idx], Yh[tr_idx])
    model = Model(members=members, seed=seed)
    model.set_scalers(mean, std, zmax, mu, sig)
    if n_ho:
        ho = torch.from_numpy(ho_idx).cuda()
        F_ho, Y_ho = F.index_select(0, ho).contiguous(), Y.index_select(0, ho).contiguous()
    history = []
    for e in range(members):
        g = np.random.default_rng([seed, e])
        best = (math.inf, None, -1)
        for step in range(steps + 1):
            if n_ho and (step % eval_every == 0 or step == steps):
                _, hl = model.grad(e, F_ho, Y_ho, want_grad=False)
                hl = float(hl.item())
                if hl < best[0]:
                    best = (hl, model.get_params(e), step)
            if step == steps:
                break
            idx = torch.from_numpy(tr_idx[g.choice(tr_idx.size, size=min(batch, tr_idx.size), replace=False)]).cuda()
            fb = F.index_select(0, idx).contiguous()
            yb = Y.index_select(0, idx).contiguous()
            _, loss = model.grad(e, fb, yb, want_grad=False)
            lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * step / steps)) + 1e-5
            model.adam_step(e, lr_t)
            if log is not None and (step % 250 == 0 or step == steps - 1):
                log(f"member {e} step {step} loss {float(loss.item()):.5f} held-out best {best[0]:.5f} at {best[2]}")
        if best[1] is not None:
            model.set_params(e, best[1])
        history.append({"member": e, "best_step": best[2], "heldout_loss": best[0]})
    return model, history


CAL_LEVELS = (0.001, 0.003, 0.01, 0.02, 0.05, 0.1, 0.2)
Z99 = 2.5758293035489   # standard errors in the library's error bound (two-sided 99 %)


def law_sensitivity(model, td, b: synth.Batch, p_obs):
    """(fap, spread, dFAP/dm, dFAP/dbeta) per pattern as the library computes
    them: its bound with law errors (0, 0), (1, 0) and (0, 1).  Leaves the
    model's law errors at zero."""
    out = []
    for em, eb in ((0.0, 0.0), (1.0, 0.0), (0.0, 1.0)):
        model.set_law_error(em, eb)
        f, bound, _ = model.fap(td, b.off, b.f_min, b.df, b.Nf, p_obs, max_err=1e9, mc_realizations=0)
        out.append((f.cpu().numpy().astype(np.float64), bound.cpu().numpy().astype(np.float64) / Z99))
    model.set_law_error(0.0, 0.0)
    f, s0 = out[0]
    dm = np.sqrt(np.maximum(out[1][1] ** 2 - s0 ** 2, 0.0))
    db = np.sqrt(np.maximum(out[2][1] ** 2 - s0 ** 2, 0.0))
    return f, s0, dm, db


def calibrate(model, b: synth.Batch, R=10000, seed=30300, levels=CAL_LEVELS, exceed=0.005):
    """The law error lsp_fap_surrogate carries to each pattern's FAP, set by
    coverage on patterns kept out of training and validation: err_m is the
    smallest value for which at most a fraction `exceed` of the residuals
    |FAP_net - FAP_MC| (every pattern at every level) lie beyond the bound
      2.576 sqrt(spread^2 + (err_m dFAP/dm)^2 + FAP_MC (1 - FAP_MC) / R),
    the last term being the calibrating Monte Carlo's own variance (found by
    bisection; err_beta is left at 0).  The residuals have heavier tails than
    a normal law, so an RMS fit of err_m would cover too few of them.
    Returns (err_m, err_beta, n_residuals)."""
    torch = _torch()
    td = _device_t(b)
    Y = monte_carlo(b, R, seed)
    Ys, _ = torch.sort(Y, dim=1)
    res, s0s, dms, var = [], [], [], []
    for a in levels:
        k = max(0, int(math.ceil((1.0 - a) * R)) - 1)
        p_obs = Ys[:, k].contiguous()
        fap_mc = (Y >= p_obs[:, None]).double().mean(dim=1).cpu().numpy()
        f, s0, dm, _ = law_sensitivity(model, td, b, p_obs)
        res.append(np.abs(f - fap_mc)); s0s.append(s0); dms.append(dm); var.append(fap_mc * (1.0 - fap_mc) / R)
    r, s0, dm, v = (np.concatenate(x) for x in (res, s0s, dms, var))

    def outside(e):
        return float(np.mean(r > Z99 * np.sqrt(s0 ** 2 + (e * dm) ** 2 + v)))

    lo, hi = 0.0, 1.0
    while outside(hi) > exceed and hi < 64.0:
        hi *= 2.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if outside(mid) <= exceed:
            hi = mid
        else:
            lo = mid
    return float(hi), 0.0, int(r.size)


def validate(model, b: synth.Batch, R=10000, seed=20260, levels=FAP_LEVELS, max_err=0.005, R_fallback=10000,
             log=None):
    """Against a Monte Carlo of R realizations per pattern, at the MC quantiles
    of the given FAP levels: the network's error, the answers of
    lsp_fap_surrogate with its fallback (R_fallback draws, another key), the
    fallback rate, Eq. (3)'s error, and the time of both paths.

    Contract per answer: |FAP - FAP_MC| <= max_err + 4 sigma, sigma the
    standard deviation of the difference: the validating Monte Carlo's
    sqrt(a(1 - a)/R), and for an answer that fell back also its own
    sqrt(a(1 - a)/R_fallback).  Four sigma keeps the chance that a correct
    answer fails anywhere among 200 patterns x 4 levels near 5 %."""
    torch = _torch()
    td = _device_t(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Y = monte_carlo(b, R, seed)
    torch.cuda.synchronize()
    t_mc = time.perf_counter() - t0
    Ys, _ = torch.sort(Y, dim=1)
    res = {"patterns": b.n, "R": R, "R_fallback": R_fallback, "max_err": max_err, "mc_seconds": t_mc, "levels": {}}
    Nt = b.Nt
    for a in levels:
        k = max(0, int(math.ceil((1.0 - a) * R)) - 1)
        p_obs = Ys[:, k].contiguous()
        fap_mc = (Y >= p_obs[:, None]).float().mean(dim=1).cpu().numpy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fap_net, bound, _ = model.fap(td, b.off, b.f_min, b.df, b.Nf, p_obs, max_err=1e9, mc_realizations=0)
        torch.cuda.synchronize()
        t_net = time.perf_counter() - t0
        t0 = time.perf_counter()
        fap_full, _, used = model.fap(td, b.off, b.f_min, b.df, b.Nf, p_obs, max_err=max_err,
                                      mc_realizations=R_fallback, seed=seed + 1)
        torch.cuda.synchronize()
        t_full = time.perf_counter() - t0
        pn = p_obs.cpu().numpy()
        fap_eq3 = np.array([lsp_fap_analytic(float(pn[i]), int(Nt[i]), int(b.Nf[i])) for i in range(b.n)])
        net = np.abs(fap_net.cpu().numpy() - fap_mc)
        full = np.abs(fap_full.cpu().numpy() - fap_mc)
        eq3 = np.abs(fap_eq3 - fap_mc)
        fb = used.cpu().numpy().astype(bool)
        se = math.sqrt(a * (1 - a) / R)
        se_fb = math.sqrt(a * (1 - a) / R_fallback)
        allowed = max_err + 4.0 * np.where(fb, math.sqrt(se ** 2 + se_fb ** 2), se)
        kept = ~fb
        res["levels"][str(a)] = {
            "net_max_abs_err": float(net.max()), "net_mean_abs_err": float(net.mean()),
            "net_frac_within_max_err": float((net <= max_err).mean()),
            "bound_mean": float(bound.mean().item()),
            "fallback_rate": float(fb.mean()),
            "kept_max_abs_err": float(net[kept].max()) if kept.any() else None,
            "with_fallback_max_abs_err": float(full.max()), "with_fallback_mean_abs_err": float(full.mean()),
            "contract_violations": int((full > allowed).sum()),
            "eq3_max_abs_err": float(eq3.max()), "eq3_mean_abs_err": float(eq3.mean()),
            "mc_standard_error": se,
            "surrogate_seconds": t_net, "with_fallback_seconds": t_full,
            "speedup_vs_mc": t_mc / max(t_net, 1e-9), "speedup_with_fallback": t_mc / max(t_full, 1e-9),
        }
        if log:
            lv = res["levels"][str(a)]
            log(f"FAP {a}: net max {net.max():.4f} mean {net.mean():.5f}; fallback rate {lv['fallback_rate']:.2f}, "
                f"kept max {lv['kept_max_abs_err']}, with fallback max {full.max():.4f}, violations "
                f"{lv['contract_violations']}; Eq.3 max {eq3.max():.3f} mean {eq3.mean():.4f}; speed x"
                f"{lv['speedup_vs_mc']:.0f} (with fallback x{lv['speedup_with_fallback']:.1f})")
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-patterns", type=int, default=2000)
    ap.add_argument("--val-patterns", type=int, default=200)
    ap.add_argument("--R", type=int, default=500)
    ap.add_argument("--R-val", type=int, default=10000)
    ap.add_argument("--cal-patterns", type=int, default=200,
                    help="patterns (an independent draw) for the law errors; 0 = none")
    ap.add_argument("--members", type=int, default=4)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--nt-max", type=int, default=20000)
    ap.add_argument("--out", default="")
    ap.add_argument("--report", default="")
    args = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    torch = _torch()
    n_all = args.train_patterns + args.val_patterns
    pats = synth.c4_patterns(n_all, nt_range=(200, args.nt_max))
    tr = synth.subset(pats, np.arange(args.train_patterns))
    va = synth.subset(pats, np.arange(args.train_patterns, n_all))
    log(f"patterns: train {tr.n} ({tr.terms * args.R:.3g} MC terms), val {va.n} ({va.terms * args.R_val:.3g})")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = features(tr)
    Y = monte_carlo(tr, args.R, seed=1)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    log(f"training data in {t_data:.1f} s")
    t0 = time.perf_counter()
    model, hist = train(F, Y, members=args.members, steps=args.steps, batch=args.batch, lr=args.lr, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"trained in {t_train:.1f} s")
    cal_info = None
    if args.cal_patterns > 0:
        cal = synth.c4_patterns(args.cal_patterns, seed_sub=1, nt_range=(200, args.nt_max))
        t0 = time.perf_counter()
        err_m, err_b, n_res = calibrate(model, cal, R=args.R_val)
        model.set_law_error(err_m, err_b)
        cal_info = {"patterns": cal.n, "R": args.R_val, "levels": list(CAL_LEVELS), "residuals": n_res,
                    "err_m": err_m, "err_beta": err_b, "seconds": time.perf_counter() - t0}
        log(f"law errors: m {err_m:.4f}, beta {err_b:.4f} ({n_res} residuals)")
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        model.save(args.out)
    res = validate(model, va, R=args.R_val, log=log)
    res["law_error_calibration"] = cal_info
    res.update({"train_patterns": tr.n, "R_train": args.R, "data_seconds": t_data, "train_seconds": t_train,
                "members": args.members, "steps": args.steps, "early_stopping": hist})
    log(json.dumps(res))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(res, f, indent=1)
    model.close()


if __name__ == "__main__":
    main(sys.argv[1:])
