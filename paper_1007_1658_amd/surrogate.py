"""Training and validation of the false-alarm surrogate.

Every numerical step runs in the library: Monte-Carlo maxima
(lsp_mc_maxpower), window features (lsp_window_features), the network's
forward, loss, backward and Adam (lsp_mlp_grad, lsp_mlp_adam_step) and the
FAP with its Monte-Carlo fallback (lsp_fap_surrogate).  This module only
chooses minibatches, learning rates and chunk sizes, and summarizes results.

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


CAL_LEVELS = (0.001, 0.003, 0.01, 0.03, 0.1, 0.3, 0.6)   # one or more per bin of the error table


def calibrate(model, b: synth.Batch, R=10000, seed=30300, levels=CAL_LEVELS):
    """The error table lsp_fap_surrogate adds to the members' spread: per bin of
    the predicted FAP (edges Model.ERR_EDGES), the RMS of (FAP_net - FAP_MC) on
    patterns kept out of training and validation, with the Monte Carlo's own
    variance FAP (1 - FAP) / R removed.  Returns (rms[7], counts[7])."""
    torch = _torch()
    td = _device_t(b)
    Y = monte_carlo(b, R, seed)
    Ys, _ = torch.sort(Y, dim=1)
    edges32 = np.array(Model.ERR_EDGES, dtype=np.float32)   # binned in float32, as the library does
    nb = len(edges32) + 1
    sq, noise, cnt = np.zeros(nb), np.zeros(nb), np.zeros(nb)
    for a in levels:
        k = max(0, int(math.ceil((1.0 - a) * R)) - 1)
        p_obs = Ys[:, k].contiguous()
        fap_mc = (Y >= p_obs[:, None]).double().mean(dim=1).cpu().numpy()
        f, _, _ = model.fap(td, b.off, b.f_min, b.df, b.Nf, p_obs, max_sigma=1e9, mc_realizations=0)
        f32 = f.cpu().numpy()
        bins = np.searchsorted(edges32, f32, side="right")
        f = f32.astype(np.float64)
        np.add.at(sq, bins, (f - fap_mc) ** 2)
        np.add.at(noise, bins, fap_mc * (1.0 - fap_mc) / R)
        np.add.at(cnt, bins, 1.0)
    rms = np.sqrt(np.maximum(0.0, (sq - noise) / np.maximum(cnt, 1.0)))
    if (cnt > 0).any():
        rms[cnt == 0] = rms[cnt > 0].max()   # unseen bins: the largest measured error
    return rms.astype(np.float32), cnt.astype(np.int64)


def validate(model, b: synth.Batch, R=10000, seed=20260, levels=FAP_LEVELS, max_sigma=0.005, log=None):
    """|FAP_surrogate - FAP_MC| at the MC quantiles for the given FAP levels, the
    same for Eq. (3), the fallback rate and the speed against Monte Carlo."""
    torch = _torch()
    td = _device_t(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Y = monte_carlo(b, R, seed)
    torch.cuda.synchronize()
    t_mc = time.perf_counter() - t0
    Ys, _ = torch.sort(Y, dim=1)
    res = {"patterns": b.n, "R": R, "mc_seconds": t_mc, "levels": {}}
    Nt = b.Nt
    t_sur = 0.0
    for a in levels:
        k = max(0, int(math.ceil((1.0 - a) * R)) - 1)
        p_obs = Ys[:, k].contiguous()
        fap_mc = (Y >= p_obs[:, None]).float().mean(dim=1).cpu().numpy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fap_net, sig, _ = model.fap(td, b.off, b.f_min, b.df, b.Nf, p_obs, max_sigma=1e9, mc_realizations=0)
        torch.cuda.synchronize()
        t_sur += time.perf_counter() - t0
        fap_full, _, used = model.fap(td, b.off, b.f_min, b.df, b.Nf, p_obs, max_sigma=max_sigma,
                                      mc_realizations=R, seed=seed + 1)
        pn = p_obs.cpu().numpy()
        fap_eq3 = np.array([lsp_fap_analytic(float(pn[i]), int(Nt[i]), int(b.Nf[i])) for i in range(b.n)])
        net = np.abs(fap_net.cpu().numpy() - fap_mc)
        full = np.abs(fap_full.cpu().numpy() - fap_mc)
        eq3 = np.abs(fap_eq3 - fap_mc)
        res["levels"][str(a)] = {
            "net_max_abs_err": float(net.max()), "net_mean_abs_err": float(net.mean()),
            "net_frac_within_0.005": float((net <= 0.005).mean()),
            "with_fallback_max_abs_err": float(full.max()), "with_fallback_mean_abs_err": float(full.mean()),
            "fallback_rate": float(used.float().mean().item()),
            "eq3_max_abs_err": float(eq3.max()), "eq3_mean_abs_err": float(eq3.mean()),
            "mc_standard_error": float(math.sqrt(a * (1 - a) / R)),
        }
        if log:
            log(f"FAP {a}: net max {net.max():.4f} mean {net.mean():.5f}; with fallback max {full.max():.4f} "
                f"(rate {res['levels'][str(a)]['fallback_rate']:.2f}); Eq.3 max {eq3.max():.3f} mean {eq3.mean():.4f}")
    res["surrogate_seconds_per_level"] = t_sur / len(levels)
    res["speedup_vs_mc"] = t_mc / max(res["surrogate_seconds_per_level"], 1e-9)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-patterns", type=int, default=2000)
    ap.add_argument("--val-patterns", type=int, default=200)
    ap.add_argument("--R", type=int, default=500)
    ap.add_argument("--R-val", type=int, default=10000)
    ap.add_argument("--cal-patterns", type=int, default=200,
                    help="patterns (an independent draw) for the error table; 0 = no table")
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
        rms, cnt = calibrate(model, cal, R=args.R_val)
        model.set_error_table(rms)
        cal_info = {"patterns": cal.n, "R": args.R_val, "edges": list(Model.ERR_EDGES),
                    "rms": [float(v) for v in rms], "counts": [int(v) for v in cnt],
                    "seconds": time.perf_counter() - t0}
        log(f"error table {np.round(rms, 4).tolist()} (counts {cnt.tolist()})")
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        model.save(args.out)
    res = validate(model, va, R=args.R_val, log=log)
    res["error_table"] = cal_info
    res.update({"train_patterns": tr.n, "R_train": args.R, "data_seconds": t_data, "train_seconds": t_train,
                "members": args.members, "steps": args.steps, "early_stopping": hist})
    log(json.dumps(res))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(res, f, indent=1)
    model.close()


if __name__ == "__main__":
    main(sys.argv[1:])
