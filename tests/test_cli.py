"""lsp_run, a plain C program on the C ABI (no Python, no torch): its output
against the FP64 oracle on c0 (GPU), and its argument handling (CPU)."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1007_1658_amd import synth
from util import REL_TOL, peak_matches, rel_err

CLI = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1007_1658_amd", "cli",
                   "lsp_run")
needs_cli = pytest.mark.skipif(not os.path.exists(CLI), reason="lsp_run not built (run build())")


def _inputs(tmp_path, c):
    tp, xp = tmp_path / "t.bin", tmp_path / "x.bin"
    np.ascontiguousarray(c.t, dtype="<f8").tofile(tp)
    np.ascontiguousarray(c.x, dtype="<f4").tofile(xp)
    return str(tp), str(xp)


@needs_cli
def test_cli_rejects_bad_arguments_before_gpu_work(tmp_path):
    r = subprocess.run([CLI], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "usage" in r.stderr
    c = synth.c0()
    tp, xp = _inputs(tmp_path, c)
    r = subprocess.run([CLI, tp, xp, str(c.f_min), str(c.df), "0", str(tmp_path / "p.bin")],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "Nf" in r.stderr
    r = subprocess.run([CLI, tp, str(tmp_path / "missing.bin"), str(c.f_min), str(c.df), "10",
                        str(tmp_path / "p.bin")], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1


@needs_cli
@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["lsp", "gls"])
def test_cli_matches_oracle_on_c0(tmp_path, mode):
    c = synth.c0()
    tp, xp = _inputs(tmp_path, c)
    out = tmp_path / "p.bin"
    args = [CLI, tp, xp, repr(c.f_min), repr(c.df), str(c.Nf), str(out)] + (["gls"] if mode == "gls" else [])
    print("running", " ".join(args[1:]), flush=True)
    r = subprocess.run(args, capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0
    Pg = np.fromfile(out, dtype="<f4").astype(np.float64)
    assert Pg.size == c.Nf
    if mode == "gls":
        P = oracle.gls(c.t, c.x.astype(np.float64), c.f_min, c.df, Nf=c.Nf)
    else:
        P = oracle.periodogram(c.t, c.x, c.f_min, c.df, Nf=c.Nf)
    assert rel_err(Pg, P) <= REL_TOL
    assert peak_matches(Pg, P)
    assert f"peak k={int(np.argmax(Pg))}" in r.stdout
