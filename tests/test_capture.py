"""Single-curve calls captured into a HIP graph (torch.cuda.graph): every replay
equals the eager result, with eager work and synchronizations between
replays; an eager call that outgrows the stream's workspace after the capture
leaves the graph's buffer alive (it is retired, not freed); a capture that
would need a larger workspace fails with LSP_ERR_CAPTURE instead of
allocating."""
import numpy as np
import pytest

from paper_1007_1658_amd import synth
from util import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1007_1658_amd as lsp  # noqa: E402


@pytest.mark.parametrize("form", ["default", "recur"])
def test_single_curve_call_replays_from_a_hip_graph(form):
    print(f"capture form={form}", flush=True)
    c = synth.c0()
    t, x = to_dev(c)
    kw = {} if form == "default" else dict(trig="recur", m=8, waves=4)
    s = torch.cuda.Stream()
    ref = torch.empty(c.Nf, dtype=torch.float32, device="cuda")
    out = torch.empty_like(ref)
    with torch.cuda.stream(s):
        lsp.lsp_periodogram_ex(t, x, c.f_min, c.df, c.Nf, Pn=ref, **kw)   # workspace set up, uncaptured
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        lsp.lsp_periodogram_ex(t, x, c.f_min, c.df, c.Nf, Pn=out, **kw)
    torch.cuda.synchronize()

    big = synth.c1()
    tb, xb = to_dev(big)
    Pb = torch.empty(big.Nf, dtype=torch.float32, device="cuda")
    for r in range(4):
        out.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {r}"
        # eager work between replays: a plain call, then (once) one on the graph's
        # stream that outgrows its workspace
        lsp.lsp_periodogram_ex(t, x, c.f_min, c.df, c.Nf, Pn=ref.clone(), **kw)
        if r == 1:
            with torch.cuda.stream(s):
                lsp.lsp_periodogram_ex(tb, xb, big.f_min, big.df, big.Nf, Pn=Pb, **kw)
            s.synchronize()
        torch.cuda.synchronize()
    del g


def test_capture_that_would_grow_the_workspace_is_refused():
    c = synth.c0()
    t, x = to_dev(c)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        lsp.lsp_periodogram(t, x, c.f_min, c.df, c.Nf)
    s.synchronize()
    big = synth.c1()
    tb, xb = to_dev(big)
    Pb = torch.empty(big.Nf, dtype=torch.float32, device="cuda")
    g = torch.cuda.CUDAGraph()
    status = None
    try:
        with torch.cuda.graph(g, stream=s):
            try:
                lsp.lsp_periodogram(tb, xb, big.f_min, big.df, big.Nf, Pn=Pb)
            except lsp.LspError as e:
                status = e.status
    except RuntimeError:
        pass  # an empty capture may be reported by torch on exit
    torch.cuda.synchronize()
    assert status == lsp.LSP_ERR_CAPTURE
    # the stream still works uncaptured afterwards
    with torch.cuda.stream(s):
        lsp.lsp_periodogram(tb, xb, big.f_min, big.df, big.Nf, Pn=Pb)
    s.synchronize()
    assert np.isfinite(Pb.cpu().numpy()).all()


def _batched_on(stream, b, out):
    t = torch.from_numpy(b.t).cuda()
    x = torch.from_numpy(b.x).cuda()
    with torch.cuda.stream(stream):
        lsp.lsp_periodogram_batched(t, x, b.off, b.f_min, b.df, b.Nf, want_pn=True, stream=stream, out=out)
    return t, x


def _batch_out(b):
    n = b.n
    return {"pmax": torch.empty(n, dtype=torch.float32, device="cuda"),
            "kbest": torch.empty(n, dtype=torch.int64, device="cuda"),
            "fbest": torch.empty(n, dtype=torch.float64, device="cuda"),
            "Pn": torch.empty(int(b.Nf.sum()), dtype=torch.float32, device="cuda")}


@pytest.mark.parametrize("form", ["mfma", "recur"])
def test_batched_call_replays_after_other_shapes(form):
    """A batched call captured by the caller replays its own shape bit for bit
    after uncaptured calls on the same stream with another plan of the same
    workspace size (another grid) and with a larger plan: the captured plan
    tables are moved aside, never overwritten or freed."""
    print(f"batched capture form={form}", flush=True)
    lsp.lsp_set_batched_form(form)
    try:
        A = synth.c3(seed_sub=5, n_curves=24, nt_range=(200, 2000))
        B = synth.Batch(A.t, A.x, A.off, 1.1 * A.f_min, 1.1 * A.df, A.Nf.copy(), "B")  # same sizes, new grid
        C = synth.c3(seed_sub=6, n_curves=64, nt_range=(200, 4000))                     # larger
        s = torch.cuda.Stream()
        ref = _batch_out(A)
        tA, xA = _batched_on(s, A, ref)             # prepares the stream's workspace, uncaptured
        s.synchronize()
        cap = _batch_out(A)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            lsp.lsp_periodogram_batched(tA, xA, A.off, A.f_min, A.df, A.Nf, want_pn=True, stream=s, out=cap)
        torch.cuda.synchronize()
        others = []
        for r, other in enumerate((B, C, A, B)):
            for v in cap.values():
                v.fill_(-1)
            g.replay()
            torch.cuda.synchronize()
            for name in ("pmax", "kbest", "Pn"):
                assert torch.equal(cap[name], ref[name]), f"replay {r}: {name}"
            # an uncaptured call with another shape on the graph's stream, checked
            # against the same call on a stream of its own
            o, o2 = _batch_out(other), _batch_out(other)
            _batched_on(s, other, o)
            s2 = torch.cuda.Stream()
            _batched_on(s2, other, o2)
            torch.cuda.synchronize()
            assert torch.equal(o["Pn"], o2["Pn"]) and torch.equal(o["pmax"], o2["pmax"])
            others.append(o)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(cap["Pn"], ref["Pn"])
        del g
    finally:
        lsp.lsp_set_batched_form("mfma")


def test_monte_carlo_call_refuses_capture():
    b = synth.c3(seed_sub=7, n_curves=4, nt_range=(200, 400))
    t = torch.from_numpy(b.t).cuda()
    s = torch.cuda.Stream()
    out = torch.empty(4 * 3, dtype=torch.float32, device="cuda")
    g = torch.cuda.CUDAGraph()
    status = None
    try:
        with torch.cuda.graph(g, stream=s):
            try:
                lsp.lsp_mc_maxpower(t, b.off, b.f_min, b.df, b.Nf, 3, seed=1, out=out, stream=s)
            except lsp.LspError as e:
                status = e.status
    except RuntimeError:
        pass  # an empty capture may be reported by torch on exit
    torch.cuda.synchronize()
    assert status == lsp.LSP_ERR_CAPTURE
