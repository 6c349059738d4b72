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
