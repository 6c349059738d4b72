"""The instruction-rate microbenchmarks run and give plausible rates on gfx950
(they back the roofline discussion; not a performance gate)."""
import math

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1007_1658_amd as lsp  # noqa: E402


def test_microbench_kinds_run():
    torch.empty(1, device="cuda")
    rates = {}
    for kind in range(9):
        ops, ms = lsp.lsp_microbench(kind, 2, 64)
        print(f"kind {kind}: {ops:.3e} ops/s in {ms:.3f} ms", flush=True)
        assert math.isfinite(ops) and ops > 0 and ms > 0
        rates[kind] = ops
    # the matrix pipe alone: between 40 % and 105 % of the 2.5 PFLOP/s dense FP16 peak
    assert 1.0e15 < rates[4] < 2.63e15
    # vector work after each MFMA cannot make the matrix pipe faster
    assert rates[7] <= rates[4] * 1.05
