"""A whole factorisation captured in a HIP graph (torch.cuda.graph around
cqr_factor_ex with a caller workspace and info word) replays to the eager
result bit for bit. Every fill in the chain is a kernel, so the graph holds
no memset nodes. Replays are interleaved with eager work and checked one by
one."""
import numpy as np
import pytest

import matgen
from tests.util import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2405_04237_amd as cqr  # noqa: E402


@pytest.mark.parametrize("sched,m,n,b,kw", [
    ("mod", 4096, 64, 16, {}),
    ("orig", 4096, 64, 16, {}),
    ("scqr3", 5000, 100, 0, {}),
    ("mod", 8192, 96, 32, {"lookahead": True}),
    ("mod", 4096, 64, 16, {"adaptive": True}),
])
def test_graph_replays_match_eager(sched, m, n, b, kw):
    a = to_dev(matgen.test_matrix(m, n, 1e10 if sched != "orig" else 1e6, seed=71))
    ws = cqr.Workspace(m, n, b, sched, a.device)
    q = cqr.empty_colmajor(m, n, a.device, ld=a.stride(1))
    r = cqr.empty_colmajor(n, n, a.device)
    cqr.qr(a, b=b, schedule=sched, out=(q, r), workspace=ws, check=False, **kw)
    torch.cuda.synchronize()
    q0, r0 = q.clone(), r.clone()
    assert int(ws.info.item()) == 0
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            cqr.qr(a, b=b, schedule=sched, out=(q, r), workspace=ws, check=False, **kw)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        q.fill_(float("nan"))
        r.zero_()
        x = torch.randn(1000, 1000, dtype=torch.float64, device=a.device)
        (x @ x).sum().item()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(q, q0) and torch.equal(r, r0), rep
        assert int(ws.info.item()) == 0
