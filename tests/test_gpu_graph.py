"""GPU: graph replay of the iteration body gives the eager launches' bits, on
repeated replays with eager work and other buffers in between."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def amg():
    import paper_2511_21268_amd as m
    assert torch.cuda.is_available()
    m.lib()
    return m


@pytest.mark.parametrize("kw", [{}, {"krylov": 1, "vcycle_fp32": 1}, {"smoother": 1}])
def test_single_graph_equals_eager(oracle, amg, kw):
    print(f"case graph single {kw}", flush=True)
    from paper_2511_21268_amd.workloads import rhs_normal
    rp, ci, v, _ = oracle.poisson_kron(3, 3, 16)
    N = len(rp) - 1
    ctx = amg.Context(rp, ci, v, **kw)
    if kw.get("smoother"):
        for l in range(ctx.nlevels - 1):
            assert ctx.set_poly(l, [4.0, -6.0, 4.0, -1.0]) == 0
    ctx.set_graph(False)
    Fs = [torch.from_numpy(rhs_normal(N, s)).cuda() for s in range(3)]
    eager = [ctx.solve(F) for F in Fs]
    ctx.set_graph(True)
    for rep in range(3):
        for F, e in zip(Fs, eager):
            g = ctx.solve(F, u=torch.zeros_like(F))
            assert g["iters"] == e["iters"] and torch.equal(g["u"], e["u"])
            ctx.spmv(g["u"])                      # eager work between replays
    # a warm start through the graph path
    w = ctx.solve(Fs[0], u=eager[0]["u"].clone())
    assert w["iters"] == 0


def test_batched_graph_equals_eager(oracle, amg):
    print("case graph batched", flush=True)
    from paper_2511_21268_amd.workloads import rhs_block
    rp, ci, v, _ = oracle.poisson_kron(3, 3, 16)
    N = len(rp) - 1
    ctx = amg.Context(rp, ci, v, krylov=1, vcycle_fp32=1, nrhs=16)
    F = torch.from_numpy(rhs_block(N, range(16))).cuda()
    ctx.set_graph(False)
    e = ctx.solve_batched(F)
    ctx.set_graph(True)
    for rep in range(3):
        g = ctx.solve_batched(F)
        assert g["iters"] == e["iters"] and torch.equal(g["U"], e["U"])
        ctx.solve(F[:, 0].contiguous())          # single solve in between
