"""GPU: the V-cycle tail in one persistent workgroup (k_vtail, k_vtail_blk)
against the per-level kernels it replaces: V-cycle outputs and whole solves
bit for bit, single vector and 16 columns, FP64 and FP32 V-cycles, with and
without graph replay; configurations outside its scope fall back."""
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


CASES = [(2, 2, 32), (3, 3, 16), (3, 2, 14)]


@pytest.mark.parametrize("d,p,n", CASES)
@pytest.mark.parametrize("fp32", [0, 1])
def test_tail_equals_per_level_kernels(oracle, amg, d, p, n, fp32):
    print(f"case tail d={d} p={p} n={n} fp32={fp32}", flush=True)
    from paper_2511_21268_amd.amg import AMG_OPT_TAIL
    from paper_2511_21268_amd.workloads import rhs_block, rhs_normal
    rp, ci, v, _ = oracle.poisson_kron(d, p, n)
    N = len(rp) - 1
    kw = dict(vcycle_fp32=1, krylov=1) if fp32 else {}
    ctx = amg.Context(rp, ci, v, **kw)
    assert ctx.option(AMG_OPT_TAIL) == 0   # off by default
    ctx.set_tail(1)
    first = ctx.option(AMG_OPT_TAIL)
    print(f"  levels {[ctx.level_info(l)[0] for l in range(ctx.nlevels)]}, tail from level {first}", flush=True)
    assert first >= 1
    r = torch.from_numpy(np.random.default_rng(1).standard_normal(N)).cuda()
    F = torch.from_numpy(rhs_normal(N, 2)).cuda()
    FB = torch.from_numpy(rhs_block(N, range(16))).cuda()
    res = {}
    for on in (1, 0):
        ctx.set_tail(on)
        z = ctx.vcycle(r)
        out = ctx.solve(F, tol=1e-8)
        bout = ctx.solve_batched(FB, tol=1e-8)
        res[on] = (z, out, bout)
    assert ctx.option(AMG_OPT_TAIL) == 0
    assert torch.equal(res[1][0], res[0][0])
    assert res[1][1]["iters"] == res[0][1]["iters"] and torch.equal(res[1][1]["u"], res[0][1]["u"])
    assert res[1][2]["iters"] == res[0][2]["iters"] and torch.equal(res[1][2]["U"], res[0][2]["U"])
    assert res[1][1]["status"] == 0 and res[1][2]["status"] == 0
    # with graph replay of the iteration body
    ctx.set_tail(1)
    ctx.set_graph(True)
    out = ctx.solve(F, tol=1e-8)
    bout = ctx.solve_batched(FB, tol=1e-8)
    ctx.set_graph(False)
    assert out["iters"] == res[0][1]["iters"] and torch.equal(out["u"], res[0][1]["u"])
    assert bout["iters"] == res[0][2]["iters"] and torch.equal(bout["U"], res[0][2]["U"])


def test_tail_scope_fallback(oracle, amg):
    """Two post-smoothing sweeps and the polynomial smoother are outside the
    tail's scope: the per-level kernels run, and the results are unchanged by
    the option."""
    print("case tail fallback", flush=True)
    from paper_2511_21268_amd.workloads import rhs_normal
    rp, ci, v, _ = oracle.poisson_kron(2, 2, 32)
    F = torch.from_numpy(rhs_normal(len(rp) - 1, 3)).cuda()
    for kw in (dict(nu_post=2), dict(smoother=1)):
        ctx = amg.Context(rp, ci, v, **kw)
        if "smoother" in kw:
            ctx.set_poly(1, [1.2, -0.3, 0.05, 0.0])
        outs = []
        for on in (1, 0):
            ctx.set_tail(on)
            outs.append(ctx.solve(F, tol=1e-8))
        assert outs[0]["iters"] == outs[1]["iters"] and torch.equal(outs[0]["u"], outs[1]["u"])
