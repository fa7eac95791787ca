"""GPU: block flexible CG over the 16-column batch (krylov = 2) against the
oracle's block FCG: the iterates after a fixed number of block steps (no
stopping decision involved), and full solves to 1e-8 (per-column iteration
counts within one of the oracle's, every true residual under the tolerance);
with the FP32 block V-cycle, fewer iterations than 16 independent FCG
recurrences."""
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


def _system(oracle, name):
    if name == "poisson p3 n10":
        rp, ci, v, _ = oracle.poisson_kron(3, 3, 10)
    else:
        rp, ci, v, _, _ = oracle.cube_system(3, 8)
    return rp, ci, v


def _rhs(n, s, seed):
    from paper_2511_21268_amd.workloads import rhs_block
    return rhs_block(n, range(seed, seed + s))


@pytest.mark.parametrize("name", ["poisson p3 n10", "cube p3 k8"])
@pytest.mark.parametrize("k", [1, 2, 3, 6])
def test_block_fixed_steps(oracle, amg, name, k):
    print(f"case {name} k={k}", flush=True)
    rp, ci, v = _system(oracle, name)
    h = oracle.Hierarchy(rp, ci, v)
    F = _rhs(h.n, 16, 3)
    ref = h.block_solve(F, tol=0.0, itmax=k)
    ctx = amg.Context(rp, ci, v, nrhs=16, krylov=2, itmax=k)
    Ft = torch.from_numpy(np.ascontiguousarray(F.T)).cuda().T
    out = ctx.solve_batched(Ft, tol=0.0, check=False)
    U = out["U"].cpu().numpy()
    err = np.linalg.norm(U - ref["U"]) / np.linalg.norm(ref["U"])
    assert err <= 1e-10, err
    assert list(out["iters"]) == [k] * 16


@pytest.mark.parametrize("name,s", [("poisson p3 n10", 16), ("cube p3 k8", 16), ("cube p3 k8", 5)])
def test_block_solve_parity(oracle, amg, name, s):
    print(f"case {name} s={s}", flush=True)
    rp, ci, v = _system(oracle, name)
    h = oracle.Hierarchy(rp, ci, v)
    F = _rhs(h.n, s, 7)
    ref = h.block_solve(F, tol=1e-8)
    ctx = amg.Context(rp, ci, v, nrhs=16, krylov=2)
    Ft = torch.from_numpy(np.ascontiguousarray(F.T)).cuda().T
    out = ctx.solve_batched(Ft, tol=1e-8)
    U = out["U"].cpu().numpy()
    it = np.array(out["iters"])
    print(f"  iterations gpu {list(it)} oracle {list(ref['iters'])}", flush=True)
    assert out["status"] == 0 and ref["rc"] == 0
    assert np.all(np.abs(it - ref["iters"]) <= 1) and abs(it.max() - ref["iters"].max()) <= 1
    import scipy.sparse as sp
    K = sp.csr_matrix((v, ci, rp), shape=(h.n, h.n))
    for j in range(s):
        assert np.linalg.norm(F[:, j] - K @ U[:, j]) <= 1.0001e-8 * np.linalg.norm(F[:, j])


def test_block_fp32_vcycle_fewer_iterations(amg):
    rp, ci, v, _ = amg.iga_poisson(3, 3, 32, want_F=False)
    F = _rhs(len(rp) - 1, 16, 0)
    Ft = torch.from_numpy(np.ascontiguousarray(F.T)).cuda().T
    blk = amg.Context(rp, ci, v, nrhs=16, krylov=2, vcycle_fp32=1).solve_batched(Ft, tol=1e-8)
    ind = amg.Context(rp, ci, v, nrhs=16, krylov=1, vcycle_fp32=1).solve_batched(Ft, tol=1e-8)
    print(f"  block max {max(blk['iters'])}, independent max {max(ind['iters'])}", flush=True)
    assert blk["status"] == 0 and max(blk["iters"]) < max(ind["iters"])


def test_block_edge_cases(oracle, amg):
    """A zero right-hand side column is done before the first step (zero
    solution, zero iterations) and does not change the other columns; a
    single column of block CG is FCG(1)."""
    rp, ci, v = _system(oracle, "poisson p3 n10")
    n = len(rp) - 1
    F = _rhs(n, 6, 11)
    F0 = F.copy(); F0[:, 3] = 0.0
    ctx = amg.Context(rp, ci, v, nrhs=16, krylov=2)
    out = ctx.solve_batched(torch.from_numpy(np.ascontiguousarray(F0.T)).cuda().T, tol=1e-8)
    U = out["U"].cpu().numpy()
    assert out["status"] == 0 and out["iters"][3] == 0 and not U[:, 3].any()
    h = oracle.Hierarchy(rp, ci, v)
    ref = h.block_solve(F0, tol=1e-8)
    assert all(abs(a - b) <= 1 for a, b in zip(out["iters"], ref["iters"]))
    one = ctx.solve_batched(torch.from_numpy(np.ascontiguousarray(F[:, :1].T)).cuda().T, tol=1e-8)
    single = amg.Context(rp, ci, v, krylov=1).solve(torch.from_numpy(F[:, 0].copy()).cuda(), tol=1e-8)
    assert abs(one["iters"][0] - single["iters"]) <= 1
    u1, us = one["U"][:, 0].cpu().numpy(), single["u"].cpu().numpy()
    assert np.linalg.norm(u1 - us) <= 1e-7 * np.linalg.norm(us)
