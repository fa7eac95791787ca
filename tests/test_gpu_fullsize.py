"""GPU parity at the benchmark sizes.

3D p=3, n=64 (N = 274,625; 86.9M entries): the whole solve against the
oracle's, aggregates of every level bit for bit.
3D p=3, n=128 (N = 2,146,689; 707M entries, the benchmark workload, same
kernels, parameters and launch shapes as bench.py): the library's generator
gives the oracle's matrix bit for bit; the whole FP64 solve against the
oracle's -- every level's sizes, aggregates, coefficients and coarse matrices
bit for bit (host and device set-up), the iteration count exactly behind the
stop-margin check, and the solution within 1e-10; sampled SpMV rows; the 16-RHS
form with the autotuned block kernels, every column's FP64 true residual.
3D p=4, n=96 (640M entries): the FP32 V-cycle inside FP64 FCG against the
FP64 PCG on the same system.
3D p=5, n=64, variable kappa: sampled rows, plain and learned solves.
The cube of Sec. 5.1 at p=3, k=96 with the paper's default preconditioner:
the V-cycle (Cholesky coarse solve) is symmetric positive definite, and the
FCG solve reaches an FP64 true residual of 1e-8.
"""
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


@pytest.mark.timeout(600)
def test_c2_full_solve_parity(oracle, amg):
    print("case c2 full: 3D p=3 n=64 seed 0", flush=True)
    from paper_2511_21268_amd.workloads import rhs_normal
    rp, ci, v, _ = oracle.poisson_kron(3, 3, 64, want_F=False)
    F = rhs_normal(len(rp) - 1, 0)
    h = oracle.Hierarchy(rp, ci, v)
    ref = h.solve(F, tol=1e-8)
    print(f"  oracle: {h.nlevels} levels, {ref['iters']} iterations", flush=True)
    ctx = amg.Context(rp, ci, v)
    assert ctx.nlevels == h.nlevels
    for l in range(h.nlevels - 1):
        a, pc = ctx.aggregates(l)
        ao, pco, _, _ = h.level_agg(l)
        assert np.array_equal(a, ao) and np.array_equal(pc, pco), l
    out = ctx.solve(torch.from_numpy(F).cuda(), tol=1e-8)
    u = out["u"].cpu().numpy()
    err = np.linalg.norm(u - ref["u"]) / np.linalg.norm(ref["u"])
    # margin of the stopping test at the oracle's last two iterations
    margin = min(abs(ref["hist"][-1] / 1e-8 - 1), abs(ref["hist"][-2] / 1e-8 - 1))
    print(f"  gpu: {out['iters']} iterations, rel.err {err:.2e}, stop margin {margin:.2e}", flush=True)
    assert margin > 1e-6, "marginal stopping test: iteration parity not decidable"
    assert out["iters"] == ref["iters"]
    assert err <= 1e-10
    true = np.linalg.norm(F - oracle.spmv(rp, ci, v, u)) / np.linalg.norm(F)
    assert true <= 1e-8


def _sampled_rows(oracle, rp, ci, v, x, y, nsample=4000, seed=4):
    N = len(rp) - 1
    rows = np.unique(np.concatenate([np.arange(0, 200), np.arange(N - 200, N),
                                     np.random.default_rng(seed).integers(0, N, nsample)]))
    for i in rows:
        s, e = rp[i], rp[i + 1]
        ref = oracle.dot(v[s:e], x[ci[s:e]])
        scale = np.abs(v[s:e]) @ np.abs(x[ci[s:e]])
        assert abs(y[i] - ref) <= 8 * np.finfo(float).eps * scale, i


@pytest.fixture(scope="module")
def c4_system(oracle):
    rp, ci, v, _ = oracle.poisson_kron(3, 3, 128, want_F=False)
    return rp, ci, v


@pytest.fixture(scope="module")
def c4_oracle(oracle, c4_system):
    """The oracle's hierarchy of the 3D p=3 n=128 system (about a minute on the
    host), shared by the tests of this module."""
    import time
    rp, ci, v = c4_system
    t = time.time()
    h = oracle.Hierarchy(rp, ci, v)
    print(f"  oracle hierarchy: {[h.level_info(l) for l in range(h.nlevels)]} in {time.time() - t:.1f} s",
          flush=True)
    return h


def _same_as_oracle(ctx, h, first_matrix=1):
    assert ctx.nlevels == h.nlevels
    for l in range(h.nlevels):
        assert ctx.level_info(l) == h.level_info(l), l
    for l in range(h.nlevels - 1):
        a, pc = ctx.aggregates(l)
        ao, pco, _, _ = h.level_agg(l)
        assert np.array_equal(a, ao) and np.array_equal(pc, pco), l
        if l + 1 >= first_matrix:
            for x, y in zip(ctx.coarse_matrix(l + 1), h.level_matrix(l + 1)):
                assert np.array_equal(x, y), l + 1


@pytest.mark.timeout(900)
def test_c4_full_solve_parity(oracle, amg, c4_system, c4_oracle):
    """The benchmark run itself (FP64 PCG, default parameters, F ~ N(0,1) seed 0)
    against the oracle (Sec. 3.1 hierarchy, Sec. 4 Krylov call)."""
    import time
    print("case c4 full: 3D p=3 n=128 seed 0", flush=True)
    from paper_2511_21268_amd.workloads import rhs_normal
    rp, ci, v = c4_system
    N = len(rp) - 1
    # the benchmark generates its system with the library: the same bits
    rg, cg, vg, _ = amg.iga_poisson(3, 3, 128, want_F=False)
    assert np.array_equal(rg, rp) and np.array_equal(cg, ci) and np.array_equal(vg, v)
    del rg, cg, vg
    print("  library generator = oracle assembly", flush=True)
    h = c4_oracle
    F = rhs_normal(N, 0)
    oracle.set_threads(16)
    t = time.time()
    ref = h.solve(F, tol=1e-8)
    print(f"  oracle solve: {ref['iters']} iterations in {time.time() - t:.1f} s (16 threads)", flush=True)
    ctx = amg.Context(rp, ci, v)
    _same_as_oracle(ctx, h)
    print("  every level's aggregates, coefficients and coarse matrix = oracle's", flush=True)
    out = ctx.solve(torch.from_numpy(F).cuda(), tol=1e-8)
    u = out["u"].cpu().numpy()
    err = np.linalg.norm(u - ref["u"]) / np.linalg.norm(ref["u"])
    margin = min(abs(ref["hist"][-1] / 1e-8 - 1), abs(ref["hist"][-2] / 1e-8 - 1))
    print(f"  gpu: {out['iters']} iterations, rel.err {err:.2e}, stop margin {margin:.2e}", flush=True)
    assert margin > 1e-6, "marginal stopping test: iteration parity not decidable"
    assert out["status"] == 0 and ref["rc"] == 0
    assert out["iters"] == ref["iters"]
    assert err <= 1e-10
    true = np.linalg.norm(F - oracle.spmv(rp, ci, v, u)) / np.linalg.norm(F)
    assert true <= 1e-8


@pytest.mark.timeout(900)
def test_c4_device_setup_against_oracle(amg, c4_system, c4_oracle):
    """Device set-up (Sec. 3.1 on the GPU) of the 3D p=3 n=128 system: every
    level equals the oracle's hierarchy bit for bit; set-up time printed."""
    import time
    print("case c4 device set-up: 3D p=3 n=128", flush=True)
    rp, ci, v = c4_system
    t = time.time()
    dev = amg.Context(rp, ci, v, setup_device=1)
    td = time.time() - t
    sw, tot, mx = dev.setup_rounds()
    print(f"  device set-up (hierarchy + device images) {td:.1f} s, rounds {tot} over {sw} sweeps (max {mx})",
          flush=True)
    _same_as_oracle(dev, c4_oracle)


@pytest.mark.timeout(900)
def test_c4_properties(oracle, amg, c4_system):
    print("case c4: 3D p=3 n=128 seed 0", flush=True)
    from paper_2511_21268_amd.workloads import rhs_normal
    rp, ci, v = c4_system
    N = len(rp) - 1
    print(f"  oracle assembled N={N} nnz={len(v)}", flush=True)
    ctx = amg.Context(rp, ci, v)
    assert ctx.format(0)["index_bytes"] == 2
    # sampled SpMV rows of the level-0 kernel
    x = np.random.default_rng(3).standard_normal(N)
    y = ctx.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
    _sampled_rows(oracle, rp, ci, v, x, y)
    print("  sampled SpMV rows ok", flush=True)
    # the library's level-0 matching sweep is the greedy matching on every edge
    mate = amg.match(rp, ci, v)
    assert oracle.check_greedy(rp, ci, v, mate) == 0
    print("  level-0 matching is the greedy matching", flush=True)
    # the solve reaches the tolerance on the FP64 system (oracle SpMV)
    F = rhs_normal(N, 0)
    out = ctx.solve(torch.from_numpy(F).cuda(), tol=1e-8)
    u = out["u"].cpu().numpy()
    true = np.linalg.norm(F - oracle.spmv(rp, ci, v, u)) / np.linalg.norm(F)
    print(f"  solve: {out['iters']} iterations, true relres {true:.3e}", flush=True)
    assert out["status"] == 0 and true <= 1e-8


@pytest.mark.timeout(900)
@pytest.mark.parametrize("krylov", [1, 2])
def test_c4_batched_properties(oracle, amg, c4_system, krylov):
    """16 right-hand sides (seeds 0..15), FP32 block V-cycle in FP64 FCG with
    the autotuned block kernels, as bench.py --mode batched runs it
    (krylov = 2: block flexible CG, as --mode blockcg)."""
    print(f"case c4 x 16: 3D p=3 n=128 seeds 0..15 krylov {krylov}", flush=True)
    from paper_2511_21268_amd.workloads import rhs_block
    rp, ci, v = c4_system
    N = len(rp) - 1
    ctx = amg.Context(rp, ci, v, vcycle_fp32=1, krylov=krylov, nrhs=16)
    print(f"  autotuned block variant {ctx.batched_variant()}", flush=True)
    Fh = rhs_block(N, range(16))
    out = ctx.solve_batched(torch.from_numpy(Fh).cuda(), tol=1e-8)
    U = out["U"].cpu().numpy()
    assert out["status"] == 0
    for j in range(16):
        true = np.linalg.norm(Fh[:, j] - oracle.spmv(rp, ci, v, U[:, j])) / np.linalg.norm(Fh[:, j])
        assert true <= 1e-8 * 1.0001, (j, true)
    print(f"  iterations {out['iters']}", flush=True)


@pytest.mark.timeout(900)
def test_c3_fp32_vcycle_properties(oracle, amg):
    """3D p=4, n=96: FP32 V-cycle in FP64 FCG against FP64 PCG, both to 1e-8 on
    the FP64 system (oracle SpMV); the change in iterations and the solution
    difference are reported; both residuals at 1e-8 bound K (u32 - u64)."""
    print("case c3: 3D p=4 n=96 seed 0", flush=True)
    from paper_2511_21268_amd.workloads import rhs_normal
    rp, ci, v, _ = oracle.poisson_kron(3, 4, 96, want_F=False)
    N = len(rp) - 1
    F = rhs_normal(N, 0)
    Ft = torch.from_numpy(F).cuda()
    res, zs = {}, {}
    rvec = torch.from_numpy(np.random.default_rng(5).standard_normal(N)).cuda()
    for name, kw in (("fp64", {}), ("fp32", dict(vcycle_fp32=1, krylov=1))):
        ctx = amg.Context(rp, ci, v, **kw)
        zs[name] = ctx.vcycle(rvec).cpu().numpy()
        out = ctx.solve(Ft, tol=1e-8)
        u = out["u"].cpu().numpy()
        r = F - oracle.spmv(rp, ci, v, u)
        true = np.linalg.norm(r) / np.linalg.norm(F)
        print(f"  {name}: {out['iters']} iterations, true relres {true:.3e}", flush=True)
        assert out["status"] == 0 and true <= 1e-8 * 1.0001
        res[name] = (u, out["iters"], r)
        if name == "fp64":
            x = np.random.default_rng(3).standard_normal(N)
            _sampled_rows(oracle, rp, ci, v, x, ctx.spmv(torch.from_numpy(x).cuda()).cpu().numpy(), nsample=2000)
        del ctx
    # the FP32 V-cycle is the one in use: it differs from the FP64 V-cycle at FP32 level
    dz = np.linalg.norm(zs["fp32"] - zs["fp64"]) / np.linalg.norm(zs["fp64"])
    print(f"  V-cycle FP32 vs FP64: {dz:.2e}", flush=True)
    assert 1e-9 < dz < 1e-4
    u64, u32 = res["fp64"][0], res["fp32"][0]
    err = np.linalg.norm(u32 - u64) / np.linalg.norm(u64)
    print(f"  iterations fp32 - fp64: {res['fp32'][1] - res['fp64'][1]}, solution difference {err:.2e}", flush=True)
    assert np.linalg.norm(res["fp64"][2] - res["fp32"][2]) <= 2.0001e-8 * np.linalg.norm(F)


@pytest.mark.timeout(900)
def test_c5_plain_and_learned(oracle, amg):
    """3D p=5, n=64, variable kappa (seed 0), f = 1: sampled SpMV rows; the
    plain l1 form and the learned smoother both reach 1e-8 on the FP64 system,
    the learned one in fewer iterations."""
    print("case c5: 3D p=5 n=64 kappa seed 0", flush=True)
    from paper_2511_21268_amd import learned
    from paper_2511_21268_amd.workloads import kappa_params
    rp, ci, v, F = amg.iga_diffusion(5, 64, *kappa_params(0))
    N = len(rp) - 1
    Ft = torch.from_numpy(F).cuda()
    its = {}
    for name in ("l1", "learned"):
        ctx = amg.Context(rp, ci, v, smoother=1 if name == "learned" else 0, itmax=6000)
        if name == "learned":
            acc, _ = learned.apply_learned(ctx)
            print(f"  accepted levels {acc}", flush=True)
        else:
            x = np.random.default_rng(3).standard_normal(N)
            _sampled_rows(oracle, rp, ci, v, x, ctx.spmv(torch.from_numpy(x).cuda()).cpu().numpy(), nsample=1000)
        out = ctx.solve(Ft, tol=1e-8)
        u = out["u"].cpu().numpy()
        true = np.linalg.norm(F - oracle.spmv(rp, ci, v, u)) / np.linalg.norm(F)
        print(f"  {name}: {out['iters']} iterations, true relres {true:.3e}", flush=True)
        assert out["status"] == 0 and true <= 1e-8 * 1.0001
        its[name] = out["iters"]
        del ctx
    assert its["learned"] < its["l1"]


@pytest.mark.timeout(900)
def test_cube96_paper_preconditioner_properties(oracle, amg):
    print("case cube p=3 k=96, the paper's default preconditioner", flush=True)
    rp, ci, v, F = amg.iga_cube(3, 96)
    prm = amg.paper_default(3)
    # with the Cholesky coarse solve the V-cycle is a fixed SPD operator
    ctx = amg.Context(rp, ci, v, **dict(prm, coarse_solver=0))
    print(f"  levels {[ctx.level_info(l)[0] for l in range(ctx.nlevels)]}, opc {ctx.opc():.3f}, "
          f"coarse formats {[ctx.format(l)['slice'] for l in range(1, ctx.nlevels - 1)]}", flush=True)
    rng = np.random.default_rng(2)
    y = torch.from_numpy(rng.standard_normal(len(F))).cuda()
    z = torch.from_numpy(rng.standard_normal(len(F))).cuda()
    By, Bz = ctx.vcycle(y), ctx.vcycle(z)
    a, b = float(torch.dot(z, By)), float(torch.dot(y, Bz))
    assert abs(a - b) <= 1e-10 * (abs(a) + abs(b)), (a, b)
    assert float(torch.dot(y, By)) > 0 and float(torch.dot(z, Bz)) > 0
    del ctx
    ctx = amg.Context(rp, ci, v, **prm)
    out = ctx.solve(torch.from_numpy(F).cuda(), tol=1e-8)
    u = out["u"].cpu().numpy()
    true = np.linalg.norm(F - oracle.spmv(rp, ci, v, u)) / np.linalg.norm(F)
    print(f"  FCG: {out['iters']} iterations, true relres {true:.2e}", flush=True)
    assert out["status"] == 0 and true <= 1e-8 * 1.0001 and out["iters"] <= 30
