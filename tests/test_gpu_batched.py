"""GPU: the batched solve (up to 16 right-hand sides sharing every block
SpMV and block V-cycle, each column with its own CG / FCG(1) scalars) against
the single-vector solve and the oracle."""
import numpy as np
import pytest
import scipy.sparse as sp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def amg():
    import paper_2511_21268_amd as m
    assert torch.cuda.is_available()
    m.lib()
    return m


def _csr(rp, ci, v):
    return sp.csr_matrix((v, ci, rp), shape=(len(rp) - 1, len(rp) - 1))


@pytest.mark.parametrize("d,p,n,k", [(2, 2, 32, 16), (3, 3, 16, 16), (3, 2, 14, 5)])
def test_batched_fp64_equals_single_and_oracle(oracle, amg, iters_match, oracle_iterate, d, p, n, k):
    print(f"case batched fp64 d={d} p={p} n={n} k={k}", flush=True)
    from paper_2511_21268_amd.workloads import rhs_block
    rp, ci, v, _ = oracle.poisson_kron(d, p, n)
    N = len(rp) - 1
    Fh = rhs_block(N, range(k))
    Fh[:, 1] = 0.0                                   # a zero column: u = 0 after 0 iterations
    ctx = amg.Context(rp, ci, v)
    Ft = torch.from_numpy(Fh).cuda()
    out = ctx.solve_batched(Ft, tol=1e-8)
    U = out["U"].cpu().numpy()
    h = oracle.Hierarchy(rp, ci, v)
    assert out["status"] == 0
    for j in range(k):
        single = ctx.solve(Ft[:, j].contiguous(), tol=1e-8)
        us = single["u"].cpu().numpy()
        assert out["iters"][j] == single["iters"], j
        assert np.array_equal(U[:, j], us), j       # same bits as the single-vector solve
        if j == 1:
            assert out["iters"][j] == 0 and not U[:, j].any()
            continue
        ref = h.solve(Fh[:, j], tol=1e-8)
        assert iters_match(out["iters"][j], ref, 1e-8), j
        uo = oracle_iterate(h, Fh[:, j], ref, out["iters"][j])
        assert np.linalg.norm(U[:, j] - uo) <= 1e-10 * np.linalg.norm(uo)


@pytest.mark.parametrize("d,p,n", [(3, 3, 16), (3, 4, 14)])
def test_batched_fp32_vcycle_fcg(oracle, amg, d, p, n):
    """16 columns, FP32 block V-cycle inside FP64 FCG: every column reaches the
    FP64 true residual 1e-8 and matches the single-vector FP32 solve."""
    print(f"case batched fp32 d={d} p={p} n={n}", flush=True)
    from paper_2511_21268_amd.workloads import rhs_block
    rp, ci, v, _ = oracle.poisson_kron(d, p, n)
    N = len(rp) - 1
    Fh = rhs_block(N, range(16))
    ctx = amg.Context(rp, ci, v, vcycle_fp32=1, krylov=1)
    Ft = torch.from_numpy(Fh).cuda()
    out = ctx.solve_batched(Ft, tol=1e-8)
    U = out["U"].cpu().numpy()
    assert out["status"] == 0
    K = _csr(rp, ci, v)
    h = oracle.Hierarchy(rp, ci, v)
    for j in range(16):
        true = np.linalg.norm(Fh[:, j] - K @ U[:, j]) / np.linalg.norm(Fh[:, j])
        assert true <= 1e-8, (j, true)
        single = ctx.solve(Ft[:, j].contiguous(), tol=1e-8)
        assert abs(out["iters"][j] - single["iters"]) <= 1
        ref = h.solve(Fh[:, j], tol=1e-8)
        err = np.linalg.norm(U[:, j] - ref["u"]) / np.linalg.norm(ref["u"])
        assert err <= 1e-6, (j, err)


def test_batched_itmax_and_args(oracle, amg):
    print("case batched edge", flush=True)
    from paper_2511_21268_amd.workloads import rhs_block
    rp, ci, v, _ = oracle.poisson_kron(2, 2, 32)
    N = len(rp) - 1
    ctx = amg.Context(rp, ci, v, itmax=2)
    out = ctx.solve_batched(torch.from_numpy(rhs_block(N, range(3))).cuda())
    assert out["status"] == 1 and out["iters"] == [2, 2, 2]
    with pytest.raises(amg.AmgError):
        ctx.solve_batched(torch.zeros(N, 17, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("fp32", [0, 1])
def test_autotuned_block_kernels(oracle, amg, fp32):
    """Context built for batched solves (nrhs = 16): the autotuner picks the
    lanes-per-row variant; every variant gives the same iterations as the
    single-vector solves and solutions equal to rounding."""
    print(f"case autotune fp32={fp32}", flush=True)
    from paper_2511_21268_amd.workloads import rhs_block
    rp, ci, v, _ = oracle.poisson_kron(3, 3, 18)
    N = len(rp) - 1
    Fh = rhs_block(N, range(16))
    kw = dict(vcycle_fp32=1, krylov=1) if fp32 else {}
    ctx = amg.Context(rp, ci, v, nrhs=16, **kw)
    lpr, thr = ctx.batched_variant()
    print(f"  autotuned: lpr={lpr} threads={thr}", flush=True)
    assert lpr in (1, 4, 8, 16) and thr in (256, 512)
    Ft = torch.from_numpy(Fh).cuda()
    singles = [ctx.solve(Ft[:, j].contiguous(), tol=1e-8) for j in range(16)]
    variants = [(1, 256)] + ([(lpr, 256), (lpr, 512)] if lpr > 1 else [])
    for (lp, th) in variants:
        ctx.set_batched_variant(lp, th)
        out = ctx.solve_batched(Ft, tol=1e-8)
        U = out["U"].cpu().numpy()
        assert out["status"] == 0
        for j in range(16):
            us = singles[j]["u"].cpu().numpy()
            assert abs(out["iters"][j] - singles[j]["iters"]) <= (0 if not fp32 else 1), (lp, th, j)
            tol = 1e-12 if not fp32 else 1e-6
            assert np.linalg.norm(U[:, j] - us) <= tol * np.linalg.norm(us), (lp, th, j)
    ctx.set_batched_variant(lpr, thr)


@pytest.mark.parametrize("kw", [{}, dict(vcycle_fp32=1, krylov=1)])
def test_batched_fused_post_equals_unfused(oracle, amg, kw):
    """Block prolongation fused into the first post-smoothing sweep through K P
    gives the unfused block V-cycle up to rounding, and the same iterations."""
    print(f"case batched fused post {kw}", flush=True)
    from paper_2511_21268_amd.workloads import rhs_block
    rp, ci, v, _ = oracle.poisson_kron(3, 3, 18)
    N = len(rp) - 1
    Ft = torch.from_numpy(rhs_block(N, range(16))).cuda()
    ctx = amg.Context(rp, ci, v, **kw)
    ctx.set_fused_post(True)
    of = ctx.solve_batched(Ft, tol=1e-8)
    ctx.set_fused_post(False)
    ou = ctx.solve_batched(Ft, tol=1e-8)
    assert of["status"] == 0 and ou["status"] == 0
    tol = 1e-12 if not kw else 1e-6
    for j in range(16):
        assert abs(of["iters"][j] - ou["iters"][j]) <= (0 if not kw else 1), j
        a, b = of["U"][:, j], ou["U"][:, j]
        assert torch.linalg.norm(a - b) <= tol * torch.linalg.norm(b), j


def test_batched_learned_polynomial_smoother(oracle, amg):
    """The batched solve with the learned degree-4 polynomial smoothers: with
    the FP64 V-cycle (one lane per row) every column matches its single-vector
    learned solve; with the autotuned FP32 block V-cycle every column reaches
    an FP64 true residual of 1e-8."""
    import os
    from paper_2511_21268_amd import learned
    from paper_2511_21268_amd.workloads import rhs_block
    if not os.path.exists(learned.WEIGHTS):
        pytest.skip("trained weights not present")
    rp, ci, v, _ = oracle.poisson_kron(3, 3, 20)
    N = len(rp) - 1
    Fh = rhs_block(N, range(6))
    Ft = torch.from_numpy(Fh).cuda()
    ctx = amg.Context(rp, ci, v, smoother=1)
    acc, _ = learned.apply_learned(ctx)
    print(f"case batched learned: accepted {acc}", flush=True)
    out = ctx.solve_batched(Ft, tol=1e-8)
    assert out["status"] == 0
    U = out["U"].cpu().numpy()
    for j in range(6):
        single = ctx.solve(Ft[:, j].contiguous(), tol=1e-8)
        us = single["u"].cpu().numpy()
        assert out["iters"][j] == single["iters"]
        assert np.linalg.norm(U[:, j] - us) <= 1e-12 * np.linalg.norm(us)
    ctx32 = amg.Context(rp, ci, v, smoother=1, vcycle_fp32=1, krylov=1, nrhs=16)
    learned.apply_learned(ctx32)
    out32 = ctx32.solve_batched(Ft, tol=1e-8)
    U32 = out32["U"].cpu().numpy()
    assert out32["status"] == 0
    for j in range(6):
        true = np.linalg.norm(Fh[:, j] - oracle.spmv(rp, ci, v, U32[:, j])) / np.linalg.norm(Fh[:, j])
        assert true <= 1e-8 * 1.0001, (j, true)
    print(f"  iterations fp64 {out['iters']} fp32 {out32['iters']}", flush=True)


@pytest.mark.parametrize("case", ["3d-p3-n16", "2d-p5-n40", "2d-p2-n61", "kappa-p4-n8"])
@pytest.mark.parametrize("fp32", [0, 1])
def test_block_window_equals_gather(oracle, amg, case, fp32):
    """The block passes with staged x windows (2 or 4 rows per lane; per
    wave, and shared by the four slices of a block) against the gather kernel
    they replace: every column bit for bit, FP64 and FP32 V-cycles;
    x-runs longer than one window (p = 5), slices straddling x-lines, a
    partly filled last slice, variable coefficients."""
    print(f"case block window {case} fp32={fp32}", flush=True)
    from paper_2511_21268_amd.workloads import kappa_params, rhs_block
    if case == "kappa-p4-n8":
        a, mk = kappa_params(3)
        rp, ci, v, _ = oracle.diffusion_quad3d(4, 8, a, mk, factorized=True)
    else:
        d, p, n = (int(t[1:]) if t[0] in "pn" else int(t[0]) for t in case.split("-"))
        rp, ci, v, _ = oracle.poisson_kron(d, p, n)
    N = len(rp) - 1
    Ft = torch.from_numpy(rhs_block(N, range(16))).cuda()
    kw = dict(vcycle_fp32=1, krylov=1) if fp32 else {}
    ctx = amg.Context(rp, ci, v, **kw)
    assert ctx.format(0)["shared_slices"] > 0
    assert ctx.option(amg.amg.AMG_OPT_BLOCK_WINDOW) == 4       # the default without autotuning
    assert ctx.option(amg.amg.AMG_OPT_WINDOW_SHARE) == 3   # shared windows in every pass, the default
    outs = {}
    for share in (0, 3):
        ctx.set_window_share(share)
        for rows in (0, 2, 4):
            ctx.set_block_window(rows)
            outs[share, rows] = ctx.solve_batched(Ft, tol=1e-8)
    ref = outs[0, 0]
    assert ref["status"] == 0
    for key, out in outs.items():
        assert out["iters"] == ref["iters"], key
        assert torch.equal(out["U"], ref["U"]), key
    print(f"  iterations {ref['iters']}", flush=True)
    for bad in (-1, 4):
        with pytest.raises(amg.AmgError):
            ctx.set_window_share(bad)
    for bad in (1, 3):
        with pytest.raises(amg.AmgError):
            ctx.set_block_window(bad)
