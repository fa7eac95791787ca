"""GPU: the paper's cube benchmark (Sec. 5.1) at the sizes of Table 1(b).

The library solves the oracle's system; against the oracle's PCG: aggregates,
iterations (the rule of the other FP64 parity tests), iterates to 1% of the
algebraic error the 1e-8 solve leaves, and the
discretization error of the GPU solution against the exact u = exp(x+z) sin y.
The iteration counts are printed beside Table 1(a)'s, which belong to the
paper's own preconditioner (smoothed aggregates of 8, Chebyshev smoothers): the
comparison is context, not a pin.  The library's own generator then solves the
full table, including k = 96."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TABLE_1A = {12: {3: 10, 4: 22, 5: 27, 6: 25}, 24: {3: 11, 4: 23, 5: 29, 6: 32}, 48: {3: 11, 4: 22, 5: 27, 6: 34},
            96: {3: 11, 4: 21}}


@pytest.fixture(scope="module")
def amg():
    import paper_2511_21268_amd as m
    assert torch.cuda.is_available()
    m.lib()
    return m


@pytest.mark.timeout(900)
@pytest.mark.parametrize("k,p", [(12, 3), (12, 4), (12, 5), (12, 6), (24, 3), (24, 4), (24, 5)])
def test_cube_parity(oracle, amg, iters_match, oracle_iterate, fixed_count_parity, k, p):
    """Runs of LONG_RUN iterations or more (k = 12, p = 5 and 6: ~955 and
    ~2460) are compared at fixed counts (no stopping decision) instead of
    through their stop.  Iterates: 1e-10, or within the oracle's own
    rounding-order spread at the same count (within_rounding): these mixed
    Dirichlet/Neumann systems amplify rounding far more than the all-Dirichlet
    ones (1e-6 between the oracle's two dot orders after 300 iterations)."""
    from conftest import LONG_RUN, order_spread, within_rounding
    print(f"case cube k={k} p={p}", flush=True)
    rp, ci, v, F, lift = oracle.cube_system(p, k)
    h = oracle.Hierarchy(rp, ci, v)
    ref = h.solve(F, tol=1e-8, itmax=6000)
    ctx = amg.Context(rp, ci, v, itmax=6000)
    for l in range(h.nlevels - 1):
        a, pc = ctx.aggregates(l)
        ao, pco, _, _ = h.level_agg(l)
        assert np.array_equal(a, ao) and np.array_equal(pc, pco), l
    out = ctx.solve(torch.from_numpy(F).cuda(), tol=1e-8)
    u = out["u"].cpu().numpy()
    assert out["status"] == 0 and out["relres_true"] <= 1e-8 * 1.0001
    e, nr = oracle.cube_error(p, k, u, lift)
    print(f"  N={len(F)}: {out['iters']} iterations (oracle {ref['iters']}; Table 1(a), paper's preconditioner: "
          f"{TABLE_1A[k][p]}), L2 error {e / nr:.2e}", flush=True)
    assert e / nr < 1e-4
    if ref["iters"] >= LONG_RUN:
        for kk, err, spread in fixed_count_parity(h, lambda kk: amg.Context(rp, ci, v, itmax=kk), F, (100, 300)):
            assert within_rounding(err, spread), (kk, err, spread)
        return
    assert iters_match(out["iters"], ref, 1e-8)
    uo = oracle_iterate(h, F, ref, out["iters"])
    # the iterate difference beside the algebraic error the solve leaves and
    # the oracle's own rounding-order spread at the same count
    ex = h.solve(F, tol=1e-13, itmax=20000)["u"]
    alg = np.linalg.norm(uo - ex) / np.linalg.norm(ex)
    err = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    spread = order_spread(h, F, out["iters"], u_asc=uo)
    eo, _ = oracle.cube_error(p, k, uo, lift)
    print(f"  iterate difference {err:.2e} (oracle order spread {spread:.2e}, algebraic error {alg:.2e}), "
          f"oracle L2 error {eo / nr:.2e}", flush=True)
    assert within_rounding(err, spread), (err, spread)


@pytest.mark.timeout(900)
def test_cube_table_library_generator(amg):
    """Every Table 1(b) case with the library's generator: sizes, convergence
    to 1e-8 (FP64 true residual)."""
    golden = os.path.join(os.path.dirname(__file__), "golden", "table1b_cube_sizes.json")
    with open(golden) as f:
        sizes = json.load(f)["sizes"]
    for k, row in sizes.items():
        for p, N in row.items():
            k_, p_ = int(k), int(p)
            rp, ci, v, F = amg.iga_cube(p_, k_)
            assert len(F) == N
            ctx = amg.Context(rp, ci, v, itmax=20000)
            Ft = torch.from_numpy(F).cuda()
            out = ctx.solve(Ft, tol=1e-8)
            print(f"  k={k_} p={p_} N={N}: {out['iters']} iterations (Table 1(a): {TABLE_1A[k_].get(p_)}), "
                  f"true relres {out['relres_true']:.2e}", flush=True)
            assert out["status"] == 0 and out["relres_true"] <= 1e-8 * 1.0001
            del ctx
