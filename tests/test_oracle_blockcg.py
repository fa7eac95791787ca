"""Oracle pins of the block flexible CG for several right-hand sides (the
O'Leary block variant of the batched solve): one column is FCG(1); finite
termination in ceil(n/s) block steps; every column's energy error is at most
that of its own preconditioned CG (the block Krylov space contains the
column's); a converged column leaves the block without changing the others;
every column reaches its tolerance."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle


def _csr(rp, ci, v):
    n = len(rp) - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n))


def _system(d=3, p=2, n=8):
    rp, ci, v, _ = oracle.poisson_kron(d, p, n)
    return rp, ci, v


def test_one_column_is_fcg():
    rp, ci, v = _system()
    h = oracle.Hierarchy(rp, ci, v, max_coarse=20)
    F = np.random.default_rng(0).standard_normal((h.n, 1))
    b = h.block_solve(F, tol=1e-10)
    f = h.solve(F[:, 0], tol=1e-10, flexible=True)
    assert b["rc"] == 0 and b["iters"][0] == f["iters"]
    assert np.linalg.norm(b["U"][:, 0] - f["u"]) <= 1e-11 * np.linalg.norm(f["u"])


def test_finite_termination():
    rp, ci, v = _system(2, 2, 8)            # n = 64
    h = oracle.Hierarchy(rp, ci, v, max_coarse=8)
    n, s = h.n, 8
    F = np.random.default_rng(1).standard_normal((n, s))
    b = h.block_solve(F, tol=1e-11, itmax=n)
    assert b["rc"] == 0 and b["iters"].max() <= n // s + 2
    K = _csr(rp, ci, v).toarray()
    X = np.linalg.solve(K, F)
    assert np.abs(b["U"] - X).max() <= 1e-8 * np.abs(X).max()


@pytest.mark.parametrize("k", [1, 2, 4])
def test_block_energy_not_worse_than_columns(k):
    rp, ci, v = _system()
    h = oracle.Hierarchy(rp, ci, v, max_coarse=20)
    K = _csr(rp, ci, v)
    F = np.random.default_rng(k).standard_normal((h.n, 4))
    X = np.column_stack([sp.linalg.spsolve(K.tocsc(), F[:, j]) for j in range(4)])
    b = h.block_solve(F, tol=0.0, itmax=k)
    for j in range(4):
        f = h.solve(F[:, j], tol=0.0, itmax=k, flexible=True)
        eb = X[:, j] - b["U"][:, j]
        ef = X[:, j] - f["u"]
        assert eb @ (K @ eb) <= (ef @ (K @ ef)) * (1 + 1e-9)
    # and strictly better in total after a few steps
    if k >= 2:
        tot_b = sum((X[:, j] - b["U"][:, j]) @ (K @ (X[:, j] - b["U"][:, j])) for j in range(4))
        tot_f = 0.0
        for j in range(4):
            e = X[:, j] - h.solve(F[:, j], tol=0.0, itmax=k, flexible=True)["u"]
            tot_f += e @ (K @ e)
        assert tot_b < tot_f


def test_converged_column_leaves_the_block():
    rp, ci, v = _system()
    h = oracle.Hierarchy(rp, ci, v, max_coarse=20)
    F = np.random.default_rng(5).standard_normal((h.n, 4))
    F0 = F.copy(); F0[:, 2] = 0.0
    a = h.block_solve(F0, tol=1e-9)
    b = h.block_solve(F[:, [0, 1, 3]], tol=1e-9)
    assert a["iters"][2] == 0 and not a["U"][:, 2].any()
    assert np.array_equal(a["U"][:, [0, 1, 3]], b["U"]) and np.array_equal(a["iters"][[0, 1, 3]], b["iters"])


def test_every_column_converges():
    rp, ci, v = _system(3, 3, 10)
    h = oracle.Hierarchy(rp, ci, v)
    K = _csr(rp, ci, v)
    F = np.random.default_rng(9).standard_normal((h.n, 16))
    F[:, 5] *= 1e-6                          # columns of very different scales
    b = h.block_solve(F, tol=1e-8)
    assert b["rc"] == 0
    for j in range(16):
        assert np.linalg.norm(F[:, j] - K @ b["U"][:, j]) <= 1.001e-8 * np.linalg.norm(F[:, j])
    single = max(h.solve(F[:, j], tol=1e-8, flexible=True)["iters"] for j in range(16))
    print(f"block FCG: max {b['iters'].max()} iterations, single FCG: max {single}")
    assert b["iters"].max() < single
