"""Pins of the oracle's solve phase (paper Sec. 3: smoother eq. (smoother), the
five steps of the two-level correction, the V-cycle's symmetry; Sec. 3.2
l1-Jacobi; Sec. 4 CG / flexible CG)."""
import numpy as np
import pytest
import scipy.sparse as sp


def _csr(rp, ci, v):
    return sp.csr_matrix((v, ci, rp), shape=(len(rp) - 1, len(rp) - 1))


@pytest.fixture(scope="module")
def c1(oracle):
    rp, ci, v, F = oracle.poisson_kron(2, 2, 32)
    return rp, ci, v, F, oracle.Hierarchy(rp, ci, v)


def test_spmv_and_dot_against_scipy(oracle, c1):
    rp, ci, v, F, _ = c1
    x = np.random.default_rng(0).standard_normal(len(rp) - 1)
    y = oracle.spmv(rp, ci, v, x)
    assert np.allclose(y, _csr(rp, ci, v) @ x, rtol=1e-14, atol=1e-15)
    assert abs(oracle.dot(x, y) - np.dot(x, y)) < 1e-12 * abs(np.dot(x, y))


def _dense_level(h, l):
    K = _csr(*h.level_matrix(l)).toarray()
    agg, pc, invd, _ = h.level_agg(l)
    return K, agg, pc, invd


def _dense_vcycle(h, l, f, poly=None):
    """The five steps of the two-level correction, recursively, written with
    dense matrices: smoother M = p(D^{-1}K) D^{-1}, R = P^T."""
    K, agg, pc, invd = _dense_level(h, l)
    if l == h.nlevels - 1:
        return np.linalg.solve(np.tril(K) + np.tril(K, -1).T, f)
    n = len(f)
    D = np.diag(invd)
    a = poly[l] if poly is not None else [1.0, 0, 0, 0]
    A = D @ K
    Mop = sum(a[k] * np.linalg.matrix_power(A, k) for k in range(4)) @ D
    nc = h.level_info(l + 1)[0]
    P = np.zeros((n, nc)); P[np.arange(n), agg] = pc
    u = Mop @ f                               # 1. pre-smoothing from zero
    rc = P.T @ (f - K @ u)                    # 2. restrict residual
    ec = _dense_vcycle(h, l + 1, rc, poly)    # 3. coarse solve
    u = u + P @ ec                            # 4. prolongate and correct
    u = u + Mop @ (f - K @ u)                 # 5. post-smoothing
    return u


def test_vcycle_equals_dense_two_level_recursion(oracle, c1):
    rp, ci, v, F, h = c1
    f = np.random.default_rng(1).standard_normal(len(F))
    z = h.vcycle(f)
    ref = _dense_vcycle(h, 0, f)
    assert np.abs(z - ref).max() <= 1e-11 * np.abs(ref).max()


def test_vcycle_is_symmetric_positive_definite(oracle, c1):
    rp, ci, v, F, h = c1
    rng = np.random.default_rng(2)
    for _ in range(5):
        x, y = rng.standard_normal((2, len(F)))
        Bx, By = h.vcycle(x), h.vcycle(y)
        assert abs(np.dot(Bx, y) - np.dot(x, By)) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(By)
        assert np.dot(Bx, x) > 0


def test_pcg_converges_and_solves(oracle, c1):
    rp, ci, v, F, h = c1
    K = _csr(rp, ci, v)
    ustar = np.random.default_rng(4).standard_normal(len(F))
    b = K @ ustar
    r = h.solve(b, tol=1e-10)
    assert r["rc"] == 0
    assert np.linalg.norm(b - K @ r["u"]) <= 1.01e-10 * np.linalg.norm(b)
    cond = np.linalg.cond(K.toarray())
    assert np.linalg.norm(r["u"] - ustar) <= cond * 2e-10 * np.linalg.norm(ustar)
    assert r["hist"][0] == pytest.approx(1.0)
    assert r["hist"][-1] <= 1e-10


def test_flexible_cg_matches_cg_for_fixed_preconditioner(oracle, c1):
    rp, ci, v, F, h = c1
    a = h.solve(F, tol=1e-8)
    b = h.solve(F, tol=1e-8, flexible=True)
    assert abs(a["iters"] - b["iters"]) <= 1
    assert np.linalg.norm(a["u"] - b["u"]) <= 1e-7 * np.linalg.norm(a["u"])


def test_single_level_is_exact_in_one_iteration(oracle):
    rp, ci, v, F = oracle.poisson_kron(2, 3, 10)
    h = oracle.Hierarchy(rp, ci, v)
    assert h.nlevels == 1
    r = h.solve(np.random.default_rng(0).standard_normal(len(F)), tol=1e-10)
    assert r["rc"] == 0 and r["iters"] == 1


def test_zero_rhs_and_itmax_and_warm_start(oracle, c1):
    rp, ci, v, F, h = c1
    r = h.solve(np.zeros_like(F))
    assert r["rc"] == 0 and r["iters"] == 0 and not r["u"].any()
    r = h.solve(F, itmax=1)
    assert r["rc"] == 1 and r["iters"] == 1
    full = h.solve(F)
    again = h.solve(F, u0=full["u"])
    assert again["iters"] == 0 and again["rc"] == 0


def test_poly_acceptance(oracle):
    assert oracle.poly_accept([1.0, 0, 0, 0])           # l1-Jacobi: e(t) = 1 - t
    assert oracle.poly_accept([2.0, -1.0, 0, 0])        # e(t) = (1 - t)^2
    assert not oracle.poly_accept([3.0, 0, 0, 0])       # e(1) = -2
    assert not oracle.poly_accept([-0.1, 0, 0, 0])      # e(t) > 1 near 0
    # e(t) = (1-t)^4 : coefficients of 1 - e(t) = 4t - 6t^2 + 4t^3 - t^4
    assert oracle.poly_accept([4.0, -6.0, 4.0, -1.0])


def test_polynomial_smoother_vcycle_dense(oracle, c1):
    rp, ci, v, F, _ = c1
    h = oracle.Hierarchy(rp, ci, v, smoother=1)
    coef = [[2.0, -1.0, 0, 0], [4.0, -6.0, 4.0, -1.0]]
    for l in range(h.nlevels - 1):
        assert h.set_poly(l, coef[l % 2]) == 0
    assert h.set_poly(0, [3.0, 0, 0, 0]) == 1     # rejected, level keeps its coefficients
    f = np.random.default_rng(5).standard_normal(len(F))
    z = h.vcycle(f)
    ref = _dense_vcycle(h, 0, f, poly=[coef[l % 2] for l in range(h.nlevels)])
    assert np.abs(z - ref).max() <= 1e-10 * np.abs(ref).max()
    r = h.solve(F)
    assert r["rc"] == 0
