"""Oracle pins of the paper's default preconditioner (Sec. 3.1 "Variants and
efficiency", Sec. 3.2, Sec. 5.1): the fourth-kind Chebyshev smoother against
its closed-form error polynomial, the smoothed prolongator and its Galerkin
product against dense products and invariants, the coarse CG against scipy's
CG, the V-cycle against a dense recursive statement, and the operator
complexities of Table 1(c)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle


def _csr(rp, ci, v, ncols=None):
    n = len(rp) - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n if ncols is None else ncols))


def _w4(theta, k):
    # fourth-kind Chebyshev polynomial W_k(cos theta) = sin((k + 1/2) theta) / sin(theta / 2)
    return np.sin((k + 0.5) * theta) / np.sin(0.5 * theta)


def _cheb_error_op(K, invd, k):
    """p_k(D^{-1}K) = W_k(I - 2 D^{-1}K) / (2k+1) by the eigen-decomposition of
    the symmetric D^{-1/2} K D^{-1/2} and the closed form of W_k."""
    ds = np.sqrt(invd)
    As = ds[:, None] * K * ds[None, :]
    lam, Q = np.linalg.eigh(As)
    assert lam.min() > 0 and lam.max() <= 1 + 1e-12
    theta = np.arccos(np.clip(1.0 - 2.0 * lam, -1.0, 1.0))
    pk = _w4(theta, k) / (2 * k + 1)
    # S = D^{-1/2} As D^{1/2}  =>  p(S) = D^{-1/2} Q p(L) Q^T D^{1/2}
    return (ds[:, None] * (Q * pk) @ Q.T) / ds[None, :], pk, lam


def _small_system():
    rp, ci, v, _ = oracle.poisson_kron(2, 2, 7)
    K = _csr(rp, ci, v).toarray()
    invd = np.zeros(len(rp) - 1)
    oracle.lib().or_l1_invdiag(len(invd), oracle._p(rp, oracle.i64p), oracle._p(ci, oracle.i32p),
                               oracle._p(v, oracle.f64p), oracle._p(invd, oracle.f64p))
    return rp, ci, v, K, invd


@pytest.mark.parametrize("k", [1, 2, 3, 8, 12, 14, 16])
def test_cheb4_error_polynomial(k):
    rp, ci, v, K, invd = _small_system()
    rng = np.random.default_rng(k)
    n = K.shape[0]
    f = rng.standard_normal(n)
    xs = np.linalg.solve(K, f)
    E, pk, lam = _cheb_error_op(K, invd, k)
    # from a random initial guess
    x0 = rng.standard_normal(n)
    x = oracle.cheb4(rp, ci, v, invd, f, x0, degree=k)
    e0 = xs - x0
    assert np.linalg.norm((xs - x) - E @ e0) <= 1e-10 * np.linalg.norm(e0)
    # from the zero guess
    x = oracle.cheb4(rp, ci, v, invd, f, None, degree=k)
    assert np.linalg.norm((xs - x) - E @ xs) <= 1e-10 * np.linalg.norm(xs)
    # the polynomial is bounded by 1 on (0, 1] and sqrt(t) |p(t)| <= 1 / (2k+1)
    assert np.all(np.abs(pk) <= 1 + 1e-12)
    assert np.all(np.sqrt(lam) * np.abs(pk) <= 1.0 / (2 * k + 1) + 1e-12)


def test_cheb4_degree1_is_scaled_jacobi():
    rp, ci, v, K, invd = _small_system()
    f = np.random.default_rng(0).standard_normal(K.shape[0])
    x = oracle.cheb4(rp, ci, v, invd, f, None, degree=1)
    assert np.allclose(x, (4.0 / 3.0) * invd * f, rtol=0, atol=1e-15 * np.abs(x).max())


def _f1_hier(rp, ci, v, **kw):
    prm = dict(sweeps_per_level=3, smooth_prolong=1, smoother=2, cheb_degree=8, coarse_solver=0, max_coarse=40)
    prm.update(kw)
    return oracle.Hierarchy(rp, ci, v, **prm)


def _dense_tentative(agg, pc, nc):
    P = np.zeros((len(agg), nc))
    P[np.arange(len(agg)), agg] = pc
    return P


@pytest.mark.parametrize("case,omega", [("cube", 4.0 / 3.0), ("poisson3d", 4.0 / 3.0), ("cube", 1.0),
                                        ("poisson3d", 0.7)])
def test_smoothed_prolongator_and_galerkin_dense(case, omega):
    if case == "cube":
        rp, ci, v, _, _ = oracle.cube_system(2, 5)
    else:
        rp, ci, v, _ = oracle.poisson_kron(3, 2, 6)
    h = _f1_hier(rp, ci, v, omega=omega)
    assert h.rc == 0 and h.nlevels >= 2
    for l in range(h.nlevels - 1):
        K = _csr(*h.level_matrix(l)).toarray()
        agg, pc, invd, _ = h.level_agg(l)
        nc = h.level_info(l + 1)[0]
        P = _dense_tentative(agg, pc, nc)
        Pbar = P - omega * (invd[:, None] * (K @ P))
        Ps = _csr(*h.prolongator(l), ncols=nc).toarray()
        assert np.abs(Ps - Pbar).max() <= 1e-14 * np.abs(Pbar).max()
        # the pattern is that of K P (aggregates within reach of each row)
        assert np.array_equal(_csr(*h.prolongator(l), ncols=nc).toarray() != 0, (np.abs(K) @ np.abs(P)) != 0)
        Kc = _csr(*h.level_matrix(l + 1)).toarray()
        ref = Pbar.T @ K @ Pbar
        assert np.abs(Kc - ref).max() <= 1e-13 * np.abs(ref).max()
        # the damping never raises the energy of a coarse basis function
        eP = np.einsum("ij,ik,kj->j", P, K, P)
        eS = np.einsum("ij,ik,kj->j", Pbar, K, Pbar)
        assert np.all(eS <= eP * (1 + 1e-12))
        # and lowers the total energy
        assert eS.sum() < eP.sum()


def test_smoothed_prolongator_neumann_invariants():
    # pure Neumann stiffness: K 1 = 0; with w = 1 the smoothed prolongator
    # still reproduces the test vector and the coarse matrix annihilates w_c
    rp, ci, v, _ = oracle.poisson_kron_bc(2, 2, 8, [0, 0, 0, 0])
    h = _f1_hier(rp, ci, v, coarse_solver=1)
    assert h.nlevels >= 2
    for l in range(h.nlevels - 1):
        nc = h.level_info(l + 1)[0]
        Ps = _csr(*h.prolongator(l), ncols=nc)
        w = h.level_agg(l)[3]
        wc = h.level_agg(l + 1)[3]
        assert np.abs(Ps @ wc - w).max() <= 1e-12 * np.abs(w).max()
        Kc = _csr(*h.level_matrix(l + 1))
        assert np.abs(Kc @ wc).max() <= 1e-11 * abs(Kc).max() * np.abs(wc).max()


@pytest.mark.parametrize("its", [1, 2, 5, 9])
def test_cg_jacobi_against_scipy(its):
    rp, ci, v, _, _ = oracle.cube_system(2, 4)
    A = _csr(rp, ci, v)
    b = np.random.default_rng(its).standard_normal(A.shape[0])
    x, it = oracle.cg_jacobi(rp, ci, v, b, tol=0.0, itmax=its)
    assert it == its
    M = sp.diags(1.0 / A.diagonal())
    xs, info = spla.cg(A, b, rtol=0.0, atol=0.0, maxiter=its, M=M)
    assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)


def test_cg_jacobi_stopping():
    rp, ci, v, _, _ = oracle.cube_system(2, 4)
    A = _csr(rp, ci, v)
    b = np.random.default_rng(1).standard_normal(A.shape[0])
    x, it = oracle.cg_jacobi(rp, ci, v, b, tol=1e-4, itmax=1000)
    assert 0 < it < 1000
    assert np.linalg.norm(b - A @ x) <= 1.001e-4 * np.linalg.norm(b)
    # one iteration earlier the tolerance was not met
    x1, _ = oracle.cg_jacobi(rp, ci, v, b, tol=0.0, itmax=it - 1)
    assert np.linalg.norm(b - A @ x1) > 0.999e-4 * np.linalg.norm(b)
    # a small SPD system is solved exactly within n iterations
    rp2, ci2, v2, _ = oracle.poisson_kron(1, 2, 12)
    A2 = _csr(rp2, ci2, v2)
    b2 = np.arange(A2.shape[0], dtype=float)
    x2, it2 = oracle.cg_jacobi(rp2, ci2, v2, b2, tol=1e-13, itmax=100)
    assert it2 <= A2.shape[0] + 2
    assert np.allclose(x2, np.linalg.solve(A2.toarray(), b2), rtol=1e-10, atol=0)
    x0, it0 = oracle.cg_jacobi(rp2, ci2, v2, np.zeros_like(b2), tol=1e-4, itmax=30)
    assert it0 == 0 and not x0.any()


def _dense_vcycle(h, l, deg):
    """The V-cycle of level l as a dense matrix, step by step: Chebyshev
    pre-smoothing from zero, residual, P'^T, recursion (Cholesky solve at the
    coarsest level), P', Chebyshev post-smoothing."""
    K = _csr(*h.level_matrix(l)).toarray()
    n = K.shape[0]
    if l == h.nlevels - 1:
        return np.linalg.inv(K)
    invd = h.level_agg(l)[2]
    E, _, _ = _cheb_error_op(K, invd, deg)
    I = np.eye(n)
    Kinv = np.linalg.inv(K)
    nc = h.level_info(l + 1)[0]
    P = _csr(*h.prolongator(l), ncols=nc).toarray()
    Bc = _dense_vcycle(h, l + 1, deg)
    # error propagation E_post (I - P Bc P^T K) E_pre, and B = (I - that) K^{-1}
    T = E @ (I - P @ Bc @ P.T @ K) @ E
    return (I - T) @ Kinv


@pytest.mark.parametrize("deg", [1, 3, 8])
def test_vcycle_f1_dense_statement(deg):
    rp, ci, v, _ = oracle.poisson_kron(3, 2, 6)
    h = _f1_hier(rp, ci, v, cheb_degree=deg, max_coarse=10)
    assert h.nlevels >= 3
    B = _dense_vcycle(h, 0, deg)
    rng = np.random.default_rng(deg)
    for _ in range(3):
        r = rng.standard_normal(h.n)
        z = h.vcycle(r)
        assert np.linalg.norm(z - B @ r) <= 1e-10 * np.linalg.norm(B @ r)
    # same polynomial before and after, transposed transfers: B symmetric
    assert np.abs(B - B.T).max() <= 1e-10 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_vcycle_coarse_cg_solves_coarsest():
    rp, ci, v, _ = oracle.poisson_kron(3, 2, 6)
    h = _f1_hier(rp, ci, v, coarse_solver=1, coarse_tol=1e-12, coarse_itmax=500)
    hc = _f1_hier(rp, ci, v, coarse_solver=0)
    r = np.random.default_rng(3).standard_normal(h.n)
    # a CG run to 1e-12 on the coarsest level gives the Cholesky V-cycle
    assert np.linalg.norm(h.vcycle(r) - hc.vcycle(r)) <= 1e-9 * np.linalg.norm(hc.vcycle(r))


def test_table1c_operator_complexity_k12():
    with open(os.path.join(os.path.dirname(__file__), "golden", "table1c_cube_opc.json")) as f:
        opc = json.load(f)["opc"]["12"]
    deg = {3: 8, 4: 12, 5: 14, 6: 16}
    for p in (3, 4, 5):
        rp, ci, v, _, _ = oracle.cube_system(p, 12)
        h = oracle.Hierarchy(rp, ci, v, sweeps_per_level=3, smooth_prolong=1, smoother=2, cheb_degree=deg[p],
                             coarse_solver=1)
        assert abs(h.opc() - opc[str(p)]) <= 0.02, (p, h.opc())


@pytest.mark.parametrize("sweeps", [1, 3, 10])
def test_bootstrap_w(sweeps):
    from paper_2511_21268_amd.workloads import random_start
    rp, ci, v, K, invd = _small_system()
    n = K.shape[0]
    w0 = random_start(n, sweeps)
    w = oracle.bootstrap_w(rp, ci, v, w0, sweeps)
    # the iteration (I - D^{-1} K)^s w0 by dense matrix powers
    E = np.eye(n) - invd[:, None] * K
    ref = np.linalg.matrix_power(E, sweeps) @ w0
    assert np.linalg.norm(w - ref) <= 1e-13 * np.linalg.norm(ref)
    # each sweep lowers the energy (spectrum of I - D^{-1}K in [0, 1)) and the
    # Rayleigh quotient (w is smoother than the random start)
    prev = w0
    for s in range(1, sweeps + 1):
        cur = oracle.bootstrap_w(rp, ci, v, w0, s)
        assert cur @ K @ cur < prev @ K @ prev
        prev = cur
    d = 1.0 / invd
    assert (w @ K @ w) / (w @ (d * w)) < (w0 @ K @ w0) / (w0 @ (d * w0))
    assert np.array_equal(oracle.bootstrap_w(rp, ci, v, w0, 0), w0)
