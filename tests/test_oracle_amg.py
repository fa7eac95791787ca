"""Pins of the oracle's hierarchy (paper Sec. 3.1: eq. (cij), eq. (maxprod),
eq. (prolongation), Galerkin product, l1 diagonal of Sec. 3.2)."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _csr(rp, ci, v, n=None):
    n = len(rp) - 1 if n is None else n
    return sp.csr_matrix((v, ci, rp), shape=(n, n))


def _random_spd(n, density, seed):
    rng = np.random.default_rng(seed)
    A = sp.random(n, n, density=density, random_state=seed, data_rvs=lambda k: rng.uniform(-1, 1, k))
    A = (A + A.T).tocsr()
    A.setdiag(0)
    A.eliminate_zeros()
    d = np.abs(A).sum(axis=1).A1 + rng.uniform(0.1, 1.0, n)
    A = (A + sp.diags(d)).tocsr()
    A.sort_indices()
    return A


def test_cij_against_exact_rationals(oracle):
    rng = np.random.default_rng(1)
    for _ in range(200):
        kii, kjj = rng.uniform(0.5, 3, 2)
        kij = rng.uniform(-1, 1) * np.sqrt(kii * kjj)
        wi, wj = rng.uniform(-2, 2, 2)
        c = oracle.cij(kij, kii, kjj, wi, wj)
        F = Fraction
        exact = 1 - 2 * F(kij) * F(wi) * F(wj) / (F(kii) * F(wi) ** 2 + F(kjj) * F(wj) ** 2)
        assert abs(c - float(exact)) <= 8 * np.spacing(max(abs(float(exact)), 1.0))
        assert 0 < c < 2     # |k_ij| < sqrt(k_ii k_jj) and AM-GM


def test_cij_in_open_interval_for_iga_matrix(oracle):
    rp, ci, v, _ = oracle.poisson_kron(3, 3, 5)
    K = _csr(rp, ci, v)
    d = K.diagonal()
    A = sp.triu(K, 1).tocoo()
    c = np.array([oracle.cij(x, d[i], d[j], 1.0, 1.0) for i, j, x in zip(A.row, A.col, A.data)])
    assert np.all((c > 0) & (c < 2))


def _fig2():
    g = json.load(open(os.path.join(GOLD, "fig2_matching.json")))
    idx = {name: k for k, name in enumerate(g["vertices"])}
    ei = np.array([idx[a] for a, b, _ in g["edges"]], np.int32)
    ej = np.array([idx[b] for a, b, _ in g["edges"]], np.int32)
    c = np.array([w for *_, w in g["edges"]], float)
    return g, idx, ei, ej, c


def _all_matchings(n, ei, ej):
    m = len(ei)
    for r in range(0, n // 2 + 1):
        for sub in itertools.combinations(range(m), r):
            used = set()
            ok = True
            for e in sub:
                if ei[e] in used or ej[e] in used:
                    ok = False
                    break
                used.add(ei[e]); used.add(ej[e])
            if ok:
                yield sub


def test_fig2_maximum_product_by_brute_force(oracle):
    g, idx, ei, ej, c = _fig2()
    best = max(_all_matchings(4, ei, ej), key=lambda s: np.prod([c[e] for e in s]) if s else 0)
    got = sorted(tuple(sorted((g["vertices"][ei[e]], g["vertices"][ej[e]]))) for e in best)
    assert got == sorted(tuple(sorted(p)) for p in g["max_product_matching"])
    assert np.prod([c[e] for e in best]) == g["max_product"]


def test_fig2_greedy_matching(oracle):
    """Greedy in descending weight order takes A-C (6), then the only disjoint
    edge B-D (1): the matching drawn in Fig. 2(b).  With only log c > 0 edges
    eligible, B-D (weight 1, log = 0) is dropped."""
    g, idx, ei, ej, c = _fig2()
    mate = oracle.greedy_edges(4, c, ei, ej)
    assert mate[idx["A"]] == idx["C"] and mate[idx["B"]] == idx["D"]
    mate = oracle.greedy_edges(4, c, ei, ej, positive_only=True)
    assert mate[idx["A"]] == idx["C"] and mate[idx["B"]] == -1 and mate[idx["D"]] == -1


def _rank_vector(sub, order_rank):
    return sorted(order_rank[e] for e in sub)


def test_greedy_is_lexicographic_optimum_by_enumeration(oracle):
    """Among all matchings, greedy under a strict order is the one whose sorted
    edge ranks are lexicographically smallest (a missing edge ranks last).
    Checked by enumeration on random graphs of <= 9 vertices with many ties."""
    rng = np.random.default_rng(7)
    for trial in range(60):
        n = int(rng.integers(3, 10))
        pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.5]
        if not pairs:
            continue
        ei = np.array([a for a, b in pairs], np.int32)
        ej = np.array([b for a, b in pairs], np.int32)
        c = rng.integers(1, 4, len(pairs)).astype(float) / 2.0   # heavy ties
        keys = sorted(range(len(pairs)), key=lambda e: (-c[e], ei[e], ej[e]))
        rank = {e: r for r, e in enumerate(keys)}
        big = len(pairs) + 1
        best = min(_all_matchings(n, ei, ej),
                   key=lambda s: _rank_vector(s, rank) + [big] * (n // 2 + 1 - len(s)))
        mate = oracle.greedy_edges(n, c, ei, ej)
        got = {tuple(sorted((i, int(mate[i])))) for i in range(n) if mate[i] >= 0}
        assert got == {(int(ei[e]), int(ej[e])) for e in best}


def test_positive_only_greedy_half_approximation(oracle):
    """With only log c > 0 edges, greedy is a 1/2-approximation of the maximum
    of sum log c (the maximum product matching), checked by enumeration."""
    rng = np.random.default_rng(11)
    for trial in range(40):
        n = int(rng.integers(4, 10))
        pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.6]
        if not pairs:
            continue
        ei = np.array([a for a, b in pairs], np.int32)
        ej = np.array([b for a, b in pairs], np.int32)
        c = rng.uniform(0.5, 2.0, len(pairs))
        lw = np.log(c)
        opt = max(sum(lw[e] for e in s if lw[e] > 0) for s in _all_matchings(n, ei, ej))
        mate = oracle.greedy_edges(n, c, ei, ej, positive_only=True)
        gsum = 0.0
        for e in range(len(pairs)):
            if mate[ei[e]] == ej[e]:
                assert c[e] > 1
                gsum += lw[e]
        assert gsum >= 0.5 * opt - 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_match_on_matrix_is_greedy_and_maximal(oracle, seed):
    A = _random_spd(300, 0.03, seed)
    w = np.random.default_rng(seed).uniform(0.5, 1.5, 300)
    mate = oracle.match(A.indptr, A.indices, A.data, w)
    assert oracle.check_greedy(A.indptr, A.indices, A.data, mate, w) == 0
    # maximal: no edge with both ends free
    Au = sp.triu(A, 1).tocoo()
    assert not np.any((mate[Au.row] < 0) & (mate[Au.col] < 0))
    # the checker does catch a perturbed matching (planted mistake)
    matched = np.flatnonzero(mate >= 0)
    i = matched[0]; j = mate[i]
    bad = mate.copy(); bad[i] = -1; bad[j] = -1
    assert oracle.check_greedy(A.indptr, A.indices, A.data, bad, w) > 0


def test_pairwise_prolongator_orthonormal_and_reproduces_w(oracle):
    A = _random_spd(200, 0.05, 5)
    w = np.random.default_rng(5).uniform(-1.5, 1.5, 200)
    w[3] = 0.0
    mate = oracle.match(A.indptr, A.indices, A.data, w)
    agg, pc, wc = oracle.pairwise_p(mate, w)
    nc = len(wc)
    P = sp.csr_matrix((pc, agg, np.arange(201)), shape=(200, nc))
    PtP = (P.T @ P).toarray()
    assert np.abs(PtP - np.eye(nc)).max() <= 4 * np.finfo(float).eps
    assert np.allclose(P @ wc, w, rtol=0, atol=4 * np.finfo(float).eps * 2)
    # coarse numbering follows the smallest member
    first = {}
    for i in range(200):
        first.setdefault(agg[i], i)
    assert list(first.keys()) == sorted(first.keys())


@pytest.mark.parametrize("sweeps", [1, 2])
def test_galerkin_equals_dense_product(oracle, sweeps):
    rp, ci, v, _ = oracle.poisson_kron(2, 2, 14)
    h = oracle.Hierarchy(rp, ci, v, sweeps_per_level=sweeps, max_coarse=10)
    assert h.nlevels >= 3
    for l in range(h.nlevels - 1):
        Kl = _csr(*h.level_matrix(l)).toarray()
        agg, pc, invd, w = h.level_agg(l)
        nc = h.level_info(l + 1)[0]
        assert agg.max() == nc - 1 and np.bincount(agg).max() <= 2 ** sweeps
        P = np.zeros((len(agg), nc)); P[np.arange(len(agg)), agg] = pc
        Kc = _csr(*h.level_matrix(l + 1)).toarray()
        ref = P.T @ Kl @ P
        assert np.abs(Kc - ref).max() <= 1e-14 * np.abs(ref).max()
        assert np.linalg.eigvalsh(0.5 * (Kc + Kc.T)).min() > 0
        wc = h.level_agg(l + 1)[3]
        assert np.allclose(P @ wc, w, rtol=0, atol=1e-15)
        assert np.abs(P.T @ P - np.eye(nc)).max() < 1e-15


def test_l1_diagonal_and_smoother_contraction(oracle):
    rp, ci, v, _ = oracle.poisson_kron(3, 3, 4)
    K = _csr(rp, ci, v).toarray()
    invd = oracle.l1_invdiag(rp, ci, v)
    d = np.abs(K).sum(axis=1)
    assert np.allclose(invd, 1.0 / d, rtol=1e-15)
    # D - K weakly diagonally dominant: spectrum of D^{-1}K in (0, 1]
    S = np.diag(np.sqrt(invd)) @ K @ np.diag(np.sqrt(invd))
    ev = np.linalg.eigvalsh(S)
    assert ev.min() > 0 and ev.max() <= 1 + 1e-14
    # rho(I - D^{-1}K) < 1 by power iteration
    x = np.random.default_rng(0).standard_normal(K.shape[0])
    for _ in range(300):
        x = x - invd * (K @ x)
        x /= np.linalg.norm(x)
    assert np.linalg.norm(x - invd * (K @ x)) < 1.0


def test_cholesky_against_numpy(oracle):
    rng = np.random.default_rng(3)
    B = rng.standard_normal((60, 60))
    A = B @ B.T + 60 * np.eye(60)
    L = oracle.cholesky(A)
    assert np.allclose(L, np.linalg.cholesky(A), rtol=1e-13, atol=1e-13)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.cholesky(-A)


def test_hierarchy_sizes_and_stop_rule(oracle):
    rp, ci, v, _ = oracle.poisson_kron(2, 2, 32)
    h = oracle.Hierarchy(rp, ci, v)
    sizes = [h.level_info(l)[0] for l in range(h.nlevels)]
    assert sizes[0] == 1024 and sizes[-1] <= 200 and all(s > 200 for s in sizes[:-1])
    assert all(b <= a for a, b in zip(sizes, sizes[1:]))
    L = h.coarse_factor()
    Kc = _csr(*h.level_matrix(h.nlevels - 1)).toarray()
    assert np.allclose(L @ L.T, np.tril(Kc) + np.tril(Kc, -1).T, rtol=0, atol=1e-12 * np.abs(Kc).max())
    # a small system is a single level
    rp, ci, v, _ = oracle.poisson_kron(2, 2, 12)
    assert oracle.Hierarchy(rp, ci, v).nlevels == 1


def test_setup_rejects_bad_input(oracle):
    rp = np.array([0, 1, 2]); ci = np.array([0, 1]); v = np.array([1.0, -1.0])
    with pytest.raises(ValueError):
        oracle.Hierarchy(rp, ci, v)
    v = np.array([1.0, np.nan])
    with pytest.raises(ValueError):
        oracle.Hierarchy(rp, ci, v)
