"""Oracle pins of the paper's cube benchmark (Sec. 5.1): -Lap u = f on the unit
cube with u = exp(x+z) sin(y), Dirichlet on three faces and Neumann data on the
other three.  The matrix sizes are those of Table 1(b); the discrete solution
converges to u in L2 at the optimal rate p+1, which fails if any part of the
right-hand side (source, a Neumann face or its sign, the Dirichlet lifting) or
the choice of Dirichlet faces is wrong."""
import json
import os

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_sizes_table_1b(oracle):
    with open(os.path.join(GOLDEN, "table1b_cube_sizes.json")) as f:
        g = json.load(f)
    for k, row in g["sizes"].items():
        for p, N in row.items():
            assert oracle.cube_size(int(p), int(k))[0] == N, (k, p)


def _solve(oracle, p, n):
    rp, ci, v, F, lift = oracle.cube_system(p, n)
    N = len(rp) - 1
    K = sp.csr_matrix((v, ci, rp), shape=(N, N))
    u0 = sla.spsolve(K.tocsc(), F)
    e, nr = oracle.cube_error(p, n, u0, lift)
    return e / nr


def test_optimal_l2_convergence(oracle):
    for p in (2, 3):
        errs = [_solve(oracle, p, n) for n in (4, 8, 16)]
        rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
        assert all(r > p + 0.8 for r in rates), (p, errs, rates)
    assert _solve(oracle, 3, 16) < 5e-8
    # p = 4 on 3, 6, 12 elements per edge: rate 5 (measured 5.02, 4.96)
    errs = [_solve(oracle, 4, n) for n in (3, 6, 12)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(r > 4.8 for r in rates), (errs, rates)


def test_lifting_is_the_projection_on_the_dirichlet_faces(oracle):
    """Dirichlet coefficients of the lifting reproduce g_D: the full-space
    function built from the lifting alone equals u on the face x = 0 up to
    the projection's accuracy (checked at sample points via the basis)."""
    p, n = 3, 8
    rp, ci, v, F, lift = oracle.cube_system(p, n)
    m = n + p
    c = lift.reshape(m, m, m)           # [k][j][i]
    t = oracle.knots(p, n)
    ys = np.linspace(0.05, 0.95, 7)
    zs = np.linspace(0.05, 0.95, 7)
    for y in ys:
        for z in zs:
            by = np.array([oracle.bspline(t, j, p, y) for j in range(m)])
            bz = np.array([oracle.bspline(t, k, p, z) for k in range(m)])
            val = np.einsum("kj,j,k->", c[:, :, 0], by, bz)      # N_0(0) = 1 on x = 0
            assert abs(val - np.exp(z) * np.sin(y)) < 1e-5, (y, z)


def test_library_generator_matches_oracle(oracle):
    """The library's cube generator (its own assembly, lifting through
    separable Kronecker terms) against the oracle's (direct sums)."""
    import paper_2511_21268_amd as amg
    amg.lib()
    for p, n in [(2, 9), (3, 6), (4, 5), (5, 4), (6, 3)]:
        rp, ci, v, F = amg.iga_cube(p, n)
        ro, co, vo, Fo, _ = oracle.cube_system(p, n)
        assert np.array_equal(rp, ro) and np.array_equal(ci, co), (p, n)
        assert np.abs(v - vo).max() <= 4e-15 * np.abs(vo).max(), (p, n)
        assert np.abs(F - Fo).max() <= 1e-13 * np.abs(Fo).max(), (p, n)
