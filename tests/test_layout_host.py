"""The device matrix layout on the host (no GPU): amg_sell_spmv_host builds the
library's SELL image and walks it as the matrix-pass kernels do.  Every layout
must give K x (checked against an independent CSR product), read only columns
in range, and -- since every row is summed in ascending column order and the
extra entries are exact zeros -- the same bits in every layout."""
import numpy as np
import pytest
import scipy.sparse as sp


@pytest.fixture(scope="module")
def amg():
    import paper_2511_21268_amd as m
    m.lib()
    return m


def _cases(oracle):
    from paper_2511_21268_amd.workloads import kappa_params
    out = {}
    out["2d-p2"] = oracle.poisson_kron(2, 2, 32)[:3]
    out["3d-p3"] = oracle.poisson_kron(3, 3, 12)[:3]
    a, mk = kappa_params(5)
    out["3d-kappa-p5"] = oracle.diffusion_quad3d(5, 6, a, mk, factorized=True)[:3]
    rp, ci, v, _ = oracle.poisson_kron(3, 2, 10)
    K = sp.csr_matrix((v, ci, rp), shape=(len(rp) - 1,) * 2)
    perm = np.random.default_rng(3).permutation(K.shape[0])
    Kp = sp.csr_matrix(K[perm][:, perm]); Kp.sort_indices()
    out["permuted"] = (Kp.indptr, Kp.indices, Kp.data)
    # column gaps beyond 16 bits: int32 columns
    n = 70000
    A = sp.diags([np.full(n, 4.0), np.full(n - 66000, -1.0), np.full(n - 66000, -1.0)], [0, 66000, -66000], format="csr")
    A.sort_indices()
    out["wide-gaps"] = (A.indptr, A.indices, A.data)
    return out


def _ref(rp, ci, v, x, ncols):
    K = sp.csr_matrix((v, ci, rp), shape=(len(rp) - 1, ncols))
    return K @ x, abs(K) @ np.abs(x)


@pytest.mark.parametrize("C", [64, 16, 4])
def test_layouts_compute_Kx(oracle, amg, C):
    for name, (rp, ci, v) in _cases(oracle).items():
        n = len(rp) - 1
        x = np.random.default_rng(1).standard_normal(n)
        ref, scale = _ref(rp, ci, v, x, n)
        ys = []
        # layouts 3 and 4 (C = 64 only): shared-offset slices through the
        # block kernels' staged x windows (runs of consecutive offsets), per
        # wave and shared by the four slices of a block
        for layout in ((0, 1, 2, 3, 4) if C == 64 else (0, 1, 2)):
            y, shared, stored = amg.sell_spmv_host(rp, ci, v, x, C_slice=C, layout=layout)
            assert np.all(np.abs(y - ref) <= 8 * np.finfo(float).eps * scale + 1e-300), (name, layout)
            assert stored >= len(v)
            if layout in (0, 2):
                assert shared == 0
            ys.append(y)
            if layout in (1, 3, 4) and name in ("2d-p2", "3d-p3", "3d-kappa-p5") and C == 64:
                assert shared > 0, name
        for y in ys[1:]:
            assert np.array_equal(ys[0], y), name


def test_rectangular_KP_image(oracle, amg):
    """K P (one column per aggregate) in the sorted layout: the columns a lane
    walks stay inside the coarse range."""
    rp, ci, v, _ = oracle.poisson_kron(3, 3, 10)
    h = oracle.Hierarchy(rp, ci, v)
    agg, pc = h.level_agg(0)[:2]
    n, nc = len(rp) - 1, int(agg.max()) + 1
    K = sp.csr_matrix((v, ci, rp), shape=(n, n))
    P = sp.csr_matrix((pc, (np.arange(n), agg)), shape=(n, nc))
    KP = (K @ P).tocsr(); KP.sort_indices()
    e = np.random.default_rng(2).standard_normal(nc)
    ref, scale = _ref(KP.indptr, KP.indices, KP.data, e, nc)
    for C in (64, 16, 4):
        for layout in (0, 2):
            y, _, _ = amg.sell_spmv_host(KP.indptr, KP.indices, KP.data, e, C_slice=C, layout=layout, ncols=nc)
            assert np.all(np.abs(y - ref) <= 8 * np.finfo(float).eps * scale + 1e-300), (C, layout)
    with pytest.raises(amg.AmgError):                   # shared offsets only for square matrices
        amg.sell_spmv_host(KP.indptr, KP.indices, KP.data, e, C_slice=64, layout=1, ncols=nc)


def test_sorted_windows_reduce_padding(oracle, amg):
    rp, ci, v, _ = oracle.poisson_kron(3, 3, 12)
    h = oracle.Hierarchy(rp, ci, v)
    rpl, cil, vl = h.level_matrix(1)
    x = np.random.default_rng(4).standard_normal(len(rpl) - 1)
    _, _, plain = amg.sell_spmv_host(rpl, cil, vl, x, C_slice=64, layout=0)
    _, _, srt = amg.sell_spmv_host(rpl, cil, vl, x, C_slice=64, layout=2)
    assert srt < plain


def test_window_walk_edge_cases(oracle, amg):
    """The staged-window walk on stencils whose x-runs are longer than one
    window (p = 5: runs of 11 split 8 + 3), whose slices straddle x-lines and
    planes (n + p - 2 not a multiple of 64), a single short slice, and a
    partially filled last slice: bitwise the gather walk."""
    cases = [(oracle.poisson_kron(2, 5, 64)[:3], True),    # x-runs of 11: windows of 8 + 3
             (oracle.poisson_kron(2, 3, 70)[:3], True),    # slices straddle x-lines
             (oracle.poisson_kron(3, 1, 66)[:3], True),    # and planes; runs of 3
             (oracle.poisson_kron(2, 2, 61)[:3], True),    # last slice partly filled
             (oracle.poisson_kron(2, 3, 3)[:3], False)]    # one slice of 16 rows, no shared list
    for (rp, ci, v), shared in cases:
        n = len(rp) - 1
        x = np.random.default_rng(n).standard_normal(n)
        y1, sh1, _ = amg.sell_spmv_host(rp, ci, v, x, C_slice=64, layout=1)
        y3, sh3, _ = amg.sell_spmv_host(rp, ci, v, x, C_slice=64, layout=3)
        y4, sh4, _ = amg.sell_spmv_host(rp, ci, v, x, C_slice=64, layout=4)
        assert sh1 == sh3 == sh4 and (sh3 > 0) == shared, n
        assert np.array_equal(y1, y3), n
        assert np.array_equal(y1, y4), n
    rp, ci, v = cases[0][0]
    for layout in (3, 4):
        with pytest.raises(Exception):
            amg.sell_spmv_host(rp, ci, v, np.zeros(len(rp) - 1), C_slice=16, layout=layout)
