"""CPU oracle (ctypes binding of liboracle.so built from oracle/*.c).

TEST INFRASTRUCTURE ONLY: the plain FP64 statement of the method of D'Ambra,
Durastante, Filippone (arXiv 2511.21268) -- IgA assembly (Sec. 2), the
matching-based AMG hierarchy (Sec. 3.1), the l1-Jacobi V-cycle and CG / flexible
CG (Sec. 3, 3.2, 4).  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import it; the HIP library never does, and this package
imports nothing from the library.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC = ["iga.c", "cube.c", "amg.c", "krylov.c", "mlp.c"]


def build(force=True):
    """Compile liboracle.so with gcc (no FMA contraction, OpenMP row loops)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-o", _LIB + ".tmp"] + [os.path.join(_HERE, s) for s in _SRC] + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None

i64p = C.POINTER(C.c_int64)
i32p = C.POINTER(C.c_int32)
f64p = C.POINTER(C.c_double)


class Params(C.Structure):
    _fields_ = [("sweeps_per_level", C.c_int), ("max_coarse", C.c_int), ("max_levels", C.c_int),
                ("nu_pre", C.c_int), ("nu_post", C.c_int), ("match_positive_only", C.c_int),
                ("smoother", C.c_int), ("smooth_prolong", C.c_int), ("cheb_degree", C.c_int),
                ("coarse_solver", C.c_int), ("coarse_itmax", C.c_int), ("omega", C.c_double),
                ("coarse_tol", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.or_gauss_legendre.argtypes = [C.c_int, f64p, f64p]
        L.or_knots.argtypes = [C.c_int, C.c_int, f64p]
        L.or_bspline.argtypes = [f64p, C.c_int, C.c_int, C.c_double]
        L.or_bspline.restype = C.c_double
        L.or_bspline_deriv.argtypes = [f64p, C.c_int, C.c_int, C.c_double]
        L.or_bspline_deriv.restype = C.c_double
        L.or_matrices_1d.argtypes = [C.c_int, C.c_int, f64p, f64p, f64p]
        L.or_poisson_size.argtypes = [C.c_int, C.c_int, C.c_int, i64p, i64p]
        L.or_poisson_kron.argtypes = [C.c_int, C.c_int, C.c_int, i64p, i32p, f64p, f64p]
        L.or_tensor_size.argtypes = [C.c_int, C.c_int, C.c_int, i32p, i64p, i64p]
        L.or_poisson_kron_bc.argtypes = [C.c_int, C.c_int, C.c_int, i32p, i64p, i32p, f64p, f64p]
        L.or_greedy_edges.argtypes = [C.c_int64, C.c_int64, f64p, i32p, i32p, C.c_int, i32p]
        L.or_diffusion_quad3d.argtypes = [C.c_int, C.c_int, C.c_int, f64p, i32p, i64p, i32p, f64p, f64p]
        L.or_cube_size.argtypes = [C.c_int, C.c_int, i64p, i64p]
        L.or_cube_system.argtypes = [C.c_int, C.c_int, i64p, i32p, f64p, f64p, f64p]
        L.or_cube_embed.argtypes = [C.c_int, C.c_int, f64p, f64p, f64p]
        L.or_cube_error.argtypes = [C.c_int, C.c_int, f64p, f64p, f64p]
        L.or_diffusion_sf3d.argtypes = [C.c_int, C.c_int, C.c_int, f64p, i32p, i64p, i32p, f64p, f64p]
        L.or_cij.argtypes = [C.c_double] * 5
        L.or_cij.restype = C.c_double
        L.or_match.argtypes = [C.c_int64, i64p, i32p, f64p, f64p, C.c_int, i32p]
        L.or_check_greedy.argtypes = [C.c_int64, i64p, i32p, f64p, f64p, C.c_int, i32p]
        L.or_check_greedy.restype = C.c_int64
        L.or_pairwise_p.argtypes = [C.c_int64, i32p, f64p, i32p, f64p, f64p]
        L.or_pairwise_p.restype = C.c_int64
        L.or_l1_invdiag.argtypes = [C.c_int64, i64p, i32p, f64p, f64p]
        L.or_cholesky.argtypes = [C.c_int, f64p]
        L.or_chol_solve.argtypes = [C.c_int, f64p, f64p, f64p]
        L.or_params_default.argtypes = [C.POINTER(Params)]
        L.or_setup.argtypes = [C.c_int64, i64p, i32p, f64p, f64p, C.POINTER(Params), C.POINTER(C.c_void_p)]
        L.or_free.argtypes = [C.c_void_p]
        L.or_set_verbose.argtypes = [C.c_int]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_dot_order.argtypes = [C.c_int]
        L.or_nlevels.argtypes = [C.c_void_p]
        L.or_level_info.argtypes = [C.c_void_p, C.c_int, i64p, i64p]
        L.or_level_matrix.argtypes = [C.c_void_p, C.c_int, i64p, i32p, f64p]
        L.or_level_agg.argtypes = [C.c_void_p, C.c_int, i32p, f64p, f64p, f64p]
        L.or_coarse_factor.argtypes = [C.c_void_p, f64p]
        L.or_set_poly.argtypes = [C.c_void_p, C.c_int, f64p]
        L.or_level_pnnz.argtypes = [C.c_void_p, C.c_int]
        L.or_level_pnnz.restype = C.c_int64
        L.or_level_prolongator.argtypes = [C.c_void_p, C.c_int, i64p, i32p, f64p]
        L.or_cheb4.argtypes = [C.c_int64, i64p, i32p, f64p, f64p, f64p, f64p, C.c_int, C.c_int]
        L.or_block_fcg.argtypes = [C.c_void_p, C.c_int, f64p, f64p, C.c_double, C.c_int, C.POINTER(C.c_int), f64p]
        L.or_bootstrap_w.argtypes = [C.c_int64, i64p, i32p, f64p, f64p, C.c_int, f64p]
        L.or_cg_jacobi.argtypes = [C.c_int64, i64p, i32p, f64p, f64p, f64p, C.c_double, C.c_int]
        L.or_spmv.argtypes = [C.c_int64, i64p, i32p, f64p, f64p, f64p]
        L.or_dot.argtypes = [C.c_int64, f64p, f64p]
        L.or_dot.restype = C.c_double
        L.or_vcycle.argtypes = [C.c_void_p, C.c_int, f64p, f64p]
        L.or_pcg.argtypes = [C.c_void_p, f64p, f64p, C.c_double, C.c_int, C.c_int,
                             C.POINTER(C.c_int), f64p, f64p]
        L.or_poly_accept.argtypes = [f64p]
        u16p = C.POINTER(C.c_uint16)
        L.or_mlp_forward.argtypes = [u16p, f64p, C.c_int, f64p]
        L.or_mlp_loss_grad.argtypes = [u16p, f64p, f64p, C.c_int, f64p]
        L.or_mlp_loss_grad.restype = C.c_double
        L.or_mlp_loss_grad_w.argtypes = [f64p, f64p, f64p, C.c_int, f64p]
        L.or_mlp_loss_grad_w.restype = C.c_double
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


# ---------------------------------------------------------------- Sec. 2
def gauss_legendre(q):
    x = np.zeros(q); w = np.zeros(q)
    lib().or_gauss_legendre(q, _p(x, f64p), _p(w, f64p))
    return x, w


def knots(p, n):
    t = np.zeros(n + 2 * p + 1)
    lib().or_knots(p, n, _p(t, f64p))
    return t


def bspline(t, i, p, x, deriv=False):
    t = _f64(t)
    f = lib().or_bspline_deriv if deriv else lib().or_bspline
    return f(_p(t, f64p), i, p, float(x))


def matrices_1d(p, n):
    """Full 1D mass M, stiffness K (m x m, m = n+p) and basis integrals."""
    m = n + p
    M = np.zeros((m, m)); K = np.zeros((m, m)); F = np.zeros(m)
    lib().or_matrices_1d(p, n, _p(M, f64p), _p(K, f64p), _p(F, f64p))
    return M, K, F


def poisson_size(d, p, n):
    N = C.c_int64(); nz = C.c_int64()
    lib().or_poisson_size(d, p, n, C.byref(N), C.byref(nz))
    return N.value, nz.value


def poisson_kron(d, p, n, want_F=True):
    """CSR (indptr int64, indices int32, data f64) of the Dirichlet-reduced
    constant-coefficient stiffness matrix, and F for f = 1."""
    N, nz = poisson_size(d, p, n)
    rp = np.zeros(N + 1, np.int64); ci = np.zeros(nz, np.int32); v = np.zeros(nz)
    F = np.zeros(N) if want_F else None
    rc = lib().or_poisson_kron(d, p, n, _p(rp, i64p), _p(ci, i32p), _p(v, f64p),
                               _p(F, f64p) if want_F else None)
    if rc:
        raise ValueError("or_poisson_kron failed")
    return rp, ci, v, F


def tensor_size(d, p, n, dirichlet):
    """(N, nnz) with Dirichlet on the flagged faces: dirichlet = [[x_lo, x_hi],
    [y_lo, y_hi], [z_lo, z_hi]] (first d rows used)."""
    fl = _i32(np.asarray(dirichlet, dtype=np.int32).reshape(-1))
    N = C.c_int64(); nz = C.c_int64()
    lib().or_tensor_size(d, p, n, _p(fl, i32p), C.byref(N), C.byref(nz))
    return N.value, nz.value


def poisson_kron_bc(d, p, n, dirichlet):
    fl = _i32(np.asarray(dirichlet, dtype=np.int32).reshape(-1))
    N, nz = tensor_size(d, p, n, dirichlet)
    rp = np.zeros(N + 1, np.int64); ci = np.zeros(nz, np.int32); v = np.zeros(nz); F = np.zeros(N)
    rc = lib().or_poisson_kron_bc(d, p, n, _p(fl, i32p), _p(rp, i64p), _p(ci, i32p), _p(v, f64p), _p(F, f64p))
    if rc:
        raise ValueError("or_poisson_kron_bc failed")
    return rp, ci, v, F


# ---------------------------------------------------------------- Sec. 5.1 cube
def cube_size(p, n):
    N = C.c_int64(); nz = C.c_int64()
    lib().or_cube_size(p, n, C.byref(N), C.byref(nz))
    return N.value, nz.value


def cube_system(p, n):
    """The paper's cube problem: (rp, ci, v, F, lift), lift in full-space order."""
    N, nz = cube_size(p, n)
    m = n + p
    rp = np.zeros(N + 1, np.int64); ci = np.zeros(nz, np.int32); v = np.zeros(nz); F = np.zeros(N)
    lift = np.zeros(m ** 3)
    rc = lib().or_cube_system(p, n, _p(rp, i64p), _p(ci, i32p), _p(v, f64p), _p(F, f64p), _p(lift, f64p))
    if rc:
        raise ValueError("or_cube_system failed")
    return rp, ci, v, F, lift


def cube_error(p, n, u0, lift):
    """(||u_h - u||_L2, ||u||_L2) for the interior solution u0."""
    m = n + p
    uf = np.zeros(m ** 3)
    u0 = _f64(u0); lift = _f64(lift)
    lib().or_cube_embed(p, n, _p(u0, f64p), _p(lift, f64p), _p(uf, f64p))
    e = C.c_double(); nr = C.c_double()
    lib().or_cube_error(p, n, _p(uf, f64p), C.byref(e), C.byref(nr))
    return e.value, nr.value


def diffusion_quad3d(p, n, a=None, mk=None, factorized=False):
    """3D stiffness with kappa(x) = exp(0.5 sum a_k cos(2 pi m_k.x)) by (p+1)^3
    Gauss points per element: the plain element loop, or (factorized=True)
    sum factorization; a = None gives kappa = 1."""
    N, nz = poisson_size(3, p, n)
    rp = np.zeros(N + 1, np.int64); ci = np.zeros(nz, np.int32); v = np.zeros(nz); F = np.zeros(N)
    nk = 0 if a is None else len(a)
    a_ = _f64(a if a is not None else np.zeros(1))
    m_ = _i32(mk if mk is not None else np.zeros((1, 3), np.int32)).reshape(-1)
    fn = lib().or_diffusion_sf3d if factorized else lib().or_diffusion_quad3d
    rc = fn(p, n, nk, _p(a_, f64p), _p(m_, i32p), _p(rp, i64p), _p(ci, i32p), _p(v, f64p), _p(F, f64p))
    if rc:
        raise ValueError("or_diffusion_quad3d failed")
    return rp, ci, v, F


# ---------------------------------------------------------------- Sec. 3.1
def cij(kij, kii, kjj, wi, wj):
    return lib().or_cij(kij, kii, kjj, wi, wj)


def match(rp, ci, v, w=None, positive_only=False):
    rp = _i64(rp); ci = _i32(ci); v = _f64(v)
    n = len(rp) - 1
    w = _f64(np.ones(n) if w is None else w)
    mate = np.zeros(n, np.int32)
    lib().or_match(n, _p(rp, i64p), _p(ci, i32p), _p(v, f64p), _p(w, f64p), int(positive_only), _p(mate, i32p))
    return mate


def greedy_edges(n, c, ei, ej, positive_only=False):
    c = _f64(c); ei = _i32(ei); ej = _i32(ej)
    mate = np.zeros(n, np.int32)
    lib().or_greedy_edges(n, len(c), _p(c, f64p), _p(ei, i32p), _p(ej, i32p), int(positive_only), _p(mate, i32p))
    return mate


def check_greedy(rp, ci, v, mate, w=None, positive_only=False):
    """Number of violations of the greedy characterisation (0 = greedy)."""
    rp = _i64(rp); ci = _i32(ci); v = _f64(v); mate = _i32(mate)
    n = len(rp) - 1
    w = _f64(np.ones(n) if w is None else w)
    return lib().or_check_greedy(n, _p(rp, i64p), _p(ci, i32p), _p(v, f64p), _p(w, f64p),
                                 int(positive_only), _p(mate, i32p))


def pairwise_p(mate, w):
    mate = _i32(mate); w = _f64(w)
    n = len(mate)
    agg = np.zeros(n, np.int32); pc = np.zeros(n); wc = np.zeros(n)
    nc = lib().or_pairwise_p(n, _p(mate, i32p), _p(w, f64p), _p(agg, i32p), _p(pc, f64p), _p(wc, f64p))
    return agg, pc, wc[:nc].copy()


def l1_invdiag(rp, ci, v):
    rp = _i64(rp); ci = _i32(ci); v = _f64(v)
    n = len(rp) - 1
    out = np.zeros(n)
    lib().or_l1_invdiag(n, _p(rp, i64p), _p(ci, i32p), _p(v, f64p), _p(out, f64p))
    return out


def cholesky(A):
    L = _f64(np.array(A, dtype=np.float64, copy=True))
    rc = lib().or_cholesky(L.shape[0], _p(L, f64p))
    if rc:
        raise np.linalg.LinAlgError("not SPD")
    return L


def chol_solve(L, b):
    L = _f64(L); b = _f64(b); x = np.zeros_like(b)
    lib().or_chol_solve(L.shape[0], _p(L, f64p), _p(b, f64p), _p(x, f64p))
    return x


def spmv(rp, ci, v, x):
    rp = _i64(rp); ci = _i32(ci); v = _f64(v); x = _f64(x)
    y = np.zeros(len(rp) - 1)
    lib().or_spmv(len(rp) - 1, _p(rp, i64p), _p(ci, i32p), _p(v, f64p), _p(x, f64p), _p(y, f64p))
    return y


def dot(x, y):
    x = _f64(x); y = _f64(y)
    return lib().or_dot(len(x), _p(x, f64p), _p(y, f64p))


def set_verbose(v):
    lib().or_set_verbose(int(v))


def poly_accept(coef):
    c = _f64(coef)
    return bool(lib().or_poly_accept(_p(c, f64p)))


# ---------------------------------------------------------------- MLP
MLP_NPARAM = 4996


def _u16(a):
    return np.ascontiguousarray(a, dtype=np.uint16)


def mlp_forward(w_bf16, X):
    w = _u16(w_bf16); X = _f64(X)
    B = X.shape[0]
    Y = np.zeros((B, 4))
    lib().or_mlp_forward(w.ctypes.data_as(C.POINTER(C.c_uint16)), _p(X, f64p), B, _p(Y, f64p))
    return Y


def mlp_loss_grad(w_bf16, X, T):
    w = _u16(w_bf16); X = _f64(X); T = _f64(T)
    g = np.zeros(MLP_NPARAM)
    loss = lib().or_mlp_loss_grad(w.ctypes.data_as(C.POINTER(C.c_uint16)), _p(X, f64p), _p(T, f64p), X.shape[0],
                                  _p(g, f64p))
    return loss, g


def mlp_loss_w(w, X, T):
    """Loss at real-valued parameters w (for finite differences)."""
    w = _f64(w); X = _f64(X); T = _f64(T)
    return lib().or_mlp_loss_grad_w(_p(w, f64p), _p(X, f64p), _p(T, f64p), X.shape[0], None)


class Hierarchy:
    """or_setup + accessors + V-cycle + CG on the oracle's hierarchy."""

    def __init__(self, rp, ci, v, w=None, **kw):
        prm = Params()
        lib().or_params_default(C.byref(prm))
        for k, val in kw.items():
            setattr(prm, k, float(val) if k in ("omega", "coarse_tol") else int(val))
        self._keep = (_i64(rp), _i32(ci), _f64(v))
        rp, ci, v = self._keep
        n = len(rp) - 1
        wv = None if w is None else _f64(w)
        h = C.c_void_p()
        self.rc = lib().or_setup(n, _p(rp, i64p), _p(ci, i32p), _p(v, f64p),
                                 _p(wv, f64p) if wv is not None else None, C.byref(prm), C.byref(h))
        self.h = h
        self.n = n
        if self.rc == -1:
            raise ValueError("oracle setup: bad argument")

    def __del__(self):
        if getattr(self, "h", None) and self.h.value:
            lib().or_free(self.h)
            self.h = None

    @property
    def nlevels(self):
        return lib().or_nlevels(self.h)

    def level_info(self, l):
        n = C.c_int64(); nz = C.c_int64()
        lib().or_level_info(self.h, l, C.byref(n), C.byref(nz))
        return n.value, nz.value

    def level_matrix(self, l):
        n, nz = self.level_info(l)
        rp = np.zeros(n + 1, np.int64); ci = np.zeros(nz, np.int32); v = np.zeros(nz)
        lib().or_level_matrix(self.h, l, _p(rp, i64p), _p(ci, i32p), _p(v, f64p))
        return rp, ci, v

    def level_agg(self, l):
        n, _ = self.level_info(l)
        agg = np.full(n, -1, np.int32); pc = np.zeros(n); invd = np.zeros(n); w = np.zeros(n)
        lib().or_level_agg(self.h, l, _p(agg, i32p), _p(pc, f64p), _p(invd, f64p), _p(w, f64p))
        return agg, pc, invd, w

    def coarse_factor(self):
        n, _ = self.level_info(self.nlevels - 1)
        L = np.zeros((n, n))
        lib().or_coarse_factor(self.h, _p(L, f64p))
        return L

    def set_poly(self, l, coef):
        c = _f64(coef)
        return lib().or_set_poly(self.h, l, _p(c, f64p))

    def prolongator(self, l):
        """The smoothed prolongator of level l as CSR (None without smoothing)."""
        nz = lib().or_level_pnnz(self.h, l)
        if nz == 0:
            return None
        n, _ = self.level_info(l)
        rp = np.zeros(n + 1, np.int64); ci = np.zeros(nz, np.int32); v = np.zeros(nz)
        lib().or_level_prolongator(self.h, l, _p(rp, i64p), _p(ci, i32p), _p(v, f64p))
        return rp, ci, v

    def opc(self):
        nz0 = self.level_info(0)[1]
        return sum(self.level_info(l)[1] for l in range(self.nlevels)) / nz0

    def vcycle(self, r, level=0):
        r = _f64(r); z = np.zeros_like(r)
        lib().or_vcycle(self.h, level, _p(r, f64p), _p(z, f64p))
        return z

    def block_solve(self, F, U0=None, tol=1e-8, itmax=1000):
        """Block flexible CG for the columns of F (n x s)."""
        F = np.asarray(F, np.float64)
        n, s = F.shape
        Fc = np.ascontiguousarray(F.T)
        U = np.zeros_like(Fc) if U0 is None else np.ascontiguousarray(np.asarray(U0, np.float64).T)
        it = (C.c_int * s)(); rel = np.zeros(s)
        rc = lib().or_block_fcg(self.h, s, _p(Fc, f64p), _p(U, f64p), tol, itmax, it, _p(rel, f64p))
        return dict(rc=rc, U=U.T.copy(), iters=np.array(list(it)), relres=rel)

    def solve(self, F, u0=None, tol=1e-8, itmax=1000, flexible=False):
        F = _f64(F)
        u = np.zeros_like(F) if u0 is None else _f64(np.array(u0, copy=True))
        it = C.c_int(); rel = C.c_double(); hist = np.zeros(itmax + 1)
        rc = lib().or_pcg(self.h, _p(F, f64p), _p(u, f64p), tol, itmax, int(flexible),
                          C.byref(it), C.byref(rel), _p(hist, f64p))
        return dict(rc=rc, u=u, iters=it.value, relres=rel.value, hist=hist[: it.value + 1].copy())


def cheb4(rp, ci, v, invd, f, x0=None, degree=8):
    """Fourth-kind Chebyshev smoother of the given degree (x0 None: from zero)."""
    rp, ci, v, invd, f = _i64(rp), _i32(ci), _f64(v), _f64(invd), _f64(f)
    x = np.zeros_like(f) if x0 is None else _f64(np.array(x0, copy=True))
    lib().or_cheb4(len(f), _p(rp, i64p), _p(ci, i32p), _p(v, f64p), _p(invd, f64p), _p(f, f64p),
                   _p(x, f64p), int(x0 is None), int(degree))
    return x


def cg_jacobi(rp, ci, v, b, tol=1e-4, itmax=30):
    """Jacobi-preconditioned CG from zero; returns (x, iterations)."""
    rp, ci, v, b = _i64(rp), _i32(ci), _f64(v), _f64(b)
    x = np.zeros_like(b)
    it = lib().or_cg_jacobi(len(b), _p(rp, i64p), _p(ci, i32p), _p(v, f64p), _p(b, f64p), _p(x, f64p),
                            float(tol), int(itmax))
    return x, it


def bootstrap_w(rp, ci, v, w0, sweeps):
    """Test vector: `sweeps` l1-Jacobi sweeps on K w = 0 from w0."""
    rp, ci, v, w0 = _i64(rp), _i32(ci), _f64(v), _f64(w0)
    w = np.zeros_like(w0)
    lib().or_bootstrap_w(len(w0), _p(rp, i64p), _p(ci, i32p), _p(v, f64p), _p(w0, f64p), int(sweeps), _p(w, f64p))
    return w


def set_threads(n):
    """Threads of the oracle's row-parallel SpMV (bitwise the same results)."""
    lib().or_set_threads(int(n))


class descending_dots:
    """Context in which the oracle sums its dot products in descending index
    order (a second rounding order of the same algorithm; the default is
    ascending): the spread between the two orders is the size of the
    differences that rounding order alone makes in a given solve."""

    def __enter__(self):
        lib().or_set_dot_order(1)
        return self

    def __exit__(self, *exc):
        lib().or_set_dot_order(0)
        return False
