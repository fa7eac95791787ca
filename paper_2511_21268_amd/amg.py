"""ctypes binding of libamgiga.so (include/amg.h): argument marshalling only.

Every step of the solve runs in the library's HIP kernels; torch is used only
to hold device vectors and to name the stream.  Loading fails loudly when the
library has not been built (there is no fallback path).
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamgiga.so")

AMG_OK, AMG_NOT_CONVERGED = 0, 1
AMG_ERR_ARG, AMG_ERR_NOT_SPD, AMG_ERR_HIP, AMG_ERR_OOM, AMG_ERR_BREAKDOWN, AMG_ERR_STATE = -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "AMG_OK", 1: "AMG_NOT_CONVERGED", -1: "AMG_ERR_ARG", -2: "AMG_ERR_NOT_SPD",
                -3: "AMG_ERR_HIP", -4: "AMG_ERR_OOM", -5: "AMG_ERR_BREAKDOWN", -6: "AMG_ERR_STATE"}

EXPORTS = ["amg_params_default", "amg_setup", "pcg_solve", "pcg_solve_batched", "amg_vcycle", "amg_spmv",
           "amg_set_poly_coeffs",
           "amg_get_level_info", "amg_get_aggregates", "amg_get_coarse_matrix", "amg_setup_host", "amg_match",
           "amg_destroy", "amg_last_error", "amg_set_profiling", "amg_get_profile", "amg_get_format",
           "amg_iga_poisson_size", "amg_iga_poisson", "amg_iga_diffusion", "amg_level_features",
           "amg_mlp_forward", "amg_mlp_backward", "amg_mlp_adam", "amg_set_learned_poly",
           "amg_get_batched_variant", "amg_set_batched_variant", "amg_set_option", "amg_sell_spmv_host",
           "amg_iga_cube_size", "amg_iga_cube", "amg_get_prolongator", "amg_get_setup_rounds",
           "amg_mlp_backward_noalloc", "amg_get_option", "amg_get_profile_pass",
           "amg_get_residual_history", "amg_stream_read"]
AMG_OPT_GRAPH, AMG_OPT_FUSE_POST, AMG_OPT_BLOCK_WINDOW, AMG_OPT_TAIL, AMG_OPT_WINDOW_SHARE, AMG_OPT_X_WINDOW = 1, 2, 3, 4, 5, 6
MLP_NPARAM, MLP_NFEAT, MLP_NACT, MLP_NDEL = 4996, 8, 128, 132
MLP_NOALLOC_MAX_B = 16384
PASS_KINDS = ("spmv", "resid", "smooth", "poly", "kp", "other")   # amg_pass_kind order


class AmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("sweeps_per_level", C.c_int), ("max_coarse", C.c_int), ("max_levels", C.c_int),
                ("nu_pre", C.c_int), ("nu_post", C.c_int), ("vcycle_fp32", C.c_int), ("smoother", C.c_int),
                ("krylov", C.c_int), ("match_positive_only", C.c_int), ("itmax", C.c_int), ("nrhs", C.c_int),
                ("slice_offsets", C.c_int), ("smooth_prolong", C.c_int), ("cheb_degree", C.c_int),
                ("coarse_solver", C.c_int), ("coarse_itmax", C.c_int), ("omega", C.c_double),
                ("coarse_tol", C.c_double), ("setup_device", C.c_int), ("bootstrap_sweeps", C.c_int)]

# The paper's default preconditioner (Sec. 3.1 variants, Sec. 5.1): aggregates
# of 8, smoothed prolongator, Chebyshev-accelerated l1-Jacobi of degree
# 8 / 12 / 14 / 16 for p = 3..6, CG coarse solver, flexible CG outside.
CHEB_DEGREE = {3: 8, 4: 12, 5: 14, 6: 16}


def paper_default(p):
    """amg_params of the paper's default preconditioner for spline degree p."""
    return dict(sweeps_per_level=3, smooth_prolong=1, smoother=2, cheb_degree=CHEB_DEGREE.get(p, 8),
                coarse_solver=1, krylov=1)


i64p = C.POINTER(C.c_int64)
i32p = C.POINTER(C.c_int32)
f64p = C.POINTER(C.c_double)
_lib = None


def lib():
    """Load libamgiga.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} missing "
                               "(run __graft_entry__.build() or python paper_2511_21268_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.amg_params_default.argtypes = [C.POINTER(Params)]
        L.amg_setup.argtypes = [C.c_int64, i64p, i32p, f64p, f64p, C.POINTER(Params), vp, C.POINTER(vp)]
        L.amg_setup_host.argtypes = [C.c_int64, i64p, i32p, f64p, f64p, C.POINTER(Params), C.POINTER(vp)]
        L.amg_match.argtypes = [C.c_int64, i64p, i32p, f64p, f64p, C.c_int, i32p]
        L.pcg_solve.argtypes = [vp, vp, vp, C.c_double, C.POINTER(C.c_int), f64p, f64p]
        L.pcg_solve_batched.argtypes = [vp, C.c_int, vp, vp, C.c_double, C.POINTER(C.c_int), f64p]
        L.amg_set_poly_coeffs.argtypes = [vp, C.c_int, f64p]
        L.amg_vcycle.argtypes = [vp, vp, vp]
        L.amg_spmv.argtypes = [vp, C.c_int, vp, vp]
        L.amg_get_level_info.argtypes = [vp, C.c_int, i64p, i64p]
        L.amg_get_aggregates.argtypes = [vp, C.c_int, i32p, f64p]
        L.amg_get_coarse_matrix.argtypes = [vp, C.c_int, i64p, i32p, f64p]
        L.amg_get_prolongator.argtypes = [vp, C.c_int, i64p, i64p, i32p, f64p]
        L.amg_get_setup_rounds.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.amg_destroy.argtypes = [vp]
        L.amg_destroy.restype = None
        L.amg_last_error.restype = C.c_char_p
        L.amg_set_profiling.argtypes = [vp, C.c_int]
        L.amg_get_profile.argtypes = [vp, i64p, f64p, f64p]
        L.amg_get_profile_pass.argtypes = [vp, C.c_int, i64p, f64p, f64p]
        L.amg_get_residual_history.argtypes = [vp, f64p, C.c_int, C.POINTER(C.c_int)]
        L.amg_stream_read.argtypes = [vp, C.c_int64, vp, C.c_int64, vp]
        L.amg_get_format.argtypes = [vp, C.c_int, C.POINTER(C.c_int), i64p, C.POINTER(C.c_int), i64p]
        L.amg_iga_poisson_size.argtypes = [C.c_int, C.c_int, C.c_int, i64p, i64p]
        L.amg_iga_poisson.argtypes = [C.c_int, C.c_int, C.c_int, i64p, i32p, f64p, f64p]
        L.amg_iga_cube_size.argtypes = [C.c_int, C.c_int, i64p, i64p]
        L.amg_iga_cube.argtypes = [C.c_int, C.c_int, i64p, i32p, f64p, f64p]
        L.amg_iga_diffusion.argtypes = [C.c_int, C.c_int, C.c_int, f64p, i32p, i64p, i32p, f64p, f64p]
        L.amg_level_features.argtypes = [vp, C.c_int, C.POINTER(C.c_float)]
        L.amg_mlp_forward.argtypes = [vp, vp, C.c_int, vp, vp, vp]
        L.amg_mlp_backward.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp, vp, vp, vp]
        L.amg_mlp_backward_noalloc.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp, vp, vp]
        L.amg_mlp_adam.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.c_float, vp]
        L.amg_set_option.argtypes = [vp, C.c_int, C.c_int]
        L.amg_get_option.argtypes = [vp, C.c_int, C.POINTER(C.c_int)]
        L.amg_sell_spmv_host.argtypes = [C.c_int64, C.c_int64, i64p, i32p, f64p, C.c_int, C.c_int, f64p, f64p,
                                         i64p, i64p]
        L.amg_get_batched_variant.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.amg_set_batched_variant.argtypes = [vp, C.c_int, C.c_int]
        L.amg_set_learned_poly.argtypes = [vp, C.POINTER(C.c_uint16), C.POINTER(C.c_int), f64p]
        _lib = L
    return _lib


def _check(st, allow=(AMG_OK,)):
    if st not in allow:
        raise AmgError(st, lib().amg_last_error().decode())
    return st


def _p(a, t):
    return a.ctypes.data_as(t)


def params_default(**kw):
    prm = Params()
    lib().amg_params_default(C.byref(prm))
    for k, v in kw.items():
        if not hasattr(prm, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(prm, k, float(v) if k in ("omega", "coarse_tol") else int(v))
    return prm


def iga_poisson(d, p, n, want_F=True):
    """Host CSR (int64 indptr, int32 indices, f64 data) of the Dirichlet-reduced
    IgA Poisson stiffness matrix, and F for f = 1 (library's own generator)."""
    N = C.c_int64(); nz = C.c_int64()
    _check(lib().amg_iga_poisson_size(d, p, n, C.byref(N), C.byref(nz)))
    rp = np.empty(N.value + 1, np.int64); ci = np.empty(nz.value, np.int32); v = np.empty(nz.value)
    F = np.empty(N.value) if want_F else None
    _check(lib().amg_iga_poisson(d, p, n, _p(rp, i64p), _p(ci, i32p), _p(v, f64p),
                                 _p(F, f64p) if want_F else None))
    return rp, ci, v, F


def iga_cube(p, n, want_F=True):
    """Host CSR and load vector of the paper's cube problem (library's generator)."""
    N = C.c_int64(); nz = C.c_int64()
    _check(lib().amg_iga_cube_size(p, n, C.byref(N), C.byref(nz)))
    rp = np.empty(N.value + 1, np.int64); ci = np.empty(nz.value, np.int32); v = np.empty(nz.value)
    F = np.empty(N.value) if want_F else None
    _check(lib().amg_iga_cube(p, n, _p(rp, i64p), _p(ci, i32p), _p(v, f64p), _p(F, f64p) if want_F else None))
    return rp, ci, v, F


def iga_diffusion(p, n, a, mk, want_F=True):
    """Host CSR of -div(kappa grad u) with kappa(x) = exp(0.5 sum a_k cos(2 pi m_k.x))
    on the unit cube (library's sum-factorized assembly), and F for f = 1."""
    N = C.c_int64(); nz = C.c_int64()
    _check(lib().amg_iga_poisson_size(3, p, n, C.byref(N), C.byref(nz)))
    a_ = np.ascontiguousarray(a, np.float64); m_ = np.ascontiguousarray(mk, np.int32).reshape(-1)
    rp = np.empty(N.value + 1, np.int64); ci = np.empty(nz.value, np.int32); v = np.empty(nz.value)
    F = np.empty(N.value) if want_F else None
    _check(lib().amg_iga_diffusion(p, n, len(a_), _p(a_, f64p), _p(m_, i32p), _p(rp, i64p), _p(ci, i32p),
                                   _p(v, f64p), _p(F, f64p) if want_F else None))
    return rp, ci, v, F


def stream_read(buf, sink, stream=None):
    """One streaming read of the device tensor buf (amg_stream_read): thread t
    of the probe writes the sum of what it read to sink[t] (float64 device
    tensor).  Asynchronous on `stream` (torch's current stream by default)."""
    import torch
    assert buf.is_cuda and sink.is_cuda and sink.dtype == torch.float64 and buf.is_contiguous()
    st = (stream or torch.cuda.current_stream()).cuda_stream
    _check(lib().amg_stream_read(C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                                 C.c_void_p(sink.data_ptr()), sink.numel(), C.c_void_p(st)))


def sell_spmv_host(indptr, indices, data, x, C_slice=64, layout=1, ncols=None):
    """y = K x through the host image of the device layout (amg_sell_spmv_host);
    returns (y, shared_slices, stored)."""
    rp = np.ascontiguousarray(indptr, np.int64); ci = np.ascontiguousarray(indices, np.int32)
    v = np.ascontiguousarray(data, np.float64); xx = np.ascontiguousarray(x, np.float64)
    n = len(rp) - 1
    y = np.zeros(n)
    sh = C.c_int64(); st = C.c_int64()
    _check(lib().amg_sell_spmv_host(n, len(xx) if ncols is None else ncols, _p(rp, i64p), _p(ci, i32p), _p(v, f64p),
                                    C_slice, layout, _p(xx, f64p), _p(y, f64p), C.byref(sh), C.byref(st)))
    return y, sh.value, st.value


def match(indptr, indices, data, w=None, positive_only=False):
    rp = np.ascontiguousarray(indptr, np.int64); ci = np.ascontiguousarray(indices, np.int32)
    v = np.ascontiguousarray(data, np.float64)
    n = len(rp) - 1
    wv = None if w is None else np.ascontiguousarray(w, np.float64)
    mate = np.empty(n, np.int32)
    _check(lib().amg_match(n, _p(rp, i64p), _p(ci, i32p), _p(v, f64p), _p(wv, f64p) if wv is not None else None,
                           int(positive_only), _p(mate, i32p)))
    return mate


class Context:
    """An amg_ctx: the hierarchy on host and device, and the solve calls."""

    def __init__(self, indptr, indices, data, w=None, stream=None, host_only=False, **params):
        rp = np.ascontiguousarray(indptr, np.int64); ci = np.ascontiguousarray(indices, np.int32)
        v = np.ascontiguousarray(data, np.float64)
        self.n = len(rp) - 1
        self.prm = params_default(**params)
        wv = None if w is None else np.ascontiguousarray(w, np.float64)
        h = C.c_void_p()
        wp = _p(wv, f64p) if wv is not None else None
        if host_only:
            st = lib().amg_setup_host(self.n, _p(rp, i64p), _p(ci, i32p), _p(v, f64p), wp, C.byref(self.prm),
                                      C.byref(h))
        else:
            import torch
            if stream is None:
                stream = torch.cuda.current_stream()
            self.stream = stream
            st = lib().amg_setup(self.n, _p(rp, i64p), _p(ci, i32p), _p(v, f64p), wp, C.byref(self.prm),
                                 C.c_void_p(stream.cuda_stream), C.byref(h))
        _check(st)
        self.h = h
        self.host_only = host_only

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().amg_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- inspection --------------------------------------------------------
    @property
    def nlevels(self):
        n = C.c_int64(); nz = C.c_int64()
        _check(lib().amg_get_level_info(self.h, -1, C.byref(n), C.byref(nz)))
        return n.value

    def level_info(self, level):
        n = C.c_int64(); nz = C.c_int64()
        _check(lib().amg_get_level_info(self.h, level, C.byref(n), C.byref(nz)))
        return n.value, nz.value

    def opc(self):
        n = C.c_int64(); nz = C.c_int64()
        _check(lib().amg_get_level_info(self.h, -1, C.byref(n), C.byref(nz)))
        return nz.value / self.level_info(0)[1]

    def aggregates(self, level):
        n, _ = self.level_info(level)
        agg = np.empty(n, np.int32); pc = np.empty(n)
        _check(lib().amg_get_aggregates(self.h, level, _p(agg, i32p), _p(pc, f64p)))
        return agg, pc

    def coarse_matrix(self, level):
        n, nz = self.level_info(level)
        rp = np.empty(n + 1, np.int64); ci = np.empty(nz, np.int32); v = np.empty(nz)
        _check(lib().amg_get_coarse_matrix(self.h, level, _p(rp, i64p), _p(ci, i32p), _p(v, f64p)))
        return rp, ci, v

    def prolongator(self, level):
        """The smoothed prolongator of `level` as CSR (None when not built)."""
        nz = C.c_int64()
        _check(lib().amg_get_prolongator(self.h, level, C.byref(nz), None, None, None))
        if nz.value == 0:
            return None
        n, _ = self.level_info(level)
        rp = np.empty(n + 1, np.int64); ci = np.empty(nz.value, np.int32); v = np.empty(nz.value)
        _check(lib().amg_get_prolongator(self.h, level, C.byref(nz), _p(rp, i64p), _p(ci, i32p), _p(v, f64p)))
        return rp, ci, v

    def setup_rounds(self):
        """(matching sweeps, rounds summed, most rounds in a sweep) of a device set-up."""
        a = C.c_int(); b = C.c_int(); d = C.c_int()
        _check(lib().amg_get_setup_rounds(self.h, C.byref(a), C.byref(b), C.byref(d)))
        return a.value, b.value, d.value

    def format(self, level=0):
        sl = C.c_int(); stored = C.c_int64(); ib = C.c_int(); sh = C.c_int64()
        _check(lib().amg_get_format(self.h, level, C.byref(sl), C.byref(stored), C.byref(ib), C.byref(sh)))
        return dict(slice=sl.value, stored=stored.value, index_bytes=ib.value, shared_slices=sh.value)

    def set_poly(self, level, coeffs):
        c = np.ascontiguousarray(coeffs, np.float64)
        return _check(lib().amg_set_poly_coeffs(self.h, level, _p(c, f64p)), allow=(AMG_OK, AMG_NOT_CONVERGED))

    def set_graph(self, on):
        _check(lib().amg_set_option(self.h, AMG_OPT_GRAPH, int(on)))

    def set_fused_post(self, on):
        _check(lib().amg_set_option(self.h, AMG_OPT_FUSE_POST, int(on)))

    def set_tail(self, on):
        _check(lib().amg_set_option(self.h, AMG_OPT_TAIL, int(on)))

    def set_x_window(self, on):
        """Single-vector matrix passes of stencil images through LDS windows of x."""
        _check(lib().amg_set_option(self.h, AMG_OPT_X_WINDOW, int(on)))

    def set_window_share(self, mask):
        """Block windows shared by the four slices of a block (batched stencil
        passes): bit 0 in the passes over FP64 values, bit 1 over FP32 values."""
        _check(lib().amg_set_option(self.h, AMG_OPT_WINDOW_SHARE, int(mask)))

    def set_block_window(self, rows):
        """0: no staged x windows; 2 or 4: windows with that many rows per lane."""
        _check(lib().amg_set_option(self.h, AMG_OPT_BLOCK_WINDOW, int(rows)))

    def option(self, opt):
        v = C.c_int()
        _check(lib().amg_get_option(self.h, opt, C.byref(v)))
        return v.value

    def batched_variant(self):
        lpr = C.c_int(); thr = C.c_int()
        _check(lib().amg_get_batched_variant(self.h, C.byref(lpr), C.byref(thr)))
        return lpr.value, thr.value

    def set_batched_variant(self, lpr, threads=256):
        _check(lib().amg_set_batched_variant(self.h, int(lpr), int(threads)))

    def features(self, level):
        f = (C.c_float * 8)()
        _check(lib().amg_level_features(self.h, level, f))
        return np.array(list(f), dtype=np.float32)

    def set_learned_poly(self, w_bf16):
        """Predict and set every level's polynomial smoother from the MLP weights
        (numpy uint16 BF16 bits).  Returns (accepted flags, coefficients)."""
        w = np.ascontiguousarray(w_bf16, np.uint16)
        assert w.size == MLP_NPARAM
        nl = max(self.nlevels - 1, 0)
        acc = (C.c_int * max(nl, 1))(); coef = np.zeros((max(nl, 1), 4))
        _check(lib().amg_set_learned_poly(self.h, w.ctypes.data_as(C.POINTER(C.c_uint16)), acc,
                                          _p(coef, f64p)))
        return [bool(acc[i]) for i in range(nl)], coef[:nl]

    # ---- measurement ---------------------------------------------------------
    def set_profiling(self, on):
        _check(lib().amg_set_profiling(self.h, int(on)))

    def residual_history(self):
        """||r_k|| / ||F|| of the last solve, k = 0 .. iterations (numpy array)."""
        cnt = C.c_int()
        _check(lib().amg_get_residual_history(self.h, None, 0, C.byref(cnt)))
        h = np.zeros(cnt.value)
        if cnt.value:
            _check(lib().amg_get_residual_history(self.h, _p(h, f64p), cnt.value, C.byref(cnt)))
        return h

    def profile(self):
        n = C.c_int64(); ms = C.c_double(); by = C.c_double()
        _check(lib().amg_get_profile(self.h, C.byref(n), C.byref(ms), C.byref(by)))
        passes = {}
        for k, name in enumerate(PASS_KINDS):
            pn = C.c_int64(); pms = C.c_double(); pby = C.c_double()
            _check(lib().amg_get_profile_pass(self.h, k, C.byref(pn), C.byref(pms), C.byref(pby)))
            if pn.value:
                passes[name] = dict(launches=pn.value, ms=pms.value, bytes=pby.value)
        return dict(launches=n.value, ms=ms.value, bytes=by.value, passes=passes)

    # ---- operators ---------------------------------------------------------------
    def vcycle(self, r):
        import torch
        assert r.dtype == torch.float64 and r.is_cuda and r.is_contiguous() and r.numel() == self.n
        z = torch.empty_like(r)
        _check(lib().amg_vcycle(self.h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr())))
        return z

    def spmv(self, x, level=0):
        import torch
        n = self.level_info(level)[0]
        assert x.dtype == torch.float64 and x.is_cuda and x.is_contiguous() and x.numel() == n
        y = torch.empty_like(x)
        _check(lib().amg_spmv(self.h, level, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())))
        return y

    # ---- solve ------------------------------------------------------------------
    def solve(self, F, u=None, tol=1e-8, check=True):
        """F: float64 device tensor (n,).  u: device tensor, initial guess (zeros
        if None), overwritten with the solution.  Returns a dict."""
        import torch
        assert F.dtype == torch.float64 and F.is_cuda and F.is_contiguous() and F.numel() == self.n
        if u is None:
            u = torch.zeros_like(F)
        assert u.dtype == torch.float64 and u.is_cuda and u.is_contiguous() and u.numel() == self.n
        it = C.c_int(); rel = C.c_double(); relt = C.c_double()
        st = lib().pcg_solve(self.h, C.c_void_p(F.data_ptr()), C.c_void_p(u.data_ptr()), float(tol),
                             C.byref(it), C.byref(rel), C.byref(relt))
        if check:
            _check(st, allow=(AMG_OK, AMG_NOT_CONVERGED))
        return dict(status=st, u=u, iters=it.value, relres=rel.value, relres_true=relt.value)

    def solve_batched(self, F, U=None, tol=1e-8, check=True):
        """F: (n, k) float64 device tensor in column-major order (a transposed
        view of a contiguous (k, n) tensor), k <= 16."""
        import torch
        n, k = F.shape
        assert n == self.n and F.dtype == torch.float64 and F.is_cuda
        Ft = F.t().contiguous()          # (k, n) row-major == (n, k) column-major
        Ut = torch.zeros_like(Ft) if U is None else U.t().contiguous()
        its = (C.c_int * k)(); rel = np.empty(k)
        st = lib().pcg_solve_batched(self.h, k, C.c_void_p(Ft.data_ptr()), C.c_void_p(Ut.data_ptr()), float(tol),
                                     its, _p(rel, f64p))
        if check:
            _check(st, allow=(AMG_OK, AMG_NOT_CONVERGED))
        return dict(status=st, U=Ut.t(), iters=list(its), relres=rel)
