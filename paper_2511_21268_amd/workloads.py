"""Seeded synthetic workloads shared by the library's callers and the tests.

Holds only sizes and random draws -- none of the method's arithmetic -- so that
the HIP path and the CPU oracle can be fed the same bits.  The stand-in for the
paper's GeoPDEs cube / L-shape / ring exports (Sec. 5) is the unit square or
cube with tensor-product B-splines of maximum regularity, homogeneous Dirichlet
on every face, lexicographic numbering with x fastest.
"""
import numpy as np

# name -> (d, p, n elements per direction, problem kind)
CONFIGS = {
    "c1": dict(d=2, p=2, n=32, kind="poisson"),     # N = 32^2   = 1,024
    "c2": dict(d=3, p=3, n=64, kind="poisson"),     # N = 65^3   = 274,625
    "c3": dict(d=3, p=4, n=96, kind="poisson"),     # N = 98^3   = 941,192
    "c4": dict(d=3, p=3, n=128, kind="poisson"),    # N = 129^3  = 2,146,689
    "c5": dict(d=3, p=5, n=64, kind="diffusion", itmax=6000),   # N = 67^3 = 300,763; plain l1: ~3000 iterations
    # the paper's cube benchmark (Sec. 5.1), its largest p = 3 case of Table 1(b)
    "cube": dict(d=3, p=3, n=96, kind="cube"),     # N = 95*96*97 = 941,094
}


def dofs(d, p, n):
    """Unknowns of the Dirichlet-reduced tensor space: (n + p - 2)^d."""
    return (n + p - 2) ** d


def rhs_normal(N, seed):
    """F ~ N(0, 1), float64, drawn in lexicographic order."""
    return np.random.default_rng(seed).standard_normal(N)


def rhs_block(N, seeds):
    """Column-major block of right-hand sides, one seed per column (N x k)."""
    return np.stack([rhs_normal(N, s) for s in seeds], axis=1)


def random_start(N, seed):
    """Random start of the test-vector relaxation: uniform on [0, 1), float64."""
    return np.random.default_rng(seed).random(N)


def kappa_params(seed, nterms=8):
    """Parameters of kappa(x) = exp(0.5 sum_k a_k cos(2 pi m_k . x)):
    a_k ~ N(0,1) then m_k in {0..3}^3, drawn in that order from one generator."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(nterms)
    m = rng.integers(0, 4, size=(nterms, 3)).astype(np.int32)
    return a, m
