"""The rule the GPU parity tests use to compare FP64 iteration counts with the
oracle's (equal, or one apart only where the oracle's stop was marginal)."""
import numpy as np


def test_iteration_rule(iters_match):
    hist = np.array([1.0, 1e-3, 1e-6, 1.00001e-8, 0.5e-8])
    ref = {"iters": 4, "hist": hist}
    assert iters_match(4, ref, 1e-8)
    assert not iters_match(2, ref, 1e-8) and not iters_match(6, ref, 1e-8)
    assert iters_match(3, ref, 1e-8)            # oracle's relres at 3 is 1e-8 (1 + 1e-5)
    assert not iters_match(5, ref, 1e-8)        # oracle's relres at 4 is 0.5e-8: not marginal
    ref2 = {"iters": 3, "hist": np.array([1.0, 1e-4, 3e-8, 0.99999e-8])}
    assert iters_match(4, ref2, 1e-8)           # gpu stopped one later at a marginal crossing
    assert not iters_match(2, ref2, 1e-8)       # relres 3e-8 at 2 is far from tol


def test_long_run_rule(iters_match):
    hist = np.linspace(1.0, 0.5e-8, 464)
    ref = {"iters": 463, "hist": hist}
    assert iters_match(465, ref, 1e-8) and iters_match(458, ref, 1e-8)
    assert not iters_match(469, ref, 1e-8)
    short = {"iters": 100, "hist": np.linspace(1.0, 0.5e-8, 101)}
    assert not iters_match(102, short, 1e-8)
