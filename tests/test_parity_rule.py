"""The rule the GPU parity tests use to compare FP64 iteration counts with the
oracle's: equal, or one apart only where the oracle's stopping residual lies
within 1e-6 (relative) of the tolerance, reported as a MarginalStop warning."""
import numpy as np
import pytest

from conftest import MarginalStop, stop_margin


def test_iteration_rule(iters_match):
    hist = np.array([1.0, 1e-3, 1e-6, 1.0000001e-8, 0.5e-8])
    ref = {"iters": 4, "hist": hist}
    assert iters_match(4, ref, 1e-8)
    assert not iters_match(2, ref, 1e-8) and not iters_match(6, ref, 1e-8)
    with pytest.warns(MarginalStop, match="oracle 4, gpu 3"):
        assert iters_match(3, ref, 1e-8)        # oracle's relres at 3 is 1e-8 (1 + 1e-7)
    assert not iters_match(5, ref, 1e-8)        # oracle's relres at 4 is 0.5e-8: not marginal
    ref2 = {"iters": 3, "hist": np.array([1.0, 1e-4, 3e-8, 0.9999999e-8])}
    with pytest.warns(MarginalStop):
        assert iters_match(4, ref2, 1e-8)       # gpu stopped one later at a marginal crossing
    assert not iters_match(2, ref2, 1e-8)       # relres 3e-8 at 2 is far from tol


def test_margin_is_one_in_a_million(iters_match):
    """A crossing 1e-5 away from tol is not marginal (the earlier rule's 1%
    window accepted it)."""
    ref = {"iters": 4, "hist": np.array([1.0, 1e-3, 1e-6, 1.00001e-8, 0.5e-8])}
    assert not iters_match(3, ref, 1e-8)
    assert stop_margin(ref, 1e-8) == pytest.approx(1e-5, rel=1e-6)


def test_no_long_run_allowance(iters_match):
    hist = np.linspace(1.0, 0.5e-8, 464)
    ref = {"iters": 463, "hist": hist}
    assert not iters_match(465, ref, 1e-8) and not iters_match(458, ref, 1e-8)
    assert not iters_match(464, ref, 1e-8)


def test_rounding_bar():
    """Iterates of long runs: 1e-10, or ORDER_FACTOR times the oracle's own
    ascending-versus-descending spread, whichever is larger."""
    from conftest import ORDER_FACTOR, within_rounding
    assert within_rounding(9e-11, 1e-14) and not within_rounding(2e-10, 1e-14)
    assert within_rounding(ORDER_FACTOR * 1e-7, 1e-7)
    assert not within_rounding(1.01 * ORDER_FACTOR * 1e-7, 1e-7)


def test_descending_dot_order(oracle):
    """The oracle's second dot order: the descending sum equals the ascending
    sum of the reversed vectors bit for bit, both lie within the sequential
    summation bound of the exactly rounded value, and the context restores the
    default order."""
    import math
    rng = np.random.default_rng(11)
    x, y = rng.standard_normal(10001), rng.standard_normal(10001)
    asc = oracle.dot(x, y)
    with oracle.descending_dots():
        desc = oracle.dot(x, y)
    assert desc == oracle.dot(x[::-1].copy(), y[::-1].copy())
    assert oracle.dot(x, y) == asc
    exact = math.fsum(float(a) * float(b) for a, b in zip(x, y))   # products rounded once, as in both sums
    bound = len(x) * np.finfo(float).eps * float(np.abs(x) @ np.abs(y))
    assert abs(asc - exact) <= bound and abs(desc - exact) <= bound
    assert asc != desc   # the two orders round differently for this draw


def test_order_spread_is_rounding_sized(oracle):
    """On a short all-Dirichlet solve the two dot orders move the iterate only
    at rounding level."""
    from conftest import order_spread
    from paper_2511_21268_amd.workloads import rhs_normal
    rp, ci, v, _ = oracle.poisson_kron(2, 2, 16)
    F = rhs_normal(len(rp) - 1, 1)
    h = oracle.Hierarchy(rp, ci, v)
    s = order_spread(h, F, 8)
    assert 0.0 < s < 1e-13
