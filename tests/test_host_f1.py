"""CPU: the library's host set-up of the paper's default preconditioner
(aggregates of 8, smoothed prolongator, Sec. 3.1 "Variants and efficiency")
equals the oracle's bit for bit: aggregates, prolongator and every Galerkin
matrix.  Built with amg_setup_host (no GPU)."""
import numpy as np
import pytest

import oracle
import paper_2511_21268_amd as amg


def _systems():
    rp, ci, v, _, _ = oracle.cube_system(3, 6)
    yield "cube p3 k6", (rp, ci, v)
    rp, ci, v, _ = oracle.poisson_kron(3, 2, 10)
    yield "poisson p2 n10", (rp, ci, v)
    rp, ci, v, _ = oracle.poisson_kron(2, 4, 24)
    yield "poisson 2D p4 n24", (rp, ci, v)


@pytest.mark.parametrize("name,sysm", list(_systems()))
@pytest.mark.parametrize("coarse,omega", [(0, 4.0 / 3.0), (1, 4.0 / 3.0), (0, 0.9)])
def test_host_f1_hierarchy_bitwise(name, sysm, coarse, omega):
    rp, ci, v = sysm
    prm = dict(sweeps_per_level=3, smooth_prolong=1, smoother=2, cheb_degree=8, coarse_solver=coarse,
               max_coarse=40, omega=omega)
    h = oracle.Hierarchy(rp, ci, v, **prm)
    ctx = amg.Context(rp, ci, v, host_only=True, krylov=1, **prm)
    assert ctx.nlevels == h.nlevels >= 2
    for l in range(h.nlevels - 1):
        a, pc = ctx.aggregates(l)
        ao, pco, _, _ = h.level_agg(l)
        assert np.array_equal(a, ao) and np.array_equal(pc, pco), (name, l)
        P = ctx.prolongator(l)
        Po = h.prolongator(l)
        for x, y in zip(P, Po):
            assert np.array_equal(x, y), (name, l)
        K = ctx.coarse_matrix(l + 1)
        Ko = h.level_matrix(l + 1)
        for x, y in zip(K, Ko):
            assert np.array_equal(x, y), (name, l + 1)
    assert abs(ctx.opc() - h.opc()) < 1e-12


def test_host_f1_param_checks():
    rp, ci, v, _ = oracle.poisson_kron(2, 2, 24)
    bad = [dict(smoother=2, vcycle_fp32=1), dict(smooth_prolong=1, nrhs=4), dict(smoother=2, nu_pre=2),
           dict(smoother=1, smooth_prolong=1), dict(cheb_degree=0), dict(cheb_degree=65), dict(omega=0.0),
           dict(omega=2.5), dict(coarse_tol=-1.0), dict(coarse_itmax=0), dict(coarse_solver=2), dict(smoother=3)]
    for kw in bad:
        with pytest.raises(amg.AmgError):
            amg.Context(rp, ci, v, host_only=True, **kw)
    ctx = amg.Context(rp, ci, v, host_only=True)
    assert ctx.prolongator(0) is None


def test_params_struct_matches_the_library():
    """The binding's amg_params mirrors the C struct: the library's defaults read
    back field by field (a shifted field would read garbage)."""
    p = amg.params_default()
    assert (p.sweeps_per_level, p.max_coarse, p.max_levels, p.nu_pre, p.nu_post) == (2, 200, 40, 1, 1)
    assert (p.vcycle_fp32, p.smoother, p.krylov, p.match_positive_only, p.itmax, p.nrhs) == (0, 0, 0, 0, 1000, 1)
    assert (p.slice_offsets, p.smooth_prolong, p.cheb_degree, p.coarse_solver, p.coarse_itmax) == (1, 0, 8, 0, 30)
    assert p.omega == 4.0 / 3.0 and p.coarse_tol == 1e-4
    assert (p.setup_device, p.bootstrap_sweeps) == (0, 0)
    q = amg.paper_default(5)
    assert q == dict(sweeps_per_level=3, smooth_prolong=1, smoother=2, cheb_degree=14, coarse_solver=1, krylov=1)
