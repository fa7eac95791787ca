"""GPU: the hierarchy set-up on the device (matching by rounds of locally
dominant edges, sort-based Galerkin product, relaxed test vector) equals the
oracle's hierarchy (Sec. 3.1: eqs. (cij), (maxprod), (prolongation),
(galerkin_matrix_projection)) bit for bit -- aggregates, prolongator
coefficients, test vectors and every coarse matrix -- and the host set-up's,
hence the same solve to the bit.  The 3D p=3 n=128 system is compared in
test_gpu_fullsize.py, which holds the oracle's hierarchy of it."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def amg():
    import paper_2511_21268_amd as m
    assert torch.cuda.is_available()
    m.lib()
    return m


def _system(oracle, name):
    """The oracle's systems (the library's generators give the same bits)."""
    from paper_2511_21268_amd.workloads import kappa_params
    if name == "cube p3 k12":
        return oracle.cube_system(3, 12)[:3]
    if name == "poisson 3D p3 n24":
        return oracle.poisson_kron(3, 3, 24, want_F=False)[:3]
    if name == "diffusion p3 n16":
        return oracle.diffusion_quad3d(3, 16, *kappa_params(3), factorized=True)[:3]
    if name == "poisson 2D p4 n64":
        return oracle.poisson_kron(2, 4, 64, want_F=False)[:3]
    raise KeyError(name)


def _same_hierarchy(a, b):
    assert a.nlevels == b.nlevels
    for l in range(a.nlevels - 1):
        x, y = a.aggregates(l), b.aggregates(l)
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]), l
        for p, q in zip(a.coarse_matrix(l + 1), b.coarse_matrix(l + 1)):
            assert np.array_equal(p, q), l + 1


def same_as_oracle(ctx, h, first_matrix=1):
    """Every level of the library context `ctx` against the oracle hierarchy
    `h`: sizes, aggregates, prolongator coefficients, and the coarse matrices
    from level `first_matrix` on, bit for bit."""
    assert ctx.nlevels == h.nlevels
    for l in range(h.nlevels):
        assert ctx.level_info(l) == h.level_info(l), l
    for l in range(h.nlevels - 1):
        a, pc = ctx.aggregates(l)
        ao, pco, _, _ = h.level_agg(l)
        assert np.array_equal(a, ao) and np.array_equal(pc, pco), l
        if l + 1 >= first_matrix:
            for x, y in zip(ctx.coarse_matrix(l + 1), h.level_matrix(l + 1)):
                assert np.array_equal(x, y), l + 1


CASES = [("cube p3 k12", dict(sweeps_per_level=2)), ("cube p3 k12", dict(sweeps_per_level=3)),
         ("poisson 3D p3 n24", dict(sweeps_per_level=2)), ("poisson 3D p3 n24", dict(sweeps_per_level=1)),
         ("diffusion p3 n16", dict(sweeps_per_level=2)), ("diffusion p3 n16", dict(match_positive_only=1)),
         ("poisson 2D p4 n64", dict(sweeps_per_level=3)),
         ("cube p3 k12", dict(bootstrap_sweeps=5)), ("diffusion p3 n16", dict(bootstrap_sweeps=3, sweeps_per_level=3))]


@pytest.mark.parametrize("ci_", range(len(CASES)))
def test_device_setup_bitwise(oracle, amg, ci_):
    from paper_2511_21268_amd.workloads import random_start
    name, prm = CASES[ci_]
    print(f"case {name} {prm}", flush=True)
    rp, ci, v = _system(oracle, name)
    w = random_start(len(rp) - 1, 11) if prm.get("bootstrap_sweeps") else None
    dev = amg.Context(rp, ci, v, w=w, setup_device=1, **prm)
    # against the oracle's hierarchy (relaxed test vector: the oracle's relaxation)
    oprm = {k: val for k, val in prm.items() if k != "bootstrap_sweeps"}
    wo = oracle.bootstrap_w(rp, ci, v, w, prm["bootstrap_sweeps"]) if w is not None else None
    same_as_oracle(dev, oracle.Hierarchy(rp, ci, v, w=wo, **oprm))
    # and the host set-up's
    host = amg.Context(rp, ci, v, w=w, host_only=True, **prm)
    _same_hierarchy(host, dev)
    sw, tot, mx = dev.setup_rounds()
    print(f"  levels {dev.nlevels}, matching sweeps {sw}, rounds {tot} (max {mx})", flush=True)
    assert sw >= 1 and 1 <= mx <= tot
    # same hierarchy, same kernels: the same solve to the bit
    ref = amg.Context(rp, ci, v, w=w, **prm)
    F = torch.from_numpy(np.random.default_rng(ci_).standard_normal(len(rp) - 1)).cuda()
    a, b = ref.solve(F, tol=1e-8), dev.solve(F, tol=1e-8)
    assert a["iters"] == b["iters"] and torch.equal(a["u"], b["u"])


@pytest.mark.timeout(600)
def test_device_setup_c2_against_oracle(oracle, amg):
    """3D p=3 n=64 (275k rows, 86.9M entries): device hierarchy = oracle's."""
    print("case device set-up c2: 3D p=3 n=64", flush=True)
    rp, ci, v, _ = oracle.poisson_kron(3, 3, 64, want_F=False)
    h = oracle.Hierarchy(rp, ci, v)
    dev = amg.Context(rp, ci, v, setup_device=1)
    same_as_oracle(dev, h)
    print(f"  levels {[h.level_info(l)[0] for l in range(h.nlevels)]}, rounds {dev.setup_rounds()}", flush=True)


def test_device_setup_rejects_nonsymmetric_pattern(oracle, amg):
    rp, ci, v = _system(oracle, "poisson 2D p4 n64")
    # drop one off-diagonal entry of row 0 (the matrix stays valid CSR)
    k = next(e for e in range(rp[0], rp[1]) if ci[e] != 0)
    keep = np.ones(len(ci), bool); keep[k] = False
    rp2 = rp.copy(); rp2[1:] -= 1
    with pytest.raises(amg.AmgError):
        amg.Context(rp2, ci[keep], v[keep], setup_device=1)


def test_device_setup_single_level_and_stall(amg):
    """A system at most max_coarse rows is one level (no matching at all); a
    two-level build with a larger coarse size still equals the host's."""
    rp, ci, v = amg.iga_poisson(2, 2, 10, want_F=False)[:3]        # 100 rows
    dev = amg.Context(rp, ci, v, setup_device=1)
    assert dev.nlevels == 1 and dev.setup_rounds() == (0, 0, 0)
    host = amg.Context(rp, ci, v, host_only=True, max_coarse=50)
    dev2 = amg.Context(rp, ci, v, setup_device=1, max_coarse=50)
    _same_hierarchy(host, dev2)
    F = torch.ones(len(rp) - 1, dtype=torch.float64, device="cuda")
    assert dev.solve(F, tol=1e-10)["iters"] == 1
