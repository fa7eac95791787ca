"""CPU: the test vector by relaxation on K w = 0 (Sec. 3.1) in the library's
host set-up equals the oracle's bit for bit, and so does the hierarchy built
on it; the device set-up option is refused without a device."""
import numpy as np
import pytest

import oracle
import paper_2511_21268_amd as amg
from paper_2511_21268_amd.workloads import random_start


@pytest.mark.parametrize("sweeps", [1, 4, 10])
@pytest.mark.parametrize("m", [1, 2, 3])
def test_bootstrap_hierarchy_bitwise(sweeps, m):
    rp, ci, v, _, _ = oracle.cube_system(3, 8)
    w0 = random_start(len(rp) - 1, 7)
    w = oracle.bootstrap_w(rp, ci, v, w0, sweeps)
    h = oracle.Hierarchy(rp, ci, v, w=w, sweeps_per_level=m)
    ctx = amg.Context(rp, ci, v, w=w0, host_only=True, bootstrap_sweeps=sweeps, sweeps_per_level=m)
    assert ctx.nlevels == h.nlevels >= 2
    for l in range(h.nlevels - 1):
        a, pc = ctx.aggregates(l)
        ao, pco, _, _ = h.level_agg(l)
        assert np.array_equal(a, ao) and np.array_equal(pc, pco)
        for x, y in zip(ctx.coarse_matrix(l + 1), h.level_matrix(l + 1)):
            assert np.array_equal(x, y)
    # the relaxed vector gives other aggregates than the plain ones
    ones = amg.Context(rp, ci, v, host_only=True, sweeps_per_level=m)
    assert not np.array_equal(ones.aggregates(0)[0], ctx.aggregates(0)[0])


def test_bootstrap_and_device_setup_arguments():
    rp, ci, v, _ = oracle.poisson_kron(2, 2, 24)
    with pytest.raises(amg.AmgError):
        amg.Context(rp, ci, v, host_only=True, bootstrap_sweeps=3)          # no random start
    with pytest.raises(amg.AmgError):
        amg.Context(rp, ci, v, host_only=True, setup_device=1)
    with pytest.raises(amg.AmgError):
        amg.Context(rp, ci, v, host_only=True, bootstrap_sweeps=1001, w=np.ones(len(rp) - 1))
    ctx = amg.Context(rp, ci, v, host_only=True)
    assert ctx.setup_rounds() == (0, 0, 0)
