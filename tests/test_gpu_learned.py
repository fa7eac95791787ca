"""GPU: the learned polynomial smoother -- MLP forward/backward/Adam kernels
against the FP64 oracle and PyTorch references, the acceptance fallback, and
what the trained network gains over the method without it."""
import ctypes as C
import os
import time

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


def _bf16_bits(t):
    return t.cpu().numpy().view(np.uint16).copy()


def test_mlp_kernels_against_oracle(oracle, amg):
    print("case mlp fwd/bwd", flush=True)
    from paper_2511_21268_amd.learned import Trainer
    tr = Trainer(seed=3)
    rng = np.random.default_rng(4)
    B = 37
    X = torch.from_numpy(rng.standard_normal((B, 8)).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.standard_normal((B, 4)).astype(np.float32)).cuda()
    act = torch.empty(B, 128, dtype=torch.float32, device="cuda")
    Y = tr.forward(X, act)
    loss = tr.backward(X, act, Y, T)
    torch.cuda.synchronize()
    w = tr.weights_bf16()
    Yo = oracle.mlp_forward(w, X.cpu().numpy().astype(np.float64))
    assert np.abs(Y.cpu().numpy() - Yo).max() <= 1e-5 * max(1.0, np.abs(Yo).max())
    lo, go = oracle.mlp_loss_grad(w, X.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64))
    g = tr.grad.cpu().numpy().astype(np.float64)
    assert abs(loss - lo) <= 1e-5 * lo
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
    big = np.abs(go) > 1e-3 * np.abs(go).max()
    assert np.all(np.abs(g[big] - go[big]) <= 1e-4 * np.abs(go[big]) + 1e-6 * np.abs(go).max())


def test_adam_and_bf16_rounding(amg):
    print("case adam", flush=True)
    from paper_2511_21268_amd.learned import Trainer
    tr = Trainer(seed=5)
    master0 = tr.master.clone()
    # BF16 copy is the round-to-nearest-even of the master weights
    ref = master0.cpu().to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(tr.weights_bf16(), ref)
    g = torch.from_numpy(np.random.default_rng(6).standard_normal(master0.numel()).astype(np.float32))
    tr.grad.copy_(g.cuda())
    p = torch.nn.Parameter(master0.cpu().clone())
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in (1, 2):
        p.grad = g.clone()
        opt.step()
        tr._adam(step, 1e-2)
    torch.cuda.synchronize()
    assert torch.allclose(tr.master.cpu(), p.detach(), rtol=1e-5, atol=1e-6)


def test_training_reduces_loss(amg):
    print("case train", flush=True)
    from paper_2511_21268_amd.learned import Trainer
    rng = np.random.default_rng(7)
    X = torch.from_numpy(rng.uniform(-1, 1, (64, 8)).astype(np.float32)).cuda()
    T = torch.sin(X[:, :4] * 2.0).contiguous()
    tr = Trainer(seed=1)
    first = tr.step(X, T, 1e-2)
    for _ in range(300):
        last = tr.step(X, T, 1e-2)
    assert last < 0.2 * first


def test_rejected_prediction_falls_back_to_l1(oracle, amg):
    print("case fallback", flush=True)
    rp, ci, v, F = oracle.poisson_kron(3, 3, 14)
    ctx = amg.Context(rp, ci, v, smoother=1)
    w = np.zeros(4996, np.float32)
    w[-4:] = 3.0                             # g = 3 at every node: e(1) = -2, rejected
    bits = torch.from_numpy(w).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    acc, coef = ctx.set_learned_poly(bits)
    assert not any(acc)
    assert abs(1.0 - coef[0].sum() - (-2.0)) < 1e-9      # e(1) = 1 - sum a_k
    plain = amg.Context(rp, ci, v)
    r = torch.from_numpy(np.random.default_rng(0).standard_normal(len(F))).cuda()
    assert torch.equal(ctx.vcycle(r), plain.vcycle(r))


def test_learned_smoother_gain(oracle, amg):
    """Held-out kappa seeds (never used in training): the work to solution
    with the trained network against l1-Jacobi (the method without it) on
    variable-coefficient problems of degree 3 and 5.  Work = the algorithmic
    bytes of every level-0 matrix pass of the solve (the library's count over
    its launches: iterations times passes per iteration times bytes per pass),
    which does not depend on timing; wall-clock times are printed beside it."""
    from paper_2511_21268_amd import learned
    if not os.path.exists(learned.WEIGHTS):
        pytest.skip("trained weights not present")
    gains, tgains = [], []
    for (p, n, seed) in [(3, 24, 0), (3, 24, 1), (5, 14, 2), (5, 18, 3)]:
        print(f"case gain p={p} n={n} seed={seed}", flush=True)
        rp, ci, v, F = learned.problem(p, n, seed)
        Ft = torch.from_numpy(F).cuda()
        res = {}
        for name in ("l1", "learned"):
            ctx = amg.Context(rp, ci, v, smoother=1 if name == "learned" else 0, itmax=2000)
            if name == "learned":
                acc, coef = learned.apply_learned(ctx)
            ctx.solve(Ft, tol=1e-8, check=False)       # warm-up
            ctx.set_profiling(True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = ctx.solve(Ft, tol=1e-8, check=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            prof = ctx.profile()
            ctx.set_profiling(False)
            res[name] = dict(status=out["status"], iters=out["iters"], s=dt, relres=out["relres_true"],
                             passes=prof["launches"], gbytes=prof["bytes"] / 1e9)
        print(f"  l1 {res['l1']}  learned {res['learned']}  accepted {acc}", flush=True)
        assert res["learned"]["status"] == 0 and res["learned"]["relres"] <= 1e-8
        assert res["learned"]["iters"] < res["l1"]["iters"]
        gains.append(res["l1"]["gbytes"] / res["learned"]["gbytes"])
        tgains.append(res["l1"]["s"] / res["learned"]["s"])
    print("work gains", gains, "time gains", tgains)
    assert min(gains) > 1.0


def test_learned_smoother_in_fp32_vcycle(oracle, amg):
    """The learned polynomials inside the FP32 V-cycle (FP64 FCG outside): the
    same accepted levels, an FP64 true residual under 1e-8, and an iteration
    count within 2% of the FP64 learned form."""
    from paper_2511_21268_amd import learned
    if not os.path.exists(learned.WEIGHTS):
        pytest.skip("trained weights not present")
    rp, ci, v, F = learned.problem(5, 18, 3)
    print("case learned fp32 p=5 n=18 seed=3", flush=True)
    Ft = torch.from_numpy(F).cuda()
    out = {}
    for name, kw in (("fp64", dict(smoother=1)), ("fp32", dict(smoother=1, vcycle_fp32=1, krylov=1))):
        ctx = amg.Context(rp, ci, v, itmax=2000, **kw)
        acc, _ = learned.apply_learned(ctx)
        o = ctx.solve(Ft, tol=1e-8)
        u = o["u"].cpu().numpy()
        true = np.linalg.norm(F - oracle.spmv(rp, ci, v, u)) / np.linalg.norm(F)
        out[name] = (list(acc), o["iters"], true)
    print(f"  {out}", flush=True)
    assert out["fp32"][0] == out["fp64"][0]
    assert out["fp32"][2] <= 1e-8 * 1.0001
    assert abs(out["fp32"][1] - out["fp64"][1]) <= max(2, 0.02 * out["fp64"][1])
