"""Learned degree-4 polynomial smoother: data generation, GPU training, use.

The network (8 level features -> 64 -> 64 -> 4, tanh) predicts, per AMG level,
the degree-4 polynomial of the smoother correction sum_k a_k (D^{-1}K)^k D^{-1} r
(polynomial acceleration of l1-Jacobi, paper Sec. 3.2), as the values of
g(t) = 1 - e(t) = sum_k a_k t^{k+1} at the Chebyshev-Lobatto nodes NODES of (0, 1]
(g(0) = 0); the library interpolates them into a_0..a_3.  In this basis an
output error moves e(t) by about twice its size, whereas errors in the monomial
coefficients (tens to hundreds) are amplified into e(1).  The library's
acceptance test (|e(t)| <= 1, e(t) < 1 on (0, 1]) decides per level, and a
rejected level falls back to l1-Jacobi, so convergence never rests on an
unchecked prediction.

Labels come from the method itself: for each training problem the smoother
family e_a(t) = T_4((1 + a - 2t)/(1 - a)) / T_4((1 + a)/(1 - a)) (the degree-4
Chebyshev polynomial of [a, 1] normalised to e(0) = 1, always accepted) is swept
over a grid of a, first on all levels together and then level by level, and
each choice is scored by the work of a full PCG solve: iterations x matrix
passes (sum over levels of stored entries x SpMVs per V-cycle).  The training
target of a level is the coefficient vector of its best a.

Training runs on the GPU with the library's own kernels (amg_mlp_forward,
amg_mlp_backward, amg_mlp_adam): BF16 weights, FP32 master copy, Adam.

CLI:  python -m paper_2511_21268_amd.learned generate --out DATA.npz
      python -m paper_2511_21268_amd.learned train --data DATA.npz --out WEIGHTS.npz
"""
import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

from . import amg
from .workloads import kappa_params

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "learned_poly4.npz")
NODES = 0.5 * (1.0 - np.cos(np.arange(1, 5) * np.pi / 4.0))
GRID = [0.5, 0.3, 0.15, 0.08, 0.04, 0.02, 0.01, 0.005]
# training problems: (p, n, kappa seed); seeds >= 100 are never used for evaluation
TRAIN = [(p, n, 100 + 10 * p + k) for p, ns in [(2, (16, 24, 40, 48)), (3, (16, 24, 32, 48)), (4, (12, 16, 24, 32)),
                                                 (5, (10, 14, 18, 24))] for k, n in enumerate(ns)]


def cheb_coeffs(a):
    """a_0..a_3 with 1 - e_a(t) = t (a_0 + a_1 t + a_2 t^2 + a_3 t^3)."""
    T4 = np.polynomial.Chebyshev([0, 0, 0, 0, 1])
    s = np.polynomial.Polynomial([(1 + a) / (1 - a), -2 / (1 - a)])
    e = (T4(s) / T4((1 + a) / (1 - a))).convert(kind=np.polynomial.Polynomial)
    c = (np.polynomial.Polynomial([1.0]) - e).coef
    c = np.concatenate([c, np.zeros(5 - len(c))])
    return c[1:5]


def node_values(coef):
    """g(t_j) = sum_k a_k t_j^{k+1} at NODES: the network's target for a_0..a_3."""
    return np.array([sum(coef[k] * t ** (k + 1) for k in range(4)) for t in NODES])


def load_weights(path=WEIGHTS):
    with np.load(path, allow_pickle=False) as z:
        return z["w_bf16"].astype(np.uint16)


def apply_learned(ctx, path=WEIGHTS):
    """Set every level of a context built with smoother=1 from the trained
    network; returns the per-level acceptance flags and coefficients."""
    return ctx.set_learned_poly(load_weights(path))


def problem(p, n, seed):
    a, mk = kappa_params(seed)
    rp, ci, v, F = amg.iga_diffusion(p, n, a, mk)
    return rp, ci, v, F


def _work(ctx, poly_levels):
    """Matrix passes of one PCG iteration weighted by stored entries."""
    w = ctx.level_info(0)[1]                      # outer SpMV
    for l in range(ctx.nlevels - 1):
        w += ctx.level_info(l)[1] * (8 if l in poly_levels else 2)
    return w


def _solve(ctx, F, tol, coefs):
    import torch
    for l, c in enumerate(coefs):
        if c is None:
            ctx.set_poly(l, [1.0, 0.0, 0.0, 0.0])
        else:
            assert ctx.set_poly(l, c) == 0
    out = ctx.solve(F, tol=tol, check=False)
    return out["iters"] if out["status"] == 0 else None


def label_problem(p, n, seed, tol=1e-6, itmax=400, log=print, setup_device=0):
    """Features and best-coefficient labels of every non-coarsest level (the
    hierarchy is the same bit for bit with the device set-up)."""
    import torch
    rp, ci, v, F = problem(p, n, seed)
    ctx = amg.Context(rp, ci, v, smoother=1, itmax=itmax, setup_device=setup_device)
    L = ctx.nlevels - 1
    Ft = torch.from_numpy(F).cuda()
    feats = np.stack([ctx.features(l) for l in range(L)])
    allp = set(range(L))
    base = _solve(ctx, Ft, tol, [None] * L)
    best = (None, float("inf"))
    for a in GRID:
        it = _solve(ctx, Ft, tol, [cheb_coeffs(a)] * L)
        if it is not None and it * _work(ctx, allp) < best[1]:
            best = (a, it * _work(ctx, allp))
    choice = [best[0]] * L
    for l in range(L):
        for a in GRID:
            trial = list(choice); trial[l] = a
            it = _solve(ctx, Ft, tol, [cheb_coeffs(x) for x in trial])
            if it is not None and it * _work(ctx, allp) < best[1]:
                best = (None, it * _work(ctx, allp)); choice = trial
    it_best = _solve(ctx, Ft, tol, [cheb_coeffs(x) for x in choice])
    log(f"p={p} n={n} seed={seed}: N={ctx.n} levels={L + 1} l1 iters={base} best a={choice} iters={it_best}")
    labels = np.stack([node_values(cheb_coeffs(a)) for a in choice])
    return feats, labels, dict(p=p, n=n, seed=seed, l1_iters=base, iters=it_best, a=choice)


def generate(out, log=print, setup_device=0):
    X, T, meta = [], [], []
    for (p, n, seed) in TRAIN:
        t = time.time()
        f, l, m = label_problem(p, n, seed, log=log, setup_device=setup_device)
        X.append(f); T.append(l); meta.append(m)
        log(f"  labelled in {time.time() - t:.1f} s")
    np.savez(out, X=np.concatenate(X).astype(np.float32), T=np.concatenate(T).astype(np.float32),
             meta=json.dumps(meta))


class Trainer:
    """Adam on the GPU through the library's MLP kernels (device buffers are
    torch tensors; the kernels are ordered on torch's current stream)."""

    def __init__(self, seed=0):
        import torch
        self.t = torch
        rng = np.random.default_rng(seed)
        master = np.zeros(amg.MLP_NPARAM, np.float32)
        # Glorot-uniform weights, zero biases
        offs = [(0, 64, 8), (512 + 64, 64, 64), (512 + 64 + 4096 + 64, 4, 64)]
        for off, fo, fi in offs:
            lim = np.sqrt(6.0 / (fi + fo))
            master[off:off + fo * fi] = rng.uniform(-lim, lim, fo * fi)
        dev = "cuda"
        self.master = torch.from_numpy(master).to(dev)
        self.w = torch.zeros(amg.MLP_NPARAM, dtype=torch.int16, device=dev)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.grad = torch.zeros_like(self.master)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.step_no = 0
        self._adam(0, 0.0)

    def _st(self):
        return C.c_void_p(self.t.cuda.current_stream().cuda_stream)

    def _adam(self, step, lr):
        amg._check(amg.lib().amg_mlp_adam(C.c_void_p(self.master.data_ptr()), C.c_void_p(self.w.data_ptr()),
                                          C.c_void_p(self.grad.data_ptr()), C.c_void_p(self.m.data_ptr()),
                                          C.c_void_p(self.v.data_ptr()), step, lr, self._st()))

    def forward(self, X, act=None):
        B = X.shape[0]
        Y = self.t.empty(B, 4, dtype=self.t.float32, device="cuda")
        amg._check(amg.lib().amg_mlp_forward(C.c_void_p(self.w.data_ptr()), C.c_void_p(X.data_ptr()), B,
                                             C.c_void_p(Y.data_ptr()),
                                             C.c_void_p(act.data_ptr()) if act is not None else None, self._st()))
        return Y

    def backward(self, X, act, Y, T):
        B = X.shape[0]
        dl = self.t.empty(B, amg.MLP_NDEL, dtype=self.t.float32, device="cuda")
        amg._check(amg.lib().amg_mlp_backward(C.c_void_p(self.w.data_ptr()), C.c_void_p(X.data_ptr()),
                                              C.c_void_p(act.data_ptr()), C.c_void_p(Y.data_ptr()),
                                              C.c_void_p(T.data_ptr()), B, C.c_void_p(dl.data_ptr()),
                                              C.c_void_p(self.grad.data_ptr()), C.c_void_p(self.loss.data_ptr()),
                                              self._st()))
        return float(self.loss.item())

    def step(self, X, T, lr):
        B = X.shape[0]
        act = self.t.empty(B, amg.MLP_NACT, dtype=self.t.float32, device="cuda")
        Y = self.forward(X, act)
        loss = self.backward(X, act, Y, T)
        self.step_no += 1
        self._adam(self.step_no, lr)
        return loss

    def weights_bf16(self):
        return self.w.cpu().numpy().view(np.uint16).copy()


def train(data, out, steps=3000, lr=3e-3, seed=0, log=print):
    import torch
    with np.load(data, allow_pickle=False) as z:
        X = torch.from_numpy(z["X"]).cuda()
        T = torch.from_numpy(z["T"]).cuda()
    tr = Trainer(seed)
    for s in range(steps):
        loss = tr.step(X, T, lr if s < steps * 2 // 3 else lr / 10)
        if s % 500 == 0 or s == steps - 1:
            log(f"step {s}: loss {loss:.5f}")
    np.savez(out, w_bf16=tr.weights_bf16(), nodes=NODES, steps=steps, lr=lr, seed=seed, loss=loss)
    return loss


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--out", required=True)
    g.add_argument("--setup-device", action="store_true", help="build the hierarchies on the device")
    t = sub.add_parser("train")
    t.add_argument("--data", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--steps", type=int, default=3000)
    args = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)  # noqa: E731
    if args.cmd == "generate":
        generate(args.out, log, setup_device=int(args.setup_device))
    else:
        train(args.data, args.out, steps=args.steps, log=log)


if __name__ == "__main__":
    sys.exit(main())
