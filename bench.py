"""Benchmark: PCG-AMG solve time to relative residual 1e-8 on one MI355X.

Workload (default): 3D Poisson on the unit cube, tensor B-splines of degree
p = 3, n = 128 elements per direction, homogeneous Dirichlet
(N = 129^3 = 2,146,689 unknowns, 707,347,971 stored entries), F ~ N(0,1) from
seed 0, FP64 CG preconditioned by the matching-based AMG V-cycle (two pairwise
matching sweeps per level, l1-Jacobi 1/1, dense Cholesky at <= 200 unknowns).

One step = one complete solve (r = F, u = 0 -> ||r|| <= 1e-8 ||F||) with F and
the hierarchy resident in HBM; set-up is done once, outside the timed region.
The level-0 sparse matrix-pass kernel is bracketed by HIP events on the
library's stream during the timed steps to give its achieved bandwidth.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PCG-AMG solve s to rel-res 1e-8 (plain FP64 vs FP32/learned); SpMV GB/s"
HBM_PEAK_GBS = 8000.0

# HBM bytes per level-0 k_sell launch (the dominant kernel of the FP64 solve)
# from the FETCH_SIZE / WRITE_SIZE counter runs, each scaled by what the counter
# reads for a plain copy of known size; not measured by this script: taken from
# TRAFFIC_SOURCE and reported only while the kernel source and its launch code
# (kernels.h, solver.hip) are the ones the counters were taken with (SHA-256 of
# the two files, concatenated), else null.
TRAFFIC_SOURCE = "profiles/k_sell_c4_fp64_pmc.md"
MEASURED_TRAFFIC = {
    # (workload, SHA-256 of kernels.h + solver.hip, x windows on): bytes per
    # launch, SpMV and residual launches of one solve
    ("c4", "9c40f6d0073b9ed475e3afc8f6f5e9f1c5137286a905a09e4dc79c308bb8d2ef", 1): 6629786832,
    ("c4", "9c40f6d0073b9ed475e3afc8f6f5e9f1c5137286a905a09e4dc79c308bb8d2ef", 0): 5936292790,
}


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.h", "solver.hip"):
        with open(os.path.join(ROOT, "paper_2511_21268_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stream_read_gbs(torch, amgmod, nbytes=4 << 30):
    """The streaming-read reference (amg_stream_read: 16-byte nontemporal loads,
    as the matrix passes) over a 4 GiB buffer of ones, best of five after one
    warm-up, timed with events on torch's current stream (the probe's stream);
    the per-thread sums are checked against the buffer's."""
    buf = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    sink = torch.empty(2048 * 256, dtype=torch.float64, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for rep in range(6):
        e0.record()
        amgmod.stream_read(buf, sink)
        e1.record()
        e1.synchronize()
        if rep:
            best = min(best, e0.elapsed_time(e1))
    assert float(sink.sum()) == nbytes // 8
    del buf, sink
    return nbytes / (best * 1e-3) / 1e9


def cpu_baseline(cfg, seed, tol, iters_gpu, u_gpu, one_core_iters):
    """The oracle (plain C, FP64) on this workload: its own assembly and
    hierarchy (untimed), then the whole solve timed on every host thread (its
    iteration count and solution set beside the GPU's), and a short sample on
    one core scaled to the full count."""
    import numpy as np

    import oracle
    from paper_2511_21268_amd.workloads import rhs_normal

    t = time.time()
    if cfg["kind"] == "cube":
        rp, ci, v, Fcube, _ = oracle.cube_system(cfg["p"], cfg["n"])
    else:
        rp, ci, v, _ = oracle.poisson_kron(cfg["d"], cfg["p"], cfg["n"], want_F=False)
    log(f"oracle: assembled K ({len(v)} entries) in {time.time() - t:.1f} s")
    t = time.time()
    oracle.set_verbose(1)
    h = oracle.Hierarchy(rp, ci, v)
    oracle.set_verbose(0)
    log(f"oracle: hierarchy of {h.nlevels} levels in {time.time() - t:.1f} s")
    F = Fcube if cfg["kind"] == "cube" else rhs_normal(len(rp) - 1, seed)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.set_threads(threads)
    t = time.time()
    res = h.solve(F, tol=tol)
    dt = time.time() - t
    err = float(np.linalg.norm(u_gpu - res["u"]) / np.linalg.norm(res["u"]))
    log(f"oracle: {res['iters']} PCG iterations in {dt:.1f} s on {threads} threads; GPU {iters_gpu} iterations, "
        f"||u_gpu - u_oracle|| / ||u_oracle|| = {err:.2e}")
    # one core: a bounded sample (bitwise the same iterates), scaled to the count
    oracle.set_threads(1)
    t = time.time()
    res1 = h.solve(F, tol=tol, itmax=one_core_iters)
    dt1 = time.time() - t
    oracle.set_threads(threads)
    log(f"oracle: {res1['iters']} PCG iterations in {dt1:.1f} s on 1 thread")
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(dt, 3), "unit": "s", "cores": threads, "kind": "oracle",
            "sample": f"the whole solve ({res['iters']} PCG iterations to rel-res {tol}) of the oracle on the same "
                      f"system, hierarchy built untimed; SpMV row-parallel over {threads} OpenMP threads",
            "parity": {"oracle_iters": res["iters"], "gpu_iters": iters_gpu, "rel_solution_diff": err},
            "one_core": {"value": round(dt1 / max(res1["iters"], 1) * res["iters"], 3), "unit": "s", "cores": 1,
                         "sample": f"{res1['iters']} iterations timed, scaled by {res['iters']} (extrapolated)"},
            "host": {"cpu": model, "logical_cpus": os.cpu_count()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--mode", default="fp64", choices=["fp64", "fp32", "batched", "blockcg", "learned", "learned32",
                                                       "paper", "cheb"],
                    help="fp64: FP64 PCG (default); fp32: FP32 V-cycle inside FP64 FCG; "
                         "batched: 16 right-hand sides, FP32 block V-cycle inside FP64 FCG; "
                         "blockcg: the same 16 right-hand sides by block flexible CG; "
                         "learned: FP64 PCG with the MLP-predicted degree-4 polynomial smoothers; "
                         "learned32: the same polynomials in the FP32 V-cycle inside FP64 FCG; "
                         "cheb: FP64 PCG with the fourth-kind Chebyshev l1-Jacobi smoother of --cheb-degree "
                         "(configuration hierarchy otherwise); "
                         "paper: FP64 FCG with the paper's default preconditioner (aggregates of 8, "
                         "smoothed prolongator, Chebyshev l1-Jacobi, CG coarse solve)")
    ap.add_argument("--cheb-degree", type=int, default=4)
    ap.add_argument("--params", default="", help="JSON object of further amg_params fields, merged into the form's")
    ap.add_argument("--learned", action="store_true",
                    help="use the trained degree-4 polynomial smoothers (sets smoother = 1) in any form")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--itmax", type=int, default=0, help="iteration limit (0: the workload's, else 1000)")
    ap.add_argument("--setup-device", action="store_true",
                    help="build the hierarchy (matching, Galerkin products) on the device")
    ap.add_argument("--graph", action="store_true",
                    help="replay each iteration's launches from HIP graphs in the timed steps (the per-launch "
                         "events that profiling records cannot be replayed, so the roofline then comes from one "
                         "further, eager, profiled solve after the timed steps)")
    ap.add_argument("--x-window", choices=["auto", "0", "1"], default="auto",
                    help="single-vector FP64 K passes through x windows (1) or gathers (0); auto: the set-up's "
                         "autotuner decides")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--one-core-iters", type=int, default=4,
                    help="iterations of the one-core oracle sample (scaled to the full count)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 2 GiB three times (to calibrate the "
                         "FETCH_SIZE / WRITE_SIZE counters against a known byte count)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding of this path "
              "(row slabs with halo exchange, all-reduced dots) is a design, not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        torch.cuda.set_device(0)
        nbytes = 2 << 30
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_dispatch": nbytes, "dispatches": 3}), flush=True)
        return

    import paper_2511_21268_amd as amg
    from paper_2511_21268_amd import amg as amgmod
    from paper_2511_21268_amd.workloads import CONFIGS, rhs_normal

    cfg = CONFIGS[args.workload]
    torch.cuda.set_device(0)
    t = time.time()
    if cfg["kind"] == "diffusion":
        from paper_2511_21268_amd.workloads import kappa_params
        rp, ci, v, Fload = amg.iga_diffusion(cfg["p"], cfg["n"], *kappa_params(args.seed))
    elif cfg["kind"] == "cube":
        rp, ci, v, Fload = amg.iga_cube(cfg["p"], cfg["n"])
    else:
        rp, ci, v, _ = amg.iga_poisson(cfg["d"], cfg["p"], cfg["n"], want_F=False)
        Fload = None
    N, nnz = len(rp) - 1, len(v)
    log(f"generated K: N={N} nnz={nnz} in {time.time() - t:.1f} s")
    nrhs = 16 if args.mode in ("batched", "blockcg") else 1
    if Fload is not None:
        F = torch.from_numpy(Fload).cuda()      # f = 1
    elif nrhs == 1:
        F = torch.from_numpy(rhs_normal(N, args.seed)).cuda()
    else:
        from paper_2511_21268_amd.workloads import rhs_block
        F = torch.from_numpy(rhs_block(N, range(args.seed, args.seed + nrhs))).cuda()
    torch.cuda.synchronize()
    t = time.time()
    kw = dict({"fp64": {}, "learned": {"smoother": 1}, "learned32": {"smoother": 1, "vcycle_fp32": 1, "krylov": 1},
               "paper": amg.paper_default(cfg["p"]),
               "blockcg": {"vcycle_fp32": 1, "krylov": 2},
               "cheb": {"smoother": 2, "cheb_degree": args.cheb_degree}}.get(
        args.mode, {"vcycle_fp32": 1, "krylov": 1}))
    kw["itmax"] = args.itmax or cfg.get("itmax", 1000)
    if nrhs > 1:
        kw["nrhs"] = nrhs
    if args.setup_device:
        kw["setup_device"] = 1
    if args.params:
        kw.update(json.loads(args.params))
    if args.learned:
        kw["smoother"] = 1
    ctx = amg.Context(rp, ci, v, **kw)
    if args.x_window != "auto":
        ctx.set_x_window(int(args.x_window))
    xwin = ctx.option(amgmod.AMG_OPT_X_WINDOW)
    if args.mode in ("learned", "learned32") or args.learned:
        from paper_2511_21268_amd import learned
        accepted, coefs = learned.apply_learned(ctx)
        log(f"learned smoothers: accepted {accepted}, coefficients {[list(map(lambda x: round(x, 3), c)) for c in coefs]}")
    torch.cuda.synchronize()
    setup_s = time.time() - t
    levels = [ctx.level_info(l) for l in range(ctx.nlevels)]
    fmt = ctx.format(0)
    log(f"setup {setup_s:.1f} s, levels {levels}, opc {ctx.opc():.3f}, format {fmt}")
    if nrhs > 1:
        log(f"block kernels (autotuned): lanes per row, threads = {ctx.batched_variant()}; window rows per lane "
            f"{ctx.option(amgmod.AMG_OPT_BLOCK_WINDOW)}, shared windows (mask: 1 FP64, 2 FP32) "
            f"{ctx.option(amgmod.AMG_OPT_WINDOW_SHARE)}")
    del rp, ci, v

    def one_solve():
        if nrhs == 1:
            u = torch.zeros_like(F)
            o = ctx.solve(F, u, tol=args.tol, check=False)
            return o, o["iters"]
        o = ctx.solve_batched(F, tol=args.tol)
        return o, max(o["iters"])

    for w in range(args.warmup):
        out, it = one_solve()
        log(f"warmup {w}: iters {out['iters']}")

    if args.graph:
        ctx.set_graph(True)
        one_solve()                    # captures the graphs outside the timed steps
    else:
        ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, marks = [], [t0]
    for s in range(args.steps):
        out, it = one_solve()          # returns once the solve has finished on the device
        iters.append(it)
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = sorted((b - a) * 1e3 for a, b in zip(marks[:-1], marks[1:]))
    if args.graph:
        ctx.set_graph(False)
        ctx.set_profiling(True)
        one_solve()
        torch.cuda.synchronize()
    prof = ctx.profile()
    ctx.set_profiling(False)
    ms = (t1 - t0) * 1e3 / args.steps
    converged = out["status"] == 0
    if not converged:
        log(f"status {out['status']}: not converged within itmax")
    if nrhs == 1:
        relres_true = out["relres_true"]
    else:
        # FP64 true residual of every column with the library's FP64 operator
        U = out["U"]
        relres_true = max(float(torch.linalg.norm(F[:, j] - ctx.spmv(U[:, j].contiguous())) /
                                torch.linalg.norm(F[:, j])) for j in range(nrhs))
    log(f"timed {args.steps} solves: {ms:.2f} ms per solve, iters {iters}, relres_true {relres_true:.3e}")
    assert not converged or relres_true <= args.tol * 1.0001, relres_true

    # the dominant kernel: the level-0 sparse matrix pass (SpMV with its dots,
    # residual, smoother sweep, polynomial step -- one kernel template); the
    # fused K P prolongation + post-smoothing pass and the others are listed
    # per kind.  achieved = algorithmic bytes per launch / average launch time,
    # both from the HIP events around every level-0 launch of the timed solves.
    dom = [k for k in ("spmv", "resid", "smooth", "poly") if k in prof["passes"]]
    dl = sum(prof["passes"][k]["launches"] for k in dom)
    dms = sum(prof["passes"][k]["ms"] for k in dom)
    dby = sum(prof["passes"][k]["bytes"] for k in dom)
    if args.mode in ("paper", "cheb") or not dom:
        dl, dms, dby = prof["launches"], prof["ms"], prof["bytes"]   # every level-0 pass
    kernel_ms = dms / max(dl, 1)
    achieved = dby / (dms * 1e-3) / 1e9 if dms > 0 else 0.0
    if nrhs > 1:
        kname = ("k_sellw_blk / k_sellws_blk (level-0 16-column SpMV / residual / smoother pass, staged x "
                 "windows, per wave / shared by a block)")
    elif args.mode in ("paper", "cheb"):
        kname = "k_sell_cheb + k_sell (level-0 Chebyshev / SpMV / residual passes)"
    else:
        kname = "k_sell (level-0 SpMV / residual / smoother pass)"
    traffic = MEASURED_TRAFFIC.get((args.workload, kernel_source_sha(), xwin)) if args.mode == "fp64" else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kname, "launches": dl, "avg_launch_ms": round(kernel_ms, 4),
                "bytes_per_launch": round(dby / max(dl, 1)),
                "traffic_source": TRAFFIC_SOURCE if traffic else None,
                "traffic_gbs": round(traffic / (kernel_ms * 1e-3) / 1e9, 1) if traffic and kernel_ms > 0 else None,
                "passes": {k: {"launches": d["launches"], "avg_ms": round(d["ms"] / max(d["launches"], 1), 4),
                               "gbs": round(d["bytes"] / (d["ms"] * 1e-3) / 1e9, 1) if d["ms"] > 0 else None,
                               "frac": round(d["bytes"] / (d["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                               if d["ms"] > 0 else None}
                           for k, d in prof["passes"].items()}}
    sgbs = stream_read_gbs(torch, amgmod)
    roofline["stream_read_gbs"] = round(sgbs, 1)
    roofline["frac_of_stream"] = round(achieved / sgbs, 4)
    log(f"level-0 passes: {json.dumps(roofline['passes'])}; streaming read {sgbs:.1f} GB/s")

    cpu = None
    if not args.no_cpu_baseline and args.mode == "fp64" and cfg["kind"] in ("poisson", "cube"):
        cpu = cpu_baseline(cfg, args.seed, args.tol, iters[-1], out["u"].cpu().numpy(), args.one_core_iters)

    form = {"fp64": "FP64 PCG", "fp32": "FP32 V-cycle in FP64 FCG",
            "batched": "16 RHS, FP32 block V-cycle in FP64 FCG",
            "blockcg": "16 RHS, FP32 block V-cycle in FP64 block flexible CG",
            "learned": "FP64 PCG, learned degree-4 polynomial smoothers", "paper": "FP64 FCG",
            "learned32": "FP32 V-cycle with learned degree-4 polynomial smoothers in FP64 FCG",
            "cheb": "FP64 PCG"}[args.mode]
    smoother = {"learned": "learned POLY4", "learned32": "learned POLY4", "cheb": f"fourth-kind Chebyshev l1-Jacobi degree {args.cheb_degree}"}.get(
        args.mode, "l1-Jacobi 1/1")
    amg_desc = f"m=2, {smoother}, Cholesky <= 200"
    if args.mode == "paper":
        amg_desc = (f"m=3 smoothed (omega 4/3), fourth-kind Chebyshev l1-Jacobi degree {kw['cheb_degree']}, "
                    f"CG-Jacobi coarse solve 1e-4 / 30 at <= 200")
    if cfg["kind"] == "diffusion":
        problem = "-div(kappa grad u) = 1, kappa from seed " + str(args.seed)
    elif cfg["kind"] == "cube":
        problem = "cube of Sec. 5.1 (u = exp(x+z) sin y, Dirichlet x=0,1 y=0, Neumann y=1 z=0,1)"
    else:
        problem = f"Poisson, F~N(0,1) seed {args.seed}{'..' + str(args.seed + nrhs - 1) if nrhs > 1 else ''}"
    rec = {"metric": METRIC, "value": round(ms / 1e3, 6), "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": False, "scaling": "strong",
           "vs_baseline": None, "dtype": "f64" if args.mode in ("fp64", "paper", "cheb", "learned") else "f32/f64",
           "data": "synthetic",
           "config": {"workload": f"{args.workload}: {cfg['d']}D {problem}, B-splines p={cfg['p']}, "
                                  f"n={cfg['n']}, N={N}, nnz={nnz}, {form} + "
                                  f"matching AMG V-cycle ({amg_desc}), tol {args.tol}",
                      "mode": args.mode, "params": kw, "nrhs": nrhs, "converged": converged,
                      "iters": iters[-1], "relres_true": relres_true, "levels": len(levels),
                      "ms_median": round(step_ms[len(step_ms) // 2], 3),
                      "opc": round(ctx.opc(), 4), "setup_s": round(setup_s, 2),
                      "setup_on_device": bool(args.setup_device),
                      "spmv_gbs": round(achieved, 1),
                      "x_window": xwin,
                      "block_variant": list(ctx.batched_variant()) if nrhs > 1 else None,
                      "block_window": ({"rows_per_lane": ctx.option(amgmod.AMG_OPT_BLOCK_WINDOW),
                                        "shared_mask": ctx.option(amgmod.AMG_OPT_WINDOW_SHARE)}
                                       if nrhs > 1 else None),
                      "graph_replay": bool(args.graph),
                      "roofline_from": "one eager profiled solve after the timed steps" if args.graph
                      else "the timed steps"},
           "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
