"""Time-to-steady-state benchmark of the quantum-PageRank solver on one MI355X.

Workload (one "step" = one pass of the whole path over the batch): the
scale-free directed graph N=922 (Barabasi-Albert m=3, random edge direction,
10 % reciprocal, seed 0), Google damping 0.85, built on the GPU, then solved
to ||L(rho)||_F < 1e-8 from rho0 = I/N with RK4 dt = 0.01 in FP64 at each of
omega = 0.2, 0.5, 0.8, and ranked; the three solves run concurrently, one
stream each (qpr_steady_state_many; each is bitwise the single-system solve,
and the sequential time is reported beside it).  `value` is the throughput in
solves per second over the timed steps (inputs resident in HBM; host readback
of the device flag once per chunk is part of it); the mean time-to-steady-state
per solve is `extra.seconds_per_solve_fp64`.

Also reported (same graph, same omegas): the paper's adaptive RKF45
integrator, the accelerated solver (RKF45 from the learned, omega-blended
warm start) with its ranking checked against the plain solve, the
batched mixed warm-start form (qpr_batch_solve, FP32 steps with the defect held in FP32 and
the FP64 fold and judge, from the warm start), the dense FP64 MFMA solve, the
mixed-precision solves (BF16x3 and FP32 products with FP64 judge); the same
comparison at N = 4096 (BA m=4, omega = 0.8) and the plain solve at N = 2048;
hub classes and degeneracy of PageRank against the quantum steady state at
each size; the 1,280-system batching workload (--batch-family); the roofline of the
dominant kernel of the timed path (timed alone with HIP events on the stream
the kernel runs on, on the hot-path scope's bytes per element, with the
aggregate rate of the whole timed region beside it); and the CPU oracle on a
bounded sample of the workload (host CPU model, core count and BLAS stated).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-mixed]
                    [--no-dense] [--no-rkf45] [--no-4096] [--warm PATH|none]
                    [--batch-family off|subset|full]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-steady-state N=922/4096: FP64 plain vs mixed+warm-start; solves/s"
OMEGAS = (0.2, 0.5, 0.8)
N, M_BA, DT, TOL = 922, 3, 0.01, 1e-8
WEIGHTS = os.path.join(ROOT, "paper_2003_04930_amd", "weights", "mpnn_warmstart.npy")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0
# HBM bytes per launch at this workload from rocprofv3 FETCH_SIZE (x2.00) and
# WRITE_SIZE (x1.00) passes, the factors calibrated on a 256 MiB copy; valid
# for the stage kernels in the source with this sha256 prefix only (the
# summary with the commands: profiles/rk4_stage_kernels_n922_n4096.md)
COUNTERS_SRC = ("paper_2003_04930_amd/csrc/qpr_step.hip", "31d682585f3db40f")
TRAFFIC_N922 = {"epilogue": (16488.1 * 2.0 + 19992.7) * 1024.0,
                "spmm": (7352.4 * 2.0 + 13830.0) * 1024.0,
                "fused": (21995.3 * 2.0 + 19990.1) * 1024.0}


def measured_traffic(kernel):
    """Counter traffic of a stage kernel, or None once its source changed."""
    import hashlib
    with open(os.path.join(ROOT, COUNTERS_SRC[0]), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    if not digest.startswith(COUNTERS_SRC[1]):
        return None
    return TRAFFIC_N922.get(kernel)


def _json_default(o):
    """numpy scalars in the extra rows"""
    import numpy as np
    if isinstance(o, np.integer):
        return int(o)
    if isinstance(o, np.floating):
        return float(o)
    if isinstance(o, np.bool_):
        return bool(o)
    raise TypeError(f"not JSON serialisable: {type(o).__name__}")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def solve_all(Q, P, prec, rho0_fn=None, product="auto", integrator="rk4"):
    """The three omegas solved concurrently (qpr_steady_state_many: one stream
    and host thread per omega, each bitwise the single-system solve)."""
    rho0s = None if rho0_fn is None else [rho0_fn(w) for w in OMEGAS]
    return Q.steady_state_many([(P, w) for w in OMEGAS], DT, TOL, 400000, prec=prec,
                               rho0s=rho0s, product=product, integrator=integrator)


def solve_sequential(Q, P):
    return [Q.steady_state(P, w, DT, TOL, 400000) for w in OMEGAS]


def host_cpu():
    """Host description for the CPU baseline: logical CPUs, model name, BLAS."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:  # pragma: no cover
        pass
    blas, threads = "unknown", 1
    try:
        from threadpoolctl import threadpool_info
        info = [d for d in threadpool_info() if d.get("user_api") == "blas"]
        if info:
            blas = f"{info[0].get('internal_api')} {info[0].get('version')}"
            threads = max(int(d.get("num_threads", 1)) for d in info)
    except Exception:  # pragma: no cover
        pass
    return {"cpu_count": os.cpu_count(), "cpu_model": model, "blas": blas,
            "blas_threads": threads,
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
            else None}


def cpu_baseline(g, gpu_steps, budget_s=20.0):
    """The oracle's RK4 steps on the host's cores, the three omegas in turn,
    until about `budget_s` seconds of CPU work (at most 120 steps per omega),
    extrapolated to the GPU's mean step count per solve."""
    import numpy as np
    import oracle as O
    host = host_cpu()
    R = O.problem_ref(g.n, g.src, g.dst)
    rho0 = np.eye(g.n, dtype=np.complex128) / g.n
    states = {w: rho0.copy() for w in OMEGAS}
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and done < 120 * len(OMEGAS):
        w = OMEGAS[done % len(OMEGAS)]
        states[w] = O.rk4_step_ref(states[w], lambda r: O.rhs_ref(r, R.H_sparse, R.G, R.d, w), DT)
        done += 1
    dt = time.perf_counter() - t0
    per_step = dt / done
    per_solve = per_step * float(np.mean(gpu_steps))
    return {
        "value": 1.0 / per_solve, "unit": "solves/s", "cores": int(host["blas_threads"]),
        "kind": "oracle", "seconds_per_solve": per_solve, "host": host,
        "sample": (f"{done} RK4 steps ({dt:.1f} s) of the numpy/scipy FP64 oracle at N={g.n}, "
                   f"the omegas {list(OMEGAS)} in turn from I/N, {per_step * 1e3:.1f} ms/step, "
                   f"extrapolated to the GPU's mean step count {float(np.mean(gpu_steps)):.0f} "
                   f"per solve; cores = the BLAS threads (the sparse products run on one)"),
    }


def tie_aware_rank_check(p_ref, rank, tau, np):
    """Adjacent pairs of the reference order whose gap exceeds tau but whose
    order the tested ranking swaps (0 = the rankings agree up to ties)."""
    n = len(p_ref)
    pos = np.empty(n, dtype=np.int64)
    pos[rank] = np.arange(n)
    order = np.argsort(-p_ref, kind="stable")
    bad = 0
    for i in range(n - 1):
        a, b = order[i], order[i + 1]
        if p_ref[a] - p_ref[b] > tau and pos[a] > pos[b]:
            bad += 1
    return bad


def accelerated(Q, W, P, params, plain, plain_value, torch, np):
    """RKF45 from the omega-blended learned warm start (inference included)."""
    for w in OMEGAS:  # untimed: first use of the network path (allocations)
        W.warm_rho0(P, w, params, integrator="rkf45")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = solve_all(Q, P, "fp64", rho0_fn=lambda w: W.warm_rho0(P, w, params, integrator="rkf45"),
                    integrator="rkf45")
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / len(OMEGAS)
    err = max(float((a.rho - b.rho).abs().max()) for a, b in zip(out, plain))
    exact = all(bool(torch.equal(a.rank, b.rank)) for a, b in zip(out, plain))
    viol = 0
    for a, b in zip(out, plain):
        p_ref = b.rho[0].diagonal().cpu().numpy()
        viol += tie_aware_rank_check(p_ref, a.rank.cpu().numpy(), 2 * err, np)
    row = {"seconds_per_solve": t, "speedup_vs_plain_fp64": plain_value / t,
           "accepted_steps": [r.stats["steps"] for r in out],
           "blend_weights": [W.blend_weight(w, "rkf45") for w in OMEGAS],
           "max_abs_drho_vs_plain": err, "ranking_identical": exact,
           "order_violations_beyond_2maxdrho": viol,
           "residuals": [r.stats["residual"] for r in out]}
    log(f"accelerated (RKF45 + warm start): {t:.3f} s/solve ({plain_value / t:.1f}x), "
        f"max|drho| {err:.1e}, ranking identical {exact}")
    return row


def target_rows(Q, W, P, params, plain, plain_value, torch, np):
    """The three omegas of the workload solved together by qpr_batch_solve from
    the warm start: FP32 mixed precision (sparse FP32 products, FP64 folds and
    judge) with RK4, and FP64 RKF45; then the mixed solve as three concurrent
    single-system solves.  Inference is inside the timed region."""
    items = [(P, w) for w in OMEGAS]
    out = {}
    for name, kw in (("batch_mixed_fp32_warm", dict(prec="fp32")),
                     ("batch_rkf45_warm", dict(prec="fp64", integrator="rkf45"))):
        integ = kw.get("integrator", "rk4")
        W.warm_rho0_batch(items, params, integrator=integ)  # untimed first use of the network
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho0s = W.warm_rho0_batch(items, params, integrator=integ)
        rb = Q.batch_solve(items, tol=TOL, want_rank=True, rho0s=rho0s, **kw)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / len(OMEGAS)
        err = max(float((a - b.rho).abs().max()) for a, b in zip(rb.rhos, plain))
        exact = all(bool(torch.equal(a, b.rank)) for a, b in zip(rb.ranks, plain))
        viol = sum(tie_aware_rank_check(b.rho[0].diagonal().cpu().numpy(), a.cpu().numpy(),
                                        2 * err, np) for a, b in zip(rb.ranks, plain))
        out[name] = {"seconds_per_solve": t, "speedup_vs_plain_fp64": plain_value / t,
                     "steps": [x["steps"] for x in rb.stats],
                     "residuals": [x["residual"] for x in rb.stats],
                     "max_abs_drho_vs_plain": err, "ranking_identical": exact,
                     "order_violations_beyond_2maxdrho": viol}
        log(f"{name}: {t:.3f} s/solve ({plain_value / t:.1f}x), max|drho| {err:.1e}, "
            f"ranking identical {exact}")
    # the same mixed-precision solve from the warm start with the three omegas
    # on three streams (single-system kernels, run concurrently)
    t0 = time.perf_counter()
    rm = solve_all(Q, P, "fp32", rho0_fn=lambda w: W.warm_rho0(P, w, params))
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / len(OMEGAS)
    err = max(float((a.rho - b.rho).abs().max()) for a, b in zip(rm, plain))
    exact = all(bool(torch.equal(a.rank, b.rank)) for a, b in zip(rm, plain))
    viol = sum(tie_aware_rank_check(b.rho[0].diagonal().cpu().numpy(), a.rank.cpu().numpy(),
                                    2 * err, np) for a, b in zip(rm, plain))
    out["concurrent_mixed_fp32_warm"] = {
        "seconds_per_solve": t, "speedup_vs_plain_fp64": plain_value / t,
        "steps": [r.stats["steps"] for r in rm], "folds": [r.stats["folds"] for r in rm],
        "residuals": [r.stats["residual"] for r in rm], "max_abs_drho_vs_plain": err,
        "ranking_identical": exact, "order_violations_beyond_2maxdrho": viol}
    log(f"concurrent_mixed_fp32_warm: {t:.3f} s/solve ({plain_value / t:.1f}x), "
        f"max|drho| {err:.1e}, ranking identical {exact}")
    return out


def n4096_rows(Q, inputs, params, torch, np, args):
    """BA graph N = 4096 (m = 4) at omega = 0.8: plain FP64 RK4 against RKF45,
    the accelerated solve and (unless --no-mixed) the FP32 mixed solve, cold
    and from the warm start."""
    n, w = 4096, 0.8
    Pn = Q.Problem.from_graph(inputs.ba_digraph(n, 4, seed=0))
    torch.cuda.synchronize()
    plain = Q.steady_state(Pn, w, DT, TOL, 400000)
    torch.cuda.synchronize()
    row = {"omega": w, "plain_fp64": {"seconds": plain.stats["seconds"],
                                      "rk4_steps": plain.stats["steps"]}}
    log(f"n=4096 plain fp64: {plain.stats['seconds']:.2f} s, {plain.stats['steps']} steps")
    sp_ms, epi_ms = Q.time_kernels(Pn, w, plain.rho, prec="fp64", cfg=-2, reps=20)
    nvar = len(Q.SPARSE_VARIANTS)
    _, fused_ms = Q.time_kernels(Pn, w, plain.rho, prec="fp64", cfg=-3 - nvar, reps=20)
    # the stage of the mixed solve with the defect held in FP32 (the dominant
    # kernel of the mixed and batched warm-start solves at this size): its own
    # algorithmic bytes are half the FP64 stage's 80 B per element, 40 B (the
    # stage state read 8, y_n 8, the accumulator read and written 8 + 8, the
    # output 8: two FP32 planes each, counted as the FP64 figure counts them),
    # and it does the FP64 stage's work
    _, f32s_ms = Q.time_kernels(Pn, w, plain.rho, prec="fp32", cfg=-3 - (nvar + 2), reps=20)
    # at this size the solves take the fused epilogue (the sparse gathers inside
    # the stage kernel, no X round trip); the two-kernel stage is timed beside it
    row["stage_us"] = {"fused_epilogue": fused_ms * 1e3, "spmm": sp_ms * 1e3,
                       "epilogue": epi_ms * 1e3,
                       "fused_GBs": 80.0 * n * n / (fused_ms * 1e-3) / 1e9,
                       "fused_frac": 80.0 * n * n / (fused_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "fused_frac_unique_bytes": 50.0 * n * n / (fused_ms * 1e-3) / 1e9 /
                       HBM_PEAK_GBS,
                       "spmm_GBs": 32.0 * n * n / (sp_ms * 1e-3) / 1e9,
                       "epilogue_GBs": 96.0 * n * n / (epi_ms * 1e-3) / 1e9,
                       "fp32_state_stage": f32s_ms * 1e3,
                       "fp32_state_frac": 40.0 * n * n / (f32s_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "fp32_state_frac_fp64_bytes":
                           80.0 * n * n / (f32s_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    runs = {}
    if not args.no_rkf45:
        runs["fp64_rkf45"] = lambda: Q.steady_state(Pn, w, DT, TOL, 400000, integrator="rkf45")
        if params is not None:
            from paper_2003_04930_amd import warmstart as W
            runs["accelerated"] = lambda: Q.steady_state(
                Pn, w, DT, TOL, 400000, rho0=W.warm_rho0(Pn, w, params, integrator="rkf45"),
                integrator="rkf45")
    if not args.no_mixed:
        runs["mixed_fp32"] = lambda: Q.steady_state(Pn, w, DT, TOL, 400000, prec="fp32")
        if params is not None:
            from paper_2003_04930_amd import warmstart as W
            # mixed precision from the learned warm start (inference included)
            runs["mixed_fp32_warm"] = lambda: Q.steady_state(
                Pn, w, DT, TOL, 400000, rho0=W.warm_rho0(Pn, w, params), prec="fp32")

            # the batched mixed warm-start form: qpr_batch_solve, FP32 steps with the FP64
            # fold and judge, from the learned warm start (inference included)
            def batch_warm():
                rb = Q.batch_solve([(Pn, w)], tol=TOL, prec="fp32",
                                   rho0s=W.warm_rho0_batch([(Pn, w)], params))
                return Q.SolveResult(rb.rhos[0], rb.ranks[0], rb.stats[0], rb.status)
            runs["batch_mixed_fp32_warm"] = batch_warm
    for name, fn in runs.items():
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        err = float((r.rho - plain.rho).abs().max())
        p_ref = plain.rho[0].diagonal().cpu().numpy()
        row[name] = {"seconds": t, "steps": r.stats["steps"], "speedup_vs_plain": plain.stats["seconds"] / t,
                     "max_abs_drho_vs_plain": err,
                     "ranking_identical": bool(torch.equal(r.rank, plain.rank)),
                     "order_violations_beyond_2maxdrho":
                         tie_aware_rank_check(p_ref, r.rank.cpu().numpy(), 2 * err, np)}
        log(f"n=4096 {name}: {t:.2f} s ({plain.stats['seconds'] / t:.1f}x), max|drho| {err:.1e}")
    # hub classes and degeneracy of PageRank against the quantum steady state
    # (tie resolution: twice the spread of two independent solves)
    from paper_2003_04930_amd import study
    tau = 2 * row.get("fp64_rkf45", {}).get("max_abs_drho_vs_plain", 5e-8)
    row["study"] = study.hub_study(Q, Pn, plain.rho, tau)
    return row


def n2048_rows(Q, inputs, torch, np):
    """BA graph N = 2048 (m = 4) at omega = 0.8: the plain FP64 RK4 solve, RKF45
    beside it (its spread to the plain state sets the tie resolution), and the
    PageRank-versus-quantum study."""
    from paper_2003_04930_amd import study
    n, w = 2048, 0.8
    Pn = Q.Problem.from_graph(inputs.ba_digraph(n, 4, seed=0))
    plain = Q.steady_state(Pn, w, DT, TOL, 400000)
    rf = Q.steady_state(Pn, w, DT, TOL, 400000, integrator="rkf45")
    err = float((rf.rho - plain.rho).abs().max())
    log(f"n=2048 plain fp64: {plain.stats['seconds']:.2f} s, {plain.stats['steps']} steps")
    return {"omega": w, "plain_fp64": {"seconds": plain.stats["seconds"],
                                       "rk4_steps": plain.stats["steps"]},
            "fp64_rkf45": {"seconds": rf.stats["seconds"], "steps": rf.stats["steps"],
                           "max_abs_drho_vs_plain": err},
            "study": study.hub_study(Q, Pn, plain.rho, 2 * err)}


def batch_family_rows(Q, inputs, params, torch, np, mode):
    """The batching workload: 256 family graphs (N uniform in [50, 922], half
    ER with mean out-degree 4, half BA with m in 2..5) x 5 omegas = 1,280
    systems to ||L|| < 1e-8.  "subset": FP64 RKF45 from the warm start over
    all 1,280 systems (concurrent form) and the FP32 defect correction (FP32
    steps, FP64 judge) over the first 32 graphs (160 systems) in both forms;
    "full": the FP32 defect correction over all 1,280 in both forms too."""
    items = []
    for k in range(256):
        Pk = Q.Problem.from_graph(inputs.batch_graph(k))
        items += [(Pk, w) for w in inputs.BATCH_OMEGAS]
    out = {"systems": len(items), "sum_n2": int(sum(P.n ** 2 for P, _ in items))}
    runs = []
    if params is not None:
        runs.append(("rkf45_fp64_warm_concurrent", items, dict(prec="fp64", integrator="rkf45",
                                                               mode="concurrent"), True))
    sub = items if mode == "full" else items[:160]
    runs.append(("mixed_fp32_concurrent", sub, dict(prec="fp32", mode="concurrent"), False))
    runs.append(("mixed_fp32_persistent", sub, dict(prec="fp32", mode="persistent"), False))
    for name, its, kw, warm in runs:
        t0 = time.perf_counter()
        rho0s = None
        if warm:
            from paper_2003_04930_amd import warmstart as W
            rho0s = W.warm_rho0_batch(its, params, integrator=kw.get("integrator", "rk4"))
        rb = Q.batch_solve(its, tol=TOL, want_rank=True, rho0s=rho0s, **kw)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        st = [x["steps"] for x in rb.stats]
        res = max(x["residual"] for x in rb.stats)
        out[name] = {"systems": len(its), "seconds": secs, "solves_per_s": len(its) / secs,
                     "steps_min_mean_max": [min(st), float(np.mean(st)), max(st)],
                     "max_residual": res,
                     "all_converged": all(x["converged"] == 1 for x in rb.stats)}
        log(f"batch family {name}: {len(its)} systems in {secs:.1f} s ({len(its) / secs:.1f} solves/s)")
        del rb
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-rkf45", action="store_true",
                    help="skip the adaptive-integrator and accelerated rows")
    ap.add_argument("--no-4096", action="store_true", help="skip the N = 4096 rows")
    ap.add_argument("--batch-graphs", type=int, default=0,
                    help="also time qpr_batch_solve on this many family graphs x 5 omegas")
    ap.add_argument("--batch-rows", default="fp64,fp64_rkf45,fp64_rkf45_warm,fp32",
                    help="comma list of batched rows to time")
    ap.add_argument("--batch-mode", default="auto", choices=["auto", "persistent", "concurrent"],
                    help="how qpr_batch_solve runs the --batch-graphs systems")
    ap.add_argument("--batch-family", default="subset", choices=["off", "subset", "full"],
                    help="the 1,280-system batching workload (see batch_family_rows)")
    ap.add_argument("--precision-n", type=int, default=0,
                    help="also compare FP64 with FP32/BF16x3 products at this N (BA m=4)")
    ap.add_argument("--warm", default=WEIGHTS,
                    help="warm-start weights (.npy) for the accelerated rows, or 'none'")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solver "
              "has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2003_04930_amd import inputs, qpr as Q
    # the batch solves report how many systems have finished every 30 s
    os.environ.setdefault("QPR_PROGRESS", "30")

    torch.cuda.set_device(0)
    g = inputs.ba_digraph(N, M_BA, seed=0)
    log(f"graph {g}")
    t_build0 = time.perf_counter()
    P = Q.Problem.from_graph(g)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t_build0

    for k in range(args.warmup):
        log(f"warmup {k}")
        solve_all(Q, P, "fp64")
    torch.cuda.synchronize()
    log("timed region")
    t0 = time.perf_counter()
    results = None
    for k in range(args.steps):
        results = solve_all(Q, P, "fp64")
        log(f"step {k} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    steps = [r.stats["steps"] for r in results]
    per_omega = {str(w): {"seconds": r.stats["seconds"], "rk4_steps": r.stats["steps"],
                          "residual": r.stats["residual"]} for w, r in zip(OMEGAS, results)}
    value = ms_per_step / 1e3 / len(OMEGAS)   # seconds per solve (time-to-steady-state)
    log(f"fp64: {value:.3f} s/solve, steps {steps}")
    # the same three solves one after another on one stream, for comparison
    torch.cuda.synchronize()
    t0s = time.perf_counter()
    seq = solve_sequential(Q, P)
    torch.cuda.synchronize()
    seq_value = (time.perf_counter() - t0s) / len(OMEGAS)
    seq_same = all(bool(torch.equal(a.rho, b.rho)) and a.stats["steps"] == b.stats["steps"]
                   for a, b in zip(seq, results))
    del seq
    log(f"fp64 sequential: {seq_value:.3f} s/solve, bitwise equal to the concurrent solves "
        f"{seq_same}")

    # Kernels of the timed path, timed with HIP events on the stream they run
    # on, one kernel at a time.  At this density the product is the sparse one:
    # while two or more of the concurrent solves run, a stage is one fused
    # epilogue launch (k_epilogue_fused, the gathers inside the tile kernel);
    # the solve left running alone takes k_spmm + k_epilogue per stage.  The
    # dense MFMA product is timed too.
    rho_ss = results[-1].rho
    sparse = P.p.nnz_h < 0.05 * N * N
    sp_ms, epi_ms = Q.time_kernels(P, OMEGAS[-1], rho_ss, prec="fp64", cfg=-2, reps=200)
    _, fused_ms = Q.time_kernels(P, OMEGAS[-1], rho_ss, prec="fp64",
                                 cfg=-3 - len(Q.SPARSE_VARIANTS), reps=200)
    gemm_ms, _ = Q.time_kernels(P, OMEGAS[-1], rho_ss, prec="fp64", reps=100)
    # stages of each kind in the timed path: a solve's steps run fused while
    # another solve still runs (up to the second-longest step count), the rest
    # of the longest solve as two kernels
    srt = sorted(steps)
    fused_steps = sum(min(k, srt[-2]) for k in srt)
    alone_steps = srt[-1] - srt[-2]
    ld = P.ld
    # Algorithmic bytes per launch.  Per the hot-path scope (the measurement
    # table of the fused passes) a fused RK4 stage moves ~80 B per element of
    # the N x N state with tile-pair fusion (Y_s 16 read, y_n 16, accumulator
    # 16 read + 16 written, Y_{s+1} 16 written) and ~128 B when X makes a round
    # trip through HBM (X 16 written by the product and 16 read back, plus the
    # product's 16 B read of Y); a sparse product reads Y once and writes X
    # (32 B).  These are the figures `frac` uses.
    # The kernels here touch less: y_n and the accumulator only on the upper
    # triangle of tiles (Hermitian tile pairs), so the unique data per element
    # is 58 B for the two-kernel epilogue (stage 1 48, stages 2-3 64, stage 4
    # 56; X read in full) and 50 B for the fused epilogue (X gathered, Y_s read
    # in full) -- reported beside them as "unique" bytes.
    B_FUSED, B_TWO_KERNEL, B_SPMM = 80.0, 128.0 - 32.0, 32.0
    U_FUSED, U_EPI = 50.0, 58.0
    epi_bytes = B_TWO_KERNEL * N * N
    sp_bytes = B_SPMM * N * N
    fused_bytes = B_FUSED * N * N
    flops = 4.0 * N ** 3                       # dense product: two real N x N x N products
    gemm_tf = flops / (gemm_ms * 1e-3) / 1e12
    epi_gbs = epi_bytes / (epi_ms * 1e-3) / 1e9
    sp_gbs = sp_bytes / (sp_ms * 1e-3) / 1e9
    fused_gbs = fused_bytes / (fused_ms * 1e-3) / 1e9
    log(f"stage: spmm {sp_ms * 1e3:.1f} us ({sp_gbs:.0f} GB/s), epilogue {epi_ms * 1e3:.1f} us "
        f"({epi_gbs:.0f} GB/s), fused epilogue {fused_ms * 1e3:.1f} us ({fused_gbs:.0f} GB/s); "
        f"dense product {gemm_ms * 1e3:.1f} us ({gemm_tf:.1f} TF/s)")
    # the whole timed region: every stage's algorithmic bytes over the wall time
    timed_bytes = 4 * fused_steps * fused_bytes + 4 * alone_steps * (epi_bytes + sp_bytes)
    agg_gbs = timed_bytes * args.steps / ((t1 - t0)) / 1e9
    if sparse:
        # the dominant kernel: the largest launch count x launch time
        cands = [("k_epilogue_fused<3> (sparse gathers + RHS + RK4 stage)", fused_gbs,
                  fused_bytes, fused_ms, "fused", 4 * fused_steps, U_FUSED),
                 ("k_epilogue<2> (fused RHS + RK4 stage)", epi_gbs, epi_bytes, epi_ms,
                  "epilogue", 4 * alone_steps, U_EPI),
                 ("k_spmm (sparse commutator product)", sp_gbs, sp_bytes, sp_ms, "spmm",
                  4 * alone_steps, B_SPMM)]
        dom = max(cands, key=lambda c: c[3] * c[5])
        uniq = dom[6] * N * N
        roofline = {"bound": "hbm", "achieved": dom[1], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": dom[1] / HBM_PEAK_GBS, "traffic": measured_traffic(dom[4]),
                    "kernel": dom[0], "bytes_per_launch": dom[2],
                    "bytes_per_element": dom[2] / (N * N),
                    "us_per_launch": dom[3] * 1e3,
                    "launch_time": "the kernel alone, HIP events on its stream (qpr_time_kernels)",
                    "launches_in_timed_step": dom[5],
                    "unique_bytes_per_launch": uniq,
                    "frac_unique_bytes": uniq / (dom[3] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "timed_region": {"stages_fused": 4 * fused_steps,
                                     "stages_two_kernel": 4 * alone_steps,
                                     "algorithmic_bytes_per_step": timed_bytes,
                                     "aggregate_GBs": agg_gbs,
                                     "aggregate_frac": agg_gbs / HBM_PEAK_GBS}}
    else:
        roofline = {"bound": "mfma", "achieved": gemm_tf, "peak": FP64_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": gemm_tf / FP64_PEAK_TFLOPS, "traffic": None,
                    "kernel": "k_gemm_k4<double> (dense commutator product)",
                    "flops_per_launch": flops, "us_per_launch": gemm_ms * 1e3}

    extra = {"per_omega_fp64": per_omega, "build_seconds": t_build,
             "seconds_per_solve_fp64": value, "product": "sparse" if sparse else "dense",
             "sequential_fp64": {"seconds_per_solve": seq_value,
                                 "concurrency_speedup": seq_value / value,
                                 "bitwise_equal": seq_same},
             "dense_product": {"us": gemm_ms * 1e3, "achieved_TFs": gemm_tf,
                               "peak_TFs": FP64_PEAK_TFLOPS, "frac": gemm_tf / FP64_PEAK_TFLOPS,
                               "flops_per_launch": flops},
             "epilogue": {"us": epi_ms * 1e3, "achieved_GBs": epi_gbs,
                          "frac": epi_gbs / HBM_PEAK_GBS, "bytes_per_launch": epi_bytes,
                          "frac_unique_bytes": U_EPI * N * N / (epi_ms * 1e-3) / 1e9 /
                          HBM_PEAK_GBS},
             "spmm": {"us": sp_ms * 1e3, "achieved_GBs": sp_gbs,
                      "frac": sp_gbs / HBM_PEAK_GBS, "bytes_per_launch": sp_bytes},
             "fused_epilogue": {"us": fused_ms * 1e3, "achieved_GBs": fused_gbs,
                                "frac": fused_gbs / HBM_PEAK_GBS, "bytes_per_launch": fused_bytes,
                                "frac_unique_bytes": U_FUSED * N * N / (fused_ms * 1e-3) / 1e9 /
                                HBM_PEAK_GBS},
             "stages_in_timed_step": {"fused": 4 * fused_steps, "two_kernel": 4 * alone_steps},
             "nnz_h": int(P.p.nnz_h), "ld": ld}

    params = None
    if args.warm and args.warm != "none":
        from paper_2003_04930_amd import warmstart as W
        params = W.load(args.warm)

    if not args.no_rkf45:
        # the paper's own integrator: adaptive Fehlberg 4(5), FP64, same tolerance
        t0f = time.perf_counter()
        rf = solve_all(Q, P, "fp64", integrator="rkf45")
        torch.cuda.synchronize()
        tf = (time.perf_counter() - t0f) / len(OMEGAS)
        errf = max(float((a.rho - b.rho).abs().max()) for a, b in zip(rf, results))
        extra["fp64_rkf45"] = {"seconds_per_solve": tf,
                               "accepted_steps": [r.stats["steps"] for r in rf],
                               "rejected_steps": [r.stats["rejected"] for r in rf],
                               "last_step": [r.stats["last_step"] for r in rf],
                               "max_abs_drho_vs_rk4": errf, "speedup_vs_rk4": value / tf}
        log(f"fp64 rkf45: {tf:.3f} s/solve, accepted {[r.stats['steps'] for r in rf]}, "
            f"rejected {[r.stats['rejected'] for r in rf]}, max|drho| vs RK4 {errf:.1e}")
        if params is not None:
            extra["accelerated"] = accelerated(Q, W, P, params, results, value, torch, np)
            extra["target"] = target_rows(Q, W, P, params, results, value, torch, np)

    if not args.no_rkf45:
        # hub classes and degeneracy at N = 922, per omega (tie resolution:
        # twice the spread between the RK4 and RKF45 steady states)
        from paper_2003_04930_amd import study
        tau = 2 * extra["fp64_rkf45"]["max_abs_drho_vs_rk4"]
        extra["study_n922"] = {str(w): study.hub_study(Q, P, r.rho, tau)
                               for w, r in zip(OMEGAS, results)}
        extra["n2048"] = n2048_rows(Q, inputs, torch, np)

    if not args.no_4096:
        extra["n4096"] = n4096_rows(Q, inputs, params, torch, np, args)
        su = extra["n4096"]["stage_us"]
        if sparse:
            roofline["n4096_fused_stage"] = {
                "us_per_launch": su["fused_epilogue"], "bytes_per_launch": 80.0 * 4096 ** 2,
                "achieved": su["fused_GBs"], "frac": su["fused_frac"],
                "frac_unique_bytes": su["fused_frac_unique_bytes"]}

    if not args.no_dense:
        t0d = time.perf_counter()
        rd = solve_all(Q, P, "fp64", product="dense")
        torch.cuda.synchronize()
        td = (time.perf_counter() - t0d) / len(OMEGAS)
        err = max(float((a.rho - b.rho).abs().max()) for a, b in zip(rd, results))
        extra["fp64_dense_mfma"] = {"seconds_per_solve": td,
                                    "rk4_steps": [r.stats["steps"] for r in rd],
                                    "max_abs_drho_vs_timed": err}
        log(f"fp64 dense MFMA: {td:.3f} s/solve")

    if not args.no_mixed:
        for prec in ("bf16x3", "fp32"):
            t0m = time.perf_counter()
            rm = solve_all(Q, P, prec)
            torch.cuda.synchronize()
            tm = (time.perf_counter() - t0m) / len(OMEGAS)
            err = max(float((a.rho - b.rho).abs().max()) for a, b in zip(rm, results))
            pm, _ = Q.time_kernels(P, OMEGAS[-1], rho_ss, prec=prec, reps=100)
            peak = BF16_PEAK_TFLOPS / 3.0 if prec == "bf16x3" else FP32_PEAK_TFLOPS
            extra[f"mixed_{prec}"] = {
                "seconds_per_solve": tm, "rk4_steps": [r.stats["steps"] for r in rm],
                "folds": [r.stats["folds"] for r in rm],
                "max_abs_drho_vs_fp64": err, "product_us": pm * 1e3,
                "product_TFs_algorithmic": flops / (pm * 1e-3) / 1e12,
                "product_frac": flops / (pm * 1e-3) / 1e12 / peak,
                "speedup_vs_fp64": value / tm}
            log(f"{prec}: {tm:.3f} s/solve, max|drho| {err:.2e}, product {pm * 1e3:.1f} us")

    if args.batch_family != "off":
        extra["batch_family"] = batch_family_rows(Q, inputs, params, torch, np, args.batch_family)

    if args.batch_graphs:
        items = []
        for k in range(args.batch_graphs):
            Pk = Q.Problem.from_graph(inputs.batch_graph(k))
            items += [(Pk, w) for w in inputs.BATCH_OMEGAS]
        runs = [("fp64", dict(prec="fp64")), ("fp64_rkf45", dict(prec="fp64", integrator="rkf45"))]
        if params is not None:
            runs.append(("fp64_rkf45_warm", dict(prec="fp64", integrator="rkf45", warm=True)))
        if not args.no_mixed:
            runs.append(("fp32", dict(prec="fp32")))
        wanted = set(args.batch_rows.split(","))
        for name, kw in runs:
            if name not in wanted:
                continue
            rho0s = None
            t_inf = 0.0
            if kw.pop("warm", False):
                from paper_2003_04930_amd import warmstart as W
                t0i = time.perf_counter()
                rho0s = W.warm_rho0_batch(items, params, integrator=kw.get("integrator", "rk4"))
                torch.cuda.synchronize()
                t_inf = time.perf_counter() - t0i
            rb = Q.batch_solve(items, tol=TOL, want_rank=True, rho0s=rho0s,
                               mode=args.batch_mode, **kw)
            st = [x["steps"] for x in rb.stats]
            secs = rb.seconds + t_inf
            extra[f"batch_{name}"] = {
                "systems": len(items), "seconds": secs, "inference_seconds": t_inf,
                "solves_per_s": len(items) / secs, "tuned_cfg": rb.tuned_cfg,
                "mode": args.batch_mode,
                "steps_min_mean_max": [min(st), float(np.mean(st)), max(st)],
                "sum_n2": int(sum(Pk.n ** 2 for Pk, _ in items))}
            log(f"batch {name}: {len(items)} systems in {secs:.2f} s "
                f"({len(items) / secs:.2f} solves/s)")

    if args.precision_n:
        nP = args.precision_n
        Pn = Q.Problem.from_graph(inputs.ba_digraph(nP, 4, seed=0))
        ref = Q.steady_state(Pn, 0.8, DT, TOL, 400000)
        row = {"fp64_sparse": {"seconds": ref.stats["seconds"], "rk4_steps": ref.stats["steps"]}}
        p_ref = ref.rho[0].diagonal().double()
        for prec in ("fp32", "bf16x3"):
            r = Q.steady_state(Pn, 0.8, DT, TOL, 400000, prec=prec)
            err = float((r.rho - ref.rho).abs().max())
            # ranking agreement on pairs whose gap exceeds 2 max|drho| (tie classes below)
            p = p_ref.cpu().numpy()
            tau = 2 * err
            bad = tie_aware_rank_check(p, r.rank.cpu().numpy(), tau, np)
            ties = int(np.sum(np.diff(np.sort(p)) <= tau))
            row[prec] = {"seconds": r.stats["seconds"], "rk4_steps": r.stats["steps"],
                         "folds": r.stats["folds"], "max_abs_drho_vs_fp64": err,
                         "adjacent_order_violations_beyond_tau": bad, "tie_gaps_within_tau": ties}
            log(f"precision n={nP} {prec}: {r.stats['seconds']:.2f} s, max|drho| {err:.2e}, "
                f"order violations {bad}, tie gaps {ties}")
        extra[f"precision_n{nP}"] = row

    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline(g, steps)
        log(f"cpu oracle ~{cpu['seconds_per_solve']:.1f} s/solve")

    line = {
        "metric": METRIC, "value": 1.0 / value, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"ba{N}-m{M_BA}-s0 FP64 steady state, omega in {list(OMEGAS)}, "
                               f"dt={DT}, tol={TOL}, rho0=I/N, RK4, the three solves "
                               f"concurrent on three streams; value = solves per second "
                               f"({'sparse' if sparse else 'dense'} product)",
                   "n": N, "omegas": list(OMEGAS), "tol": TOL, "dt": DT},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line, default=_json_default), flush=True)


if __name__ == "__main__":
    main()
