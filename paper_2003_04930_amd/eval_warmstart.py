"""What the learned warm start gains on unseen graphs.

    python -m paper_2003_04930_amd.eval_warmstart [--graphs 500] [--rk4-graphs 100]
        [--n-max 4096] [--weights PATH] [--out summary.json]

Test graphs k = 0.. (seeds 20000 + k): N log-uniform in [50, n_max], even k
Erdos-Renyi with mean out-degree 4, odd k Barabasi-Albert with m in 2..5
(directed as the workloads), omega = the five batch values in turn.  Every
system is solved to ||L(rho)||_F < 1e-8 in FP64 from three start states --
I/N, diag(PageRank of G) and the network's omega-blended prediction
(inference inside the timed start) -- with the adaptive RKF45 integrator for
all graphs and with RK4 (dt = 0.01) for the first --rk4-graphs of them.  The
solves of one start and integrator run together (qpr_batch_solve, concurrent
form).  Reported: accepted steps relative to the I/N start and to the
PageRank start, per omega, the largest state difference between the warm and
the I/N solve, and how many rankings agree exactly.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2003_04930_amd import inputs, qpr as Q, warmstart as W  # noqa: E402

DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "mpnn_warmstart.npy")
TOL = 1e-8


def test_graph(k, n_max):
    """Unseen graph k: seed 20000 + k, N log-uniform in [50, n_max]."""
    rng = np.random.default_rng(20000 + k)
    n = int(np.exp(rng.uniform(np.log(50), np.log(n_max))))
    if k % 2 == 0:
        return inputs.er_digraph(n, 4.0 / (n - 1), seed=20000 + k)
    return inputs.ba_digraph(n, int(rng.integers(2, 6)), seed=20000 + k)


def log(msg):
    print(f"[eval] {msg}", file=sys.stderr, flush=True)


def solve_group(items, starts, integrator, chunk):
    """Steps and states of the systems `items` from the start states given by
    `starts(items_slice)`, in slices of `chunk` systems."""
    import torch
    steps, diag, ranks, rhos_keep = [], [], [], []
    for i in range(0, len(items), chunk):
        sl = items[i:i + chunk]
        rho0s = starts(sl)
        rb = Q.batch_solve(sl, tol=TOL, max_steps=2_000_000, rho0s=rho0s, integrator=integrator,
                           mode="concurrent")
        for r, rk, st in zip(rb.rhos, rb.ranks, rb.stats):
            assert st["converged"] == 1
            steps.append(int(st["steps"]))
            rhos_keep.append(r)
            ranks.append(rk)
        del rb
        torch.cuda.synchronize()
        log(f"  {integrator}: {min(i + chunk, len(items))}/{len(items)} systems")
    return steps, rhos_keep, ranks


def summarise(name, om, cold, pr, warm):
    cold, pr, warm = (np.asarray(x, float) for x in (cold, pr, warm))
    out = {"systems": int(cold.size),
           "ratio_warm_vs_identity": float(np.mean(warm / cold)),
           "ratio_pagerank_vs_identity": float(np.mean(pr / cold)),
           "ratio_warm_vs_pagerank": float(np.mean(warm / pr)),
           "fraction_warm_fewer_steps_than_identity": float(np.mean(warm < cold)),
           "total_steps": {"identity": int(cold.sum()), "pagerank": int(pr.sum()),
                           "warm": int(warm.sum())},
           "by_omega": {}}
    for w in sorted(set(om)):
        m = np.asarray(om) == w
        out["by_omega"][str(w)] = {
            "systems": int(m.sum()),
            "ratio_warm_vs_identity": float(np.mean(warm[m] / cold[m])),
            "ratio_pagerank_vs_identity": float(np.mean(pr[m] / cold[m])),
            "ratio_warm_vs_pagerank": float(np.mean(warm[m] / pr[m])),
            "blend_weight": W.blend_weight(w, name)}
    log(f"{name}: warm/I {out['ratio_warm_vs_identity']:.3f}, PR/I "
        f"{out['ratio_pagerank_vs_identity']:.3f}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--graphs", type=int, default=500)
    ap.add_argument("--rk4-graphs", type=int, default=100)
    ap.add_argument("--n-max", type=int, default=4096)
    ap.add_argument("--chunk", type=int, default=40)
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch

    params = W.load(args.weights)
    t0 = time.perf_counter()
    graphs = [test_graph(k, args.n_max) for k in range(args.graphs)]
    items = [(Q.Problem.from_graph(g), inputs.BATCH_OMEGAS[k % 5]) for k, g in enumerate(graphs)]
    om = [w for _, w in items]
    log(f"{len(items)} systems, N {min(g.n for g in graphs)}..{max(g.n for g in graphs)}, "
        f"built in {time.perf_counter() - t0:.1f} s")

    def identity(sl):
        return None

    def pagerank(sl):
        return [W.pagerank_rho0(P) for P, _ in sl]

    integ_now = ["rk4"]

    def warm(sl):
        return W.warm_rho0_batch(sl, params, integrator=integ_now[0])

    summary = {"graphs": len(items), "n_max": args.n_max, "tol": TOL,
               "n_quartiles": [int(x) for x in np.percentile([g.n for g in graphs],
                                                            [0, 25, 50, 75, 100])]}
    for integ, count in (("rkf45", len(items)), ("rk4", min(args.rk4_graphs, len(items)))):
        integ_now[0] = integ
        sub = items[:count]
        res = {}
        for name, fn in (("identity", identity), ("pagerank", pagerank), ("warm", warm)):
            t1 = time.perf_counter()
            res[name] = solve_group(sub, fn, integ, args.chunk)
            log(f"{integ} from {name}: {count} systems in {time.perf_counter() - t1:.1f} s")
        drho = max(float((a - b).abs().max()) for a, b in zip(res["warm"][1], res["identity"][1]))
        same_rank = sum(bool(torch.equal(a, b)) for a, b in zip(res["warm"][2], res["identity"][2]))
        row = summarise(integ, om[:count], res["identity"][0], res["pagerank"][0], res["warm"][0])
        row.update({"max_abs_drho_warm_vs_identity": drho, "rankings_identical": same_rank})
        summary[integ] = row
        del res
        summary["seconds"] = time.perf_counter() - t0
        if args.out:  # after each integrator, so a later failure keeps this one
            with open(args.out, "w") as fh:
                fh.write(json.dumps(summary) + "\n")
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
