"""Train the warm-start network and measure what it gains.

    python -m paper_2003_04930_amd.train_warmstart [--train-graphs 200]
        [--test-graphs 40] [--steps 3000] [--out weights.npy]

1. Training data: graphs 10000.. of the batched family (N uniform in
   [50, 922], ER mean out-degree 4 or BA m in 2..5), each at the five batch
   omegas; steady states from the batched FP64 solver (||L||_F < 1e-8).
2. Training: Adam on the mean per-graph KL divergence, all on the GPU through
   the library's forward/backward/Adam kernels.
3. Gain: on unseen graphs (seeds 20000.., N log-uniform in [50, n_max]) the
   FP64 steady-state solve runs from rho0 = I/N, from diag(PageRank), from
   diag(p_hat) and from the omega-blended start (warmstart.blend_weight); the
   steps to the tolerance are compared (the solve always finishes and judges
   in FP64, so every start reaches the same state; rankings are compared).

Prints one JSON line with the summary.
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


def test_graph(k, n_max):
    rng = np.random.default_rng(20000 + k)
    n = int(np.exp(rng.uniform(np.log(50), np.log(n_max))))
    if k % 2 == 0:
        return inputs.er_digraph(n, 4.0 / (n - 1), seed=20000 + k)
    return inputs.ba_digraph(n, int(rng.integers(2, 6)), seed=20000 + k)


def log(msg):
    print(f"[warmstart] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-graphs", type=int, default=200)
    ap.add_argument("--test-graphs", type=int, default=40)
    ap.add_argument("--n-max-test", type=int, default=1500)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch-graphs", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--load", default=None, help="skip training, evaluate these weights")
    ap.add_argument("--data", default="batch", choices=["batch", "rkf45"],
                    help="steady states for training: batched RK4 or single RKF45 solves")
    args = ap.parse_args()
    import torch

    summary = {}
    if args.load is None:
        t0 = time.perf_counter()
        items = []
        for k in range(args.train_graphs):
            g = inputs.family_graph(10000 + k)
            P = Q.Problem.from_graph(g)
            for w in inputs.BATCH_OMEGAS:
                items.append((P, w))
        log(f"{len(items)} training systems built")
        targets = []
        step = 200
        for i in range(0, len(items), step):
            chunk = items[i:i + step]
            t1 = time.perf_counter()
            if args.data == "batch":
                rhos = Q.batch_solve(chunk, tol=1e-8, want_rank=False).rhos
            else:
                rhos = [Q.steady_state(P, w, 0.01, 1e-8, 400000, want_rank=False,
                                       integrator="rkf45").rho for P, w in chunk]
            targets += [r[0].diagonal().to(torch.float32).clone() for r in rhos]
            log(f"steady states {i + len(rhos)}/{len(items)} ({time.perf_counter() - t1:.1f} s)")
        t_data = time.perf_counter() - t0
        t1 = time.perf_counter()
        params, hist = W.train(items, targets, steps=args.steps, batch_graphs=args.batch_graphs,
                               lr=args.lr, seed=0, log=500)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t1
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        W.save(params, args.out)
        summary.update({"train_systems": len(items), "data_seconds": t_data,
                        "train_seconds": t_train, "loss_first": hist[0],
                        "loss_last100": float(np.mean(hist[-100:]))})
        log(f"trained: loss {hist[0]:.3e} -> {np.mean(hist[-100:]):.3e} in {t_train:.1f} s")
    else:
        params = W.load(args.load)

    rows = []
    for k in range(args.test_graphs):
        g = test_graph(k, args.n_max_test)
        P = Q.Problem.from_graph(g)
        w = inputs.BATCH_OMEGAS[k % len(inputs.BATCH_OMEGAS)]
        cold = Q.steady_state(P, w, 0.01, 1e-8, 400000)
        pr = Q.steady_state(P, w, 0.01, 1e-8, 400000, rho0=W.pagerank_rho0(P), want_rank=False)
        raw = Q.steady_state(P, w, 0.01, 1e-8, 400000, rho0=W.warm_rho0(P, w, params, blend=False),
                             want_rank=False)
        t0 = time.perf_counter()
        rho0 = W.warm_rho0(P, w, params)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
        warm = Q.steady_state(P, w, 0.01, 1e-8, 400000, rho0=rho0)
        err = float((warm.rho - cold.rho).abs().max())
        rows.append({"n": g.n, "omega": w, "cold": cold.stats["steps"], "pagerank": pr.stats["steps"],
                     "raw": raw.stats["steps"], "warm": warm.stats["steps"],
                     "cold_s": cold.stats["seconds"], "warm_s": warm.stats["seconds"] + t_inf,
                     "max_drho": err, "rank_equal": bool(torch.equal(warm.rank, cold.rank))})
        log(f"test {k}: n={g.n} w={w} steps cold/pr/raw/warm {rows[-1]['cold']}/"
            f"{rows[-1]['pagerank']}/{rows[-1]['raw']}/{rows[-1]['warm']}")
    if rows:
        cold = np.array([r["cold"] for r in rows], float)
        prs = np.array([r["pagerank"] for r in rows], float)
        raw = np.array([r["raw"] for r in rows], float)
        warm = np.array([r["warm"] for r in rows], float)
        om = np.array([r["omega"] for r in rows], float)
        by_omega = {}
        for w in sorted(set(om.tolist())):
            m = om == w
            by_omega[str(w)] = {"systems": int(m.sum()),
                                "ratio_warm_vs_identity": float(np.mean(warm[m] / cold[m])),
                                "ratio_raw_vs_identity": float(np.mean(raw[m] / cold[m])),
                                "ratio_pagerank_vs_identity": float(np.mean(prs[m] / cold[m]))}
        summary.update({
            "test_systems": len(rows),
            "mean_steps": {"identity": cold.mean(), "pagerank": prs.mean(), "mpnn_raw": raw.mean(),
                           "mpnn_blended": warm.mean()},
            "mean_step_ratio_mpnn_vs_identity": float(np.mean(warm / cold)),
            "mean_step_ratio_raw_vs_identity": float(np.mean(raw / cold)),
            "mean_step_ratio_mpnn_vs_pagerank": float(np.mean(warm / prs)),
            "fraction_improved_vs_identity": float(np.mean(warm < cold)),
            "by_omega": by_omega,
            "max_drho_warm_vs_cold": max(r["max_drho"] for r in rows),
            "all_ranks_equal": all(r["rank_equal"] for r in rows),
            "rows": rows,
        })
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
