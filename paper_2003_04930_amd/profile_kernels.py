"""Launch one solver kernel repeatedly for hardware-counter passes.

    rocprofv3 --pmc FETCH_SIZE -d OUT -- python -m paper_2003_04930_amd.profile_kernels \
        --n 922 --kernel sparse --reps 20

Runs `reps` launches of the chosen kernel on the benchmark graph (BA m=3 for
N=922, m=4 otherwise; rho = the FP64 steady state at omega = 0.8 is not
needed for traffic, a random density matrix is used), then a plain
device-to-device copy of --copy-mb MiB so the counters can be calibrated
against a kernel whose traffic is known (copy reads and writes exactly that
many bytes).

Kernels: sparse (FP64 sparse product plus the epilogues of the four RK4
stages; --variant picks the sparse-product kernel variant, default the
library's), fused (the fused epilogue of the four stages, gathers inside),
fp32sparse (the FP32-operand sparse product of the mixed solve),
fused32s (the fused stages of the mixed solve with the defect held in FP32),
dense (FP64 MFMA product), blocksparse / blocksparse32 (the tile-skipping MFMA
product, FP64 / FP32 operands), bf16x3 / fp32 (low-precision MFMA products);
each followed by the epilogues of `reps` RK4 steps.
"""
from __future__ import annotations

import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=922)
    ap.add_argument("--kernel", default="sparse",
                    choices=["sparse", "fused", "fp32sparse", "fused32s", "dense", "fp32", "bf16x3",
                             "blocksparse", "blocksparse32"])
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--copy-mb", type=int, default=256)
    ap.add_argument("--variant", type=int, default=-1,
                    help="sparse-product variant index (-1 = default)")
    args = ap.parse_args()
    import torch
    from paper_2003_04930_amd import inputs, qpr as Q

    g = inputs.ba_digraph(args.n, 3 if args.n <= 1000 else 4, seed=0)
    P = Q.Problem.from_graph(g)
    rho = Q.planar(inputs.random_density(args.n, seed=1))
    prec = {"sparse": "fp64", "fused": "fp64", "dense": "fp64", "blocksparse": "fp64",
            "fp32sparse": "fp32", "fused32s": "fp32", "blocksparse32": "fp32"}.get(args.kernel,
                                                                                  args.kernel)
    sparse = args.kernel in ("sparse", "fp32sparse")
    cfg = (-2 if args.variant < 0 else -3 - args.variant) if sparse else -1
    nvar = len(Q.SPARSE_VARIANTS)
    if args.kernel == "fused":  # the fused epilogue alone (no product launch)
        cfg = -3 - nvar
    if args.kernel in ("blocksparse", "blocksparse32"):
        cfg = -3 - (nvar + 1)
    if args.kernel == "fused32s":
        cfg = -3 - (nvar + 2)
    prod_ms, epi_ms = Q.time_kernels(P, 0.8, rho, prec=prec, cfg=cfg, reps=args.reps)
    nbytes = args.copy_mb << 20
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"[profile] n={args.n} kernel={args.kernel} variant={args.variant} reps={args.reps} "
          f"product_us={prod_ms * 1e3:.2f} epilogue_us={epi_ms * 1e3:.2f} "
          f"copy_bytes={nbytes}", flush=True)


if __name__ == "__main__":
    main()
