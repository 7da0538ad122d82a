"""Write ss_ba<N>_w08_diag.txt for N = 2048 and 4096: the oracle's
steady-state populations Re rho_aa of the precision workload graphs (BA
m = 4, seed 0, random direction, 10 % reciprocal) at omega = 0.8,
alpha = 0.85, teleport F of Eq. (S2), zero-diagonal H.

The steady state is the oracle's null vector of L (Eq. (1)): the trace-one
rho with L(rho) = 0, found by unpreconditioned GMRES on the traceless
subspace (steady_null_ref), no time stepping -- the oracle's RK4 to
||L|| < 1e-12 would take hours of CPU at this size.  The N = 922 goldens
agree with this route to 2.9e-12 in the populations.

Calls only the oracle and the seeded graph generator:

    OMP_NUM_THREADS=8 python tests/golden/make_ss_ba_w08.py [N ...]

(default both).  About five minutes and 5 GB at N = 2048, half an hour and
20 GB at N = 4096 (GMRES keeps 60 vectors of N^2 complex values).
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_2003_04930_amd import inputs  # noqa: E402

M, OMEGA = 4, 0.8


def write(N):
    out = os.path.join(HERE, f"ss_ba{N}_w08_diag.txt")
    g = inputs.ba_digraph(N, M, seed=0)
    R = O.problem_ref(g.n, g.src, g.dst)
    f = lambda r: O.rhs_ref(r, R.H_sparse, R.G, R.d, OMEGA)
    t0 = time.time()
    rho, res, its = O.steady_null_ref(f, g.n, tol=1e-12, restart=60, maxiter=2000)
    secs = time.time() - t0
    p = np.diag(rho).real
    herm = float(np.max(np.abs(rho - rho.conj().T)))
    lam_min = float(np.linalg.eigvalsh(0.5 * (rho + rho.conj().T))[0])
    with open(out + ".part", "w") as fh:
        fh.write("# Steady-state populations Re rho_aa of the oracle (written by\n"
                 "# make_ss_ba_w08.py, which calls only oracle/ and the graph generator):\n"
                 f"# BA m=4 N={N} seed 0 workload graph, alpha 0.85, teleport F,\n"
                 "# H = max(A, A^T) with zero diagonal, omega 0.8; the GMRES null vector of L\n"
                 f"# (relative tolerance 1e-12, {its} iterations, {secs:.0f} s).\n"
                 f"# ||L(rho)||_F = {res!r}, tr rho = {float(np.trace(rho).real)!r},\n"
                 f"# max |rho - rho^dag| = {herm!r}, lambda_min = {lam_min!r}\n")
        for a, v in enumerate(p):
            fh.write(f"{a} {float(v)!r}\n")
    os.replace(out + ".part", out)
    print(f"N={N}: GMRES {its} iterations in {secs:.0f} s, residual {res:.2e}, "
          f"lambda_min {lam_min:.2e}", flush=True)


if __name__ == "__main__":
    for n in [int(a) for a in sys.argv[1:]] or [2048, 4096]:
        write(n)
