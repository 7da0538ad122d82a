"""Write ss_ba922_diag.txt: the oracle's steady-state populations of the
N = 922 scale-free workload graph (BA m = 3, seed 0, random direction, 10 %
reciprocal) at omega = 0.2, 0.5, 0.8, alpha = 0.85, teleport F of Eq. (S2),
zero-diagonal H, from rho0 = I/N with the oracle's classical RK4 (dt = 0.01)
until ||L(y_n)||_F < 1e-12 (Eq. (1), Supplementary Note 2).

Calls only the oracle and the seeded graph generator:

    OMP_NUM_THREADS=2 python tests/golden/make_ss_ba922.py [omega ...]

With omegas given, each is written to ss_ba922_diag.<omega>.part; without,
the parts are merged into ss_ba922_diag.txt.  About an hour of CPU per omega.
With --check, the omega = 0.8 column is compared with the GMRES null vector
of L (the oracle's time-stepping-free steady state).
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_2003_04930_amd import inputs  # noqa: E402

OMEGAS = (0.2, 0.5, 0.8)
TOL, DT = 1e-12, 0.01


def solve(omega):
    g = inputs.ba_digraph(922, 3, seed=0)
    R = O.problem_ref(g.n, g.src, g.dst)
    f = lambda r: O.rhs_ref(r, R.H_sparse, R.G, R.d, omega)
    y, steps, res = O.steady_ref(np.eye(g.n) / g.n, f, DT, TOL, 400000)
    return np.diag(y).real.copy(), steps, res, float(np.trace(y).real)


def cross_check(omega=0.8):
    """The stored populations against the oracle's other route to the steady
    state, the GMRES null vector of L (no time stepping)."""
    g = inputs.ba_digraph(922, 3, seed=0)
    R = O.problem_ref(g.n, g.src, g.dst)
    f = lambda r: O.rhs_ref(r, R.H_sparse, R.G, R.d, omega)
    rho, res, its = O.steady_null_ref(f, g.n, tol=1e-12, restart=60, maxiter=400)
    col = OMEGAS.index(omega)
    stored = []
    with open(os.path.join(HERE, "ss_ba922_diag.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                stored.append(float(line.split()[1 + col]))
    d = float(np.max(np.abs(np.diag(rho).real - np.array(stored))))
    print(f"omega {omega}: GMRES null vector ({its} iterations, residual {res:.2e}) "
          f"against the stored populations: max |dp| = {d:.2e}")


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--check":
        cross_check()
        return
    if len(sys.argv) > 1:
        for w in map(float, sys.argv[1:]):
            p, steps, res, tr = solve(w)
            with open(os.path.join(HERE, f"ss_ba922_diag.{w}.part"), "w") as fh:
                fh.write(f"{steps} {res!r} {tr!r}\n")
                fh.write("\n".join(repr(float(v)) for v in p) + "\n")
        return
    cols, meta = [], []
    for w in OMEGAS:
        with open(os.path.join(HERE, f"ss_ba922_diag.{w}.part")) as fh:
            steps, res, tr = fh.readline().split()
            meta.append((w, int(steps), float(res), float(tr)))
            cols.append([float(x) for x in fh.read().split()])
    with open(os.path.join(HERE, "ss_ba922_diag.txt"), "w") as fh:
        fh.write("# Steady-state populations Re rho_aa of the oracle (written by\n"
                 "# make_ss_ba922.py, which calls only oracle/ and the graph generator):\n"
                 "# BA m=3 N=922 seed 0 workload graph, alpha 0.85, teleport F, H = max(A, A^T),\n"
                 "# RK4 dt=0.01 from I/N to ||L(y_n)||_F < 1e-12.\n")
        for w, steps, res, tr in meta:
            fh.write(f"# omega {w}: {steps} steps, residual {res:.3e}, trace {tr!r}\n")
        fh.write("# columns: node  p(omega=0.2)  p(omega=0.5)  p(omega=0.8)\n")
        for a in range(len(cols[0])):
            fh.write(f"{a} " + " ".join(repr(c[a]) for c in cols) + "\n")


if __name__ == "__main__":
    main()
