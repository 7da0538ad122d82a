"""Steady states of the precision workload (BA m = 4, seed 0, N = 2048 and
4096, omega = 0.8, RK4 dt = 0.01 to ||L(rho)||_F < 1e-8) in every precision,
each re-measured by the CPU FP64 oracle.

For each solver the oracle's right-hand side gives the residual of the
returned state (it must be below the tolerance), and the state must be trace
one, bitwise Hermitian and positive semidefinite.  The low-precision solves
are compared with the plain FP64 GPU solve, whose residual the oracle has
just confirmed: max |d rho| below the 1e-6 bound of the mixed solves, and the
ranking equal on every pair whose gap exceeds 2 max |d rho| (closer pairs
are tie classes, compared only as a count).  Every solve is also compared
with the oracle's own steady state (tests/golden/ss_ba<N>_w08_diag.txt, the
GMRES null vector of L written by make_ss_ba_w08.py from oracle/ only):
populations within 1e-6 and the oracle's ranking on every pair whose oracle
gap exceeds twice the measured population error.  The smallest eigenvalue of the plain state is computed
(eigvalsh); for the others Weyl's inequality
lambda_min(rho) >= lambda_min(rho_plain) - ||rho - rho_plain||_F bounds it.
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_2003_04930_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OMEGA, DT, TOL = 0.8, 0.01, 1e-8
HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(os.path.dirname(HERE), "paper_2003_04930_amd", "weights",
                       "mpnn_warmstart.npy")


def oracle_populations(n):
    """The oracle's steady-state populations of the size-n workload graph."""
    p = []
    with open(os.path.join(HERE, "golden", f"ss_ba{n}_w08_diag.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                p.append(float(line.split()[1]))
    p = np.array(p)
    assert p.shape == (n,)
    return p


@pytest.fixture(scope="module")
def Q():
    from paper_2003_04930_amd import qpr
    qpr.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return qpr


_CACHE = {}


def workload(Q, n):
    """(problem, oracle problem, plain FP64 solve, its lambda_min), once per n."""
    if n not in _CACHE:
        g = inputs.ba_digraph(n, 4, seed=0)
        P = Q.Problem.from_graph(g)
        R = O.problem_ref(g.n, g.src, g.dst)
        plain = Q.steady_state(P, OMEGA, DT, TOL, 400000)
        rho = Q.to_complex(plain.rho)
        import scipy.linalg as sla
        lmin = float(sla.eigvalsh(rho, subset_by_index=[0, 0])[0])
        _CACHE[n] = (g, P, R, plain, rho, lmin)
    return _CACHE[n]


def oracle_checks(R, rho):
    res = np.sqrt(np.sum(np.abs(O.rhs_ref(rho, R.H_sparse, R.G, R.d, OMEGA)) ** 2))
    assert res < TOL * (1 + 1e-6), res
    assert abs(np.trace(rho).real - 1) < 1e-11
    assert abs(np.trace(rho).imag) < 1e-13
    assert np.array_equal(rho, rho.conj().T)


def against_oracle_steady_state(n, rho, rank):
    """Max population error against the oracle's steady state and its ranking
    on every pair the error resolves."""
    p_or = oracle_populations(n)
    err = float(np.max(np.abs(np.diag(rho).real - p_or)))
    assert err < 1e-6, err
    assert tie_aware_same_order(p_or, rank, 2 * err + 1e-15) == 0
    return err


def tie_aware_same_order(p_ref, rank, tau):
    """Number of pairs with p_ref gap > tau whose order `rank` reverses."""
    n = p_ref.size
    pos = np.empty(n, dtype=np.int64)
    pos[rank] = np.arange(n)
    order = np.argsort(-p_ref, kind="stable")
    ps = p_ref[order]
    bad = 0
    # for each node, every node at least tau below it must come later
    lo = np.searchsorted(-ps, -ps + tau, side="right")   # first index with p < p_i - tau
    suffix_min = np.minimum.accumulate(pos[order][::-1])[::-1]
    for i in range(n):
        if lo[i] < n and suffix_min[lo[i]] < pos[order[i]]:
            bad += 1
    return bad


@pytest.mark.parametrize("n", [2048, 4096])
def test_ba_m4_plain_fp64(Q, n):
    g, P, R, plain, rho, lmin = workload(Q, n)
    assert plain.stats["converged"] == 1
    oracle_checks(R, rho)
    assert lmin >= -1e-12, lmin
    assert plain.stats["herm_err"] == 0.0
    # the GPU's ranking of its own state is the oracle's rank rule (exact)
    assert np.array_equal(plain.rank.cpu().numpy(), O.rank_ref(np.diag(rho).real))
    err = against_oracle_steady_state(n, rho, plain.rank.cpu().numpy())
    assert err < 1e-7, err


def _compare_with_plain(Q, n, got_rho, got_rank):
    g, P, R, plain, rho, lmin = workload(Q, n)
    a = Q.to_complex(got_rho)
    oracle_checks(R, a)
    d = np.max(np.abs(a - rho))
    assert d < 1e-6, d
    assert lmin - np.linalg.norm(a - rho) >= -1e-12
    p_ref = np.diag(rho).real
    assert tie_aware_same_order(p_ref, got_rank.cpu().numpy(), 2 * d + 1e-15) == 0
    against_oracle_steady_state(n, a, got_rank.cpu().numpy())


@pytest.mark.parametrize("n", [2048, 4096])
def test_ba_m4_batched_fp32_mixed_from_warm_start(Q, n):
    """The batched mixed warm-start form: qpr_batch_solve with the FP32 product and the FP64
    fold-and-judge defect correction, started from the learned warm start."""
    from paper_2003_04930_amd import warmstart as W
    g, P, R, plain, rho, lmin = workload(Q, n)
    params = W.load(WEIGHTS)
    rho0 = W.warm_rho0_batch([(P, OMEGA)], params)
    out = Q.batch_solve([(P, OMEGA)], tol=TOL, prec="fp32", rho0s=rho0)
    st = out.stats[0]
    assert st["converged"] == 1 and st["folds"] >= 2
    assert st["herm_err"] == 0.0
    _compare_with_plain(Q, n, out.rhos[0], out.ranks[0])


@pytest.mark.parametrize("n", [2048, 4096])
def test_ba_m4_bf16x3(Q, n):
    """Three bf16 slices on the matrix cores with FP32 accumulation, FP64
    folds and judge."""
    g, P, R, plain, rho, lmin = workload(Q, n)
    out = Q.steady_state(P, OMEGA, DT, TOL, 400000, prec="bf16x3")
    assert out.stats["converged"] == 1
    assert out.stats["herm_err"] == 0.0
    _compare_with_plain(Q, n, out.rho, out.rank)


@pytest.mark.parametrize("n", [2048, 4096])
def test_ba_m4_fp32_mixed_cold(Q, n):
    """The FP32 defect correction from I/N (single-system solve)."""
    g, P, R, plain, rho, lmin = workload(Q, n)
    out = Q.steady_state(P, OMEGA, DT, TOL, 400000, prec="fp32")
    assert out.stats["converged"] == 1
    _compare_with_plain(Q, n, out.rho, out.rank)
