"""Degenerate inputs of the HIP path against the CPU FP64 oracle: the
smallest size, graphs without edges (every column dangling, H_off = 0),
complete graphs (long neighbour lists, dense and sparse products), sizes on
and just past a padding boundary, the omega = 1 classical limit and the
doubly-stochastic fixed point I/N.

Tolerances as in test_gpu_parity.py: 1e-12 on right-hand sides of trace-one
states, step-locked RK4 trajectories within 1e-10 of the oracle.
"""
import numpy as np
import pytest

import oracle as O
from paper_2003_04930_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def Q():
    from paper_2003_04930_amd import qpr
    qpr.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return qpr


def complete(n):
    src, dst = np.nonzero(~np.eye(n, dtype=bool))
    return inputs.Graph(n, src.astype(np.int32), dst.astype(np.int32), f"complete{n}")


CASES = {
    "n2_edge": lambda: inputs.Graph(2, np.array([0], np.int32), np.array([1], np.int32)),
    "n2_empty": lambda: inputs.Graph(2, np.zeros(0, np.int32), np.zeros(0, np.int32)),
    "empty40": lambda: inputs.Graph(40, np.zeros(0, np.int32), np.zeros(0, np.int32)),
    "complete30": lambda: complete(30),
    "er64": lambda: inputs.er_digraph(64, 0.08, seed=11),      # ld = n: no padding
    "er65": lambda: inputs.er_digraph(65, 0.08, seed=12),      # ld = 128: 63 padded rows
    # leaves 1..8 -> hub 0: the hub is dangling, its H row a full group of eight
    "star9": lambda: inputs.Graph(9, np.arange(1, 9, dtype=np.int32), np.zeros(8, np.int32)),
}


@pytest.mark.parametrize("product", ["dense", "sparse", "fused"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_rhs_and_steps_on_degenerate_graphs(Q, name, product):
    g = CASES[name]()
    P = Q.Problem.from_graph(g)
    R = O.problem_ref(g.n, g.src, g.dst)
    rho = inputs.random_density(g.n, seed=g.n + 1)
    for omega in (0.0, 0.6, 1.0):
        got = Q.to_complex(Q.rhs(P, omega, Q.planar(rho), product=product))
        want = O.rhs_ref(rho, R.H, R.G, R.d, omega)
        assert np.max(np.abs(got - want)) < 1e-12 * max(1.0, np.max(np.abs(want))), omega
        assert np.array_equal(got, got.conj().T)
    x = Q.planar(rho)
    Q.rk4_step(P, 0.6, 0.01, 25, x, product=product)
    want = O.rk4_ref(rho, lambda r: O.rhs_ref(r, R.H, R.G, R.d, 0.6), 0.01, 25)
    assert np.max(np.abs(Q.to_complex(x) - want)) < 1e-10


@pytest.mark.parametrize("name", ["star9", "er64", "er65"])
def test_steady_state_step_locked_on_degenerate_graphs(Q, name):
    g = CASES[name]()
    P = Q.Problem.from_graph(g)
    R = O.problem_ref(g.n, g.src, g.dst)
    f = lambda r: O.rhs_ref(r, R.H, R.G, R.d, 0.7)
    want, nsteps, _ = O.steady_ref(np.eye(g.n) / g.n, f, 0.01, 1e-10, 200000)
    out = Q.steady_state(P, 0.7, 0.01, 1e-10, 200000, product="sparse")
    assert nsteps > 100                             # a real trajectory
    assert out.stats["converged"] == 1 and out.stats["steps"] == nsteps
    assert np.max(np.abs(Q.to_complex(out.rho) - want)) < 1e-10


def test_classical_limit_reaches_pagerank(Q):
    """omega = 1: the diagonal follows the classical walk on G and the steady
    state is diag(PageRank) (power iteration on G, here and in the oracle)."""
    g = inputs.ba_digraph(150, 2, seed=5)
    P = Q.Problem.from_graph(g)
    R = O.problem_ref(g.n, g.src, g.dst)
    out = Q.steady_state(P, 1.0, 0.01, 1e-11, 400000)
    p = out.rho[0].diagonal().cpu().numpy()
    pr = O.pagerank_power(R.G)
    assert np.max(np.abs(p - pr)) < 1e-9
    assert np.max(np.abs(P.vector("pagerank").cpu().numpy() - pr)) < 1e-13
    off = out.rho.clone()
    off[0].fill_diagonal_(0.0)
    assert float(off.abs().max()) < 1e-12          # coherences decay at omega = 1


@pytest.mark.parametrize("product", ["dense", "sparse"])
def test_doubly_stochastic_fixed_point(Q, product):
    """On the complete graph G is doubly stochastic and I/N is the steady
    state for every omega: the solve stops at step 0 with that state."""
    g = complete(24)
    P = Q.Problem.from_graph(g)
    for omega in (0.2, 0.9):
        out = Q.steady_state(P, omega, 0.01, 1e-12, 1000, product=product)
        assert out.stats["converged"] == 1 and out.stats["steps"] == 0
        assert np.max(np.abs(Q.to_complex(out.rho) - np.eye(24) / 24)) < 1e-15


@pytest.fixture(scope="module")
def n8192(Q):
    """BA N = 8192 (m = 4) with a rank-16 random density (any Hermitian
    trace-one state serves) and the oracle's right-hand side and RK4 step."""
    n = 8192
    g = inputs.ba_digraph(n, 4, seed=0)
    R = O.problem_ref(g.n, g.src, g.dst)
    rho = inputs.random_density(n, seed=3, rank=16)
    f = lambda r: O.rhs_ref(r, R.H_sparse, R.G, R.d, 0.7)
    return Q.Problem.from_graph(g), rho, f(rho), O.rk4_ref(rho, f, 0.01, 1)


@pytest.mark.parametrize("product", ["sparse", "dense", "fused"])
def test_rhs_and_stages_at_n8192(Q, n8192, product):
    """The largest size tested: the right-hand side and one RK4 step (all four
    stage kernels) against the oracle over every element."""
    P, rho, want_rhs, want_step = n8192
    got = Q.to_complex(Q.rhs(P, 0.7, Q.planar(rho), product=product))
    assert np.max(np.abs(got - want_rhs)) < 1e-12 * max(1.0, np.max(np.abs(want_rhs)))
    assert np.array_equal(got, got.conj().T)
    del got
    x = Q.planar(rho)
    Q.rk4_step(P, 0.7, 0.01, 1, x, product=product)
    assert np.max(np.abs(Q.to_complex(x) - want_step)) < 1e-12
