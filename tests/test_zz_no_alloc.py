"""qpr_rk4_step_noalloc (workspace in the library's static device array)
against qpr_rk4_step (caller workspace), called through the C ABI: the same
kernels on the same inputs, so the states and diagnostics agree bitwise.  Two
no-allocation calls in a row, the second on a smaller problem, so that what
the first left in the shared array must not leak into the second; then the
size and precision limits."""
import numpy as np
import pytest

from paper_2003_04930_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def Q():
    from paper_2003_04930_amd import qpr
    qpr.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return qpr


def _pair(Q, g, omega, nsteps, product, seed):
    P = Q.Problem.from_graph(g)
    rho = Q.planar(inputs.random_density(g.n, seed=seed))
    want = rho.clone()
    dw = Q.rk4_step(P, omega, 0.01, nsteps, want, diag=True, product=product)
    got = rho.clone()
    dg = torch.zeros(4, dtype=torch.float64, device="cuda")
    Q.rk4_step_noalloc(P, omega, 0.01, nsteps, got, diag=dg, product=product)
    torch.cuda.synchronize()
    return want, got, dw, dg


@pytest.mark.parametrize("product", ["auto", "fused", "dense"])
def test_noalloc_matches_workspace_entry_point(Q, product):
    big = inputs.ba_digraph(1000, 3, seed=5)      # ld 1024: the largest size served
    small = inputs.er_digraph(70, 0.06, seed=3)   # ld 128, ragged
    for g, om, k, seed in ((big, 0.7, 3, 1), (small, 0.4, 5, 2)):
        want, got, dw, dg = _pair(Q, g, om, k, product, seed)
        assert torch.equal(got, want), (g, product)
        assert torch.equal(dg, dw)
        assert float(dg[2]) == 0.0                # bitwise Hermitian


def test_noalloc_limits(Q):
    g = inputs.ba_digraph(1100, 2, seed=1)
    P = Q.Problem.from_graph(g)
    rho = Q.planar(inputs.random_density(g.n, seed=4))
    with pytest.raises(Q.QprError) as e:
        Q.rk4_step_noalloc(P, 0.5, 0.01, 1, rho)
    assert e.value.status == Q.QPR_E_ARG
    P2 = Q.Problem.from_graph(inputs.er_digraph(40, 0.1, seed=1))
    r2 = Q.planar(inputs.random_density(40, seed=5))
    L = Q.lib()
    st = L.qpr_rk4_step_noalloc(Q.C.byref(P2.p), 0.5, 0.01, 1, Q._ptr(r2), Q.PREC["fp32"], None,
                                None, Q._stream())
    assert st == Q.QPR_E_ARG
    # after the rejected calls the entry point still works
    want, got, dw, dg = _pair(Q, inputs.er_digraph(40, 0.1, seed=1), 0.5, 2, "auto", 6)
    assert torch.equal(got, want) and torch.equal(dg, dw)
