"""Batched solve (qpr_batch_solve) against single-system solves and the oracle.

The batched kernels run the same tile code with the same per-system
reduction order as the single-system kernels, so an FP64 batch must
reproduce each single solve bit for bit (same step count, same state);
the FP32 batch is judged in FP64 and must meet the tolerance as re-measured
by the oracle and stay within 1e-6 of the oracle's steady state.
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
    assert torch.cuda.is_available()
    return qpr


def small_family():
    gs = [inputs.er_digraph(40, 0.1, seed=1), inputs.ba_digraph(75, 2, seed=2),
          inputs.er_digraph(130, 0.03, seed=3), inputs.ba_digraph(200, 3, seed=4),
          inputs.batch_graph(0), inputs.batch_graph(1)]
    return gs


@pytest.mark.parametrize("product", ["sparse", "dense", "fused"])
def test_fp64_batch_equals_single_solves(Q, product):
    gs = small_family()[:4]
    probs = [Q.Problem.from_graph(g) for g in gs]
    items = [(P, w) for P in probs for w in (0.3, 0.8)]
    out = Q.batch_solve(items, tol=1e-9, product=product, chunk=16)
    for k, (P, w) in enumerate(items):
        ref = Q.steady_state(P, w, 0.01, 1e-9, 400000, product=product)
        assert out.stats[k]["converged"] == 1
        assert out.stats[k]["steps"] == ref.stats["steps"]
        assert torch.equal(out.rhos[k], ref.rho)
        assert torch.equal(out.ranks[k], ref.rank)


@pytest.mark.parametrize("product", ["sparse", "dense", "fused"])
def test_rkf45_batch_equals_single_solves(Q, product):
    """Each system keeps its own Fehlberg step size and control; the batched
    kernels reproduce the single adaptive solves bit for bit."""
    gs = small_family()[:4]
    probs = [Q.Problem.from_graph(g) for g in gs]
    items = [(P, w) for P in probs for w in (0.2, 0.9)]
    out = Q.batch_solve(items, tol=1e-9, product=product, chunk=8, integrator="rkf45")
    for k, (P, w) in enumerate(items):
        ref = Q.steady_state(P, w, 0.01, 1e-9, 400000, product=product, integrator="rkf45")
        st = out.stats[k]
        assert st["converged"] == 1
        assert st["steps"] == ref.stats["steps"] and st["rejected"] == ref.stats["rejected"]
        assert st["last_step"] == ref.stats["last_step"]
        assert torch.equal(out.rhos[k], ref.rho)
        assert torch.equal(out.ranks[k], ref.rank)


def test_rkf45_batch_rejects_low_precision(Q):
    P = Q.Problem.from_graph(inputs.er_digraph(20, 0.2, seed=0))
    with pytest.raises(Q.QprError) as e:
        Q.batch_solve([(P, 0.5)], prec="fp32", integrator="rkf45")
    assert e.value.status == Q.QPR_E_ARG


def test_batch_graph_replay_equals_eager(Q):
    gs = small_family()[:3]
    items = [(Q.Problem.from_graph(g), w) for g in gs for w in (0.5,)]
    a = Q.batch_solve(items, tol=1e-9, chunk=8, use_graph=True)
    b = Q.batch_solve(items, tol=1e-9, chunk=8, use_graph=False)
    for x, y in zip(a.rhos, b.rhos):
        assert torch.equal(x, y)


@pytest.mark.parametrize("product", ["sparse", "dense", "fused"])
def test_fp32_batch_meets_fp64_judge_and_oracle(Q, product):
    gs = small_family()
    items = [(Q.Problem.from_graph(g), w) for g in gs for w in (0.1, 0.9)]
    out = Q.batch_solve(items, prec="fp32", tol=1e-8, chunk=32, product=product)
    # the dense FP32 product is tuned on the batch; the sparse one has no tiles
    assert (out.tuned_cfg >= 0) == (product == "dense")
    for k, ((P, w), g) in enumerate(zip(items, [g for g in gs for _ in (0.1, 0.9)])):
        st = out.stats[k]
        assert st["converged"] == 1 and st["folds"] >= 1
        rho = Q.to_complex(out.rhos[k])
        R = O.problem_ref(g.n, g.src, g.dst)
        f = lambda r: O.rhs_ref(r, R.H_sparse, R.G, R.d, w)
        assert np.sqrt(np.sum(np.abs(f(rho)) ** 2)) < 1e-8 * (1 + 1e-6)
        assert abs(np.trace(rho).real - 1) < 1e-12
        if g.n <= 130:
            want, _, _ = O.steady_ref(np.eye(g.n) / g.n, f, 0.01, 1e-10, 400000)
            assert np.max(np.abs(rho - want)) < 1e-6


def test_batch_argument_errors(Q):
    g = inputs.er_digraph(20, 0.2, seed=0)
    P = Q.Problem.from_graph(g)
    with pytest.raises(Q.QprError) as e:
        Q.batch_solve([(P, 1.5)])
    assert e.value.status == Q.QPR_E_ARG
    with pytest.raises(Q.QprError) as e:
        Q.batch_solve([(P, 0.5)], prec="bf16x3")
    assert e.value.status == Q.QPR_E_ARG
    out = Q.batch_solve([(P, 0.5)], tol=1e-14, max_steps=20, allow_not_converged=True)
    assert out.status == Q.QPR_E_NOT_CONVERGED and out.stats[0]["steps"] == 20
