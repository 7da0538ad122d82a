"""Mixed-precision products (FP32, BF16x3) and the FP64-judged defect
correction, against the CPU FP64 oracle.

Bounds: a low-precision product row sums at most deg(a) terms of the FP32
(or 3-slice bf16, 24-bit) representation of rho with FP32 (dense MFMA) or FP64
(sparse gathers, rounded once to FP32) accumulation, so
|X_lowp - X| <= c * 2^-24 * deg_max * max|rho|; the right-hand side inherits
that times (1 - omega).  The steady state is judged by the FP64 residual, so
the mixed solution must satisfy ||L(rho)||_F < tol re-measured by the oracle
and lie within 1e-6 of the oracle's steady state (the bound set for the mixed
solves).
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


@pytest.mark.parametrize("prec,product", [("fp32", "sparse"), ("fp32", "fused"), ("fp32", "dense"),
                                          ("bf16x3", "dense")])
@pytest.mark.parametrize("n,m,omega", [(70, 2, 0.3), (130, 3, 0.8), (922, 3, 0.5)])
def test_lowp_rhs_error_bound(Q, prec, product, n, m, omega):
    g = inputs.ba_digraph(n, m, seed=n)
    P = Q.Problem.from_graph(g)
    R = O.problem_ref(g.n, g.src, g.dst)
    rho = inputs.random_density(n, seed=3)
    got = Q.to_complex(Q.rhs(P, omega, Q.planar(rho), prec=prec, product=product))
    want = O.rhs_ref(rho, R.H_sparse, R.G, R.d, omega)
    deg = int((R.H != 0).sum(axis=1).max())
    bound = 8 * 2.0 ** -24 * (deg + 1) * np.max(np.abs(rho)) * (1 - omega) + 1e-15
    err = np.max(np.abs(got - want))
    assert err <= bound, (err, bound)
    assert err > 0 or omega == 1.0          # it really is the low-precision path
    assert np.array_equal(got, got.conj().T)


@pytest.mark.parametrize("prec,product", [("fp32", "sparse"), ("fp32", "fused"), ("fp32", "dense"),
                                          ("bf16x3", "dense"), ("fp32", "auto")])
def test_mixed_steady_state_matches_oracle(Q, prec, product):
    """("fp32", "auto") is the defect held in FP32 (every state plane of the
    steps single precision); the explicit products keep it in FP64."""
    g = inputs.ba_digraph(130, 3, seed=1)
    P = Q.Problem.from_graph(g)
    R = O.problem_ref(g.n, g.src, g.dst)
    omega, dt, tol = 0.6, 0.01, 1e-9
    f = lambda r: O.rhs_ref(r, R.H, R.G, R.d, omega)
    want, nsteps, _ = O.steady_ref(np.eye(g.n) / g.n, f, dt, tol, 200000)
    out = Q.steady_state(P, omega, dt, tol, 200000, prec=prec, chunk=32, fold_every=32,
                         product=product)
    got = Q.to_complex(out.rho)
    assert out.stats["converged"] == 1
    assert out.stats["folds"] >= 2
    assert np.sqrt(np.sum(np.abs(f(got)) ** 2)) < tol * (1 + 1e-6)
    assert np.max(np.abs(got - want)) < 1e-6
    assert abs(np.trace(got).real - 1) < 1e-12
    assert out.stats["herm_err"] == 0.0
    # step count within one fold period of the plain FP64 integration
    assert abs(out.stats["steps"] - nsteps) <= 32 + 5
    p_want = np.diag(want).real
    tau = 2 * np.max(np.abs(got - want)) + 1e-15
    order = out.rank.cpu().numpy()
    pos = np.empty_like(order)
    pos[order] = np.arange(g.n)
    for i in range(g.n):
        for j in range(g.n):
            if p_want[i] > p_want[j] + tau:
                assert pos[i] < pos[j]


@pytest.mark.parametrize("prec,product", [("fp32", "sparse"), ("fp32", "fused"), ("fp32", "dense"),
                                          ("bf16x3", "dense"), ("fp32", "auto")])
def test_mixed_n922_against_fp64_gpu(Q, prec, product):
    g = inputs.ba_digraph(922, 3, seed=0)
    P = Q.Problem.from_graph(g)
    R = O.problem_ref(g.n, g.src, g.dst)
    ref = Q.steady_state(P, 0.8, 0.01, 1e-8, 200000)
    out = Q.steady_state(P, 0.8, 0.01, 1e-8, 200000, prec=prec, product=product)
    a, b = Q.to_complex(out.rho), Q.to_complex(ref.rho)
    assert np.max(np.abs(a - b)) < 1e-6
    res = np.sqrt(np.sum(np.abs(O.rhs_ref(a, R.H_sparse, R.G, R.d, 0.8)) ** 2))
    assert res < 1e-8 * (1 + 1e-6)


def test_lowp_rk4_trajectory_close_to_fp64(Q):
    g = inputs.ba_digraph(200, 3, seed=4)
    P = Q.Problem.from_graph(g)
    rho0 = inputs.random_density(200, seed=9)
    x64 = Q.planar(rho0)
    Q.rk4_step(P, 0.5, 0.01, 30, x64)
    for prec, product in (("fp32", "sparse"), ("fp32", "dense"), ("bf16x3", "dense")):
        x = Q.planar(rho0)
        Q.rk4_step(P, 0.5, 0.01, 30, x, prec=prec, product=product)
        err = (x - x64).abs().max().item()
        assert 0 < err < 1e-7


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_every_dense_tile_configuration(Q, prec):
    """Every tile configuration of the dense product runs the MFMA
    accumulation along k in the same order (and, for BF16x3, the slices in the
    same order), so all configurations of one instruction shape give bitwise
    the same right-hand side (BF16x3 has two: 16 x 16 x 32 and, named _m32_,
    32 x 32 x 16, which sums the products in sixteens); every one matches the
    oracle within the precision's bound.  N = 250 pads to ld = 256, which every
    tile shape divides."""
    g = inputs.ba_digraph(250, 3, seed=21)
    P = Q.Problem.from_graph(g)
    R = O.problem_ref(g.n, g.src, g.dst)
    rho = inputs.random_density(g.n, seed=22)
    want = O.rhs_ref(rho, R.H_sparse, R.G, R.d, 0.4)
    deg = int((R.H != 0).sum(axis=1).max())
    bound = (1e-12 if prec == "fp64" else
             8 * 2.0 ** -24 * (deg + 1) * np.max(np.abs(rho)) * 0.6 + 1e-15)
    names = Q.product_configs(prec)
    outs = []
    for cfg, name in enumerate(names):
        got = Q.to_complex(Q.rhs(P, 0.4, Q.planar(rho), prec=prec, product="dense", gemm_cfg=cfg))
        assert np.max(np.abs(got - want)) <= bound, name
        outs.append(got)
    first = {}
    for name, got in zip(names, outs):
        family = "_m32_" in name
        if family in first:
            assert np.array_equal(got, first[family]), name
        else:
            first[family] = got


@pytest.mark.parametrize("name,n,m", [("ba130", 130, 3), ("ba922", 922, 3)])
def test_fp32_fused_equals_fp32_sparse_bitwise(Q, name, n, m):
    """The fused FP32 stage gathers the FP32 state copy, sums in FP64 in the
    separate FP32 product's order and rounds X once to FP32, alternating its
    two FP32 copies: right-hand side, RK4 steps and the defect-corrected
    steady state are bitwise those of the two-kernel FP32 stage."""
    P = Q.Problem.from_graph(inputs.ba_digraph(n, m, seed=0))
    rho = Q.planar(inputs.random_density(n, seed=23))
    assert torch.equal(Q.rhs(P, 0.6, rho, prec="fp32", product="sparse"),
                       Q.rhs(P, 0.6, rho, prec="fp32", product="fused"))
    xa, xb = rho.clone(), rho.clone()
    Q.rk4_step(P, 0.6, 0.01, 5, xa, prec="fp32", product="sparse")
    Q.rk4_step(P, 0.6, 0.01, 5, xb, prec="fp32", product="fused")
    assert torch.equal(xa, xb)
    tol = 1e-8 if n > 200 else 1e-9
    a = Q.steady_state(P, 0.7, 0.01, tol, 400000, prec="fp32", product="sparse", fold_every=50)
    b = Q.steady_state(P, 0.7, 0.01, tol, 400000, prec="fp32", product="fused", fold_every=50)
    assert torch.equal(a.rho, b.rho)
    assert a.stats["steps"] == b.stats["steps"] and a.stats["folds"] == b.stats["folds"]


@pytest.mark.parametrize("n,m,omega", [(70, 2, 0.3), (130, 3, 0.6), (300, 2, 0.9)])
def test_fp32_defect_state_matches_fp64_defect_state(Q, n, m, omega):
    """The same defect correction with the defect held in FP32 and in FP64:
    both converge to the oracle-measured tolerance, agree within the mixed
    bound, and the FP32-state solve is bitwise Hermitian and trace one."""
    g = inputs.ba_digraph(n, m, seed=n + 1)
    P = Q.Problem.from_graph(g)
    R = O.problem_ref(g.n, g.src, g.dst)
    f = lambda r: O.rhs_ref(r, R.H_sparse, R.G, R.d, omega)
    a = Q.steady_state(P, omega, 0.01, 1e-9, 400000, prec="fp32", delta_state="fp32",
                       product="sparse")
    b = Q.steady_state(P, omega, 0.01, 1e-9, 400000, prec="fp32", delta_state="fp64",
                       product="fused")
    ra, rb = Q.to_complex(a.rho), Q.to_complex(b.rho)
    for r in (ra, rb):
        assert np.sqrt(np.sum(np.abs(f(r)) ** 2)) < 1e-9 * (1 + 1e-6)
    assert np.max(np.abs(ra - rb)) < 1e-6
    assert a.stats["herm_err"] == 0.0 and a.stats["trace_err"] < 1e-12
    assert a.stats["converged"] == 1 and a.stats["folds"] >= 2


def test_fp32_defect_state_option_errors(Q):
    P = Q.Problem.from_graph(inputs.ba_digraph(130, 3, seed=1))
    with pytest.raises(Q.QprError):   # an FP32 defect needs the sparse product
        Q.steady_state(P, 0.5, 0.01, 1e-8, 1000, prec="fp32", product="dense",
                       delta_state="fp32")
    with pytest.raises(Q.QprError):   # and the FP32 product
        Q.steady_state(P, 0.5, 0.01, 1e-8, 1000, prec="bf16x3", delta_state="fp32")
