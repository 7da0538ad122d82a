"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances (FP64 throughout): the right-hand side and stage updates differ
from the oracle only in summation order, |dL| <= ~deg * eps * max|rho|, so
1e-12 absolute on trace-one states; step-locked trajectories stay within
1e-10 (the bound set for plain FP64; observed ~1e-14); integer and
index outputs (CSR, degrees, ranking) are compared exactly.
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


def oracle_problem(g, **kw):
    return O.problem_ref(g.n, g.src, g.dst, **kw)


GRAPHS = {
    "er16": lambda: inputs.er_digraph(16, 0.2, seed=0),
    "er70": lambda: inputs.er_digraph(70, 0.06, seed=3),         # ragged: 70 -> ld 128
    "ba130": lambda: inputs.ba_digraph(130, 3, seed=1),           # several tiles + tail
    "ba300": lambda: inputs.ba_digraph(300, 2, seed=2),
}


# ------------------------------------------------------------------- build
@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("teleport,hdiag", [("paper_f", "zero"), ("uniform", "paper")])
def test_build_matches_oracle(Q, name, teleport, hdiag):
    g = GRAPHS[name]()
    # add a self-loop and a duplicate to exercise the cleaning rules
    src = np.concatenate([g.src, [0, g.src[0]]]).astype(np.int32)
    dst = np.concatenate([g.dst, [0, g.dst[0]]]).astype(np.int32)
    P = Q.Problem(g.n, src, dst, teleport=teleport, hdiag=hdiag)
    R = O.problem_ref(g.n, src, dst, teleport=teleport, hdiag=hdiag)
    n = g.n
    H = P.h_off().cpu().numpy()
    offdiag = R.H - np.diag(np.diag(R.H))
    assert np.array_equal(H[:n, :n], offdiag)
    assert np.all(H[n:, :] == 0) and np.all(H[:, n:] == 0)
    assert np.array_equal(P.vector("h_diag").cpu().numpy(), np.diag(R.H))
    # the oracle sums each column of G in float64: its own error is ~n eps
    assert np.max(np.abs(P.vector("d").cpu().numpy() - R.d)) < 2 * n * np.finfo(float).eps
    assert np.array_equal(P.vector("outdeg").cpu().numpy(), O.out_degree(R.A).astype(np.int32))
    assert np.array_equal(P.vector("indeg").cpu().numpy(), R.A.sum(axis=1).astype(np.int32))
    assert np.array_equal(P.vector("dangling").cpu().numpy(), (O.out_degree(R.A) == 0).astype(np.int32))
    ptr = P.vector("in_ptr").cpu().numpy()
    idx = P.vector("in_idx").cpu().numpy()
    for a in range(n):
        assert list(idx[ptr[a]:ptr[a + 1]]) == list(np.nonzero(R.A[a])[0])
    assert P.p.n_self_loops == 1
    assert P.p.nnz_a == int(R.A.sum())
    assert P.p.nnz_h == int(np.count_nonzero(offdiag))
    pr = P.vector("pagerank").cpu().numpy()
    assert np.max(np.abs(pr - O.pagerank_power(R.G))) < 1e-13
    lam = np.linalg.eigvalsh(R.H)
    assert P.p.h_lo <= lam[0] + 1e-12 and lam[-1] <= P.p.h_hi + 1e-12


# --------------------------------------------------------------------- rhs
@pytest.mark.parametrize("product", ["dense", "sparse", "fused", "blocksparse"])
@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("omega", [0.0, 0.35, 0.8, 1.0])
def test_rhs_fp64_matches_oracle(Q, name, omega, product):
    g = GRAPHS[name]()
    for teleport, hdiag in (("paper_f", "zero"), ("uniform", "paper")):
        P = Q.Problem.from_graph(g, teleport=teleport, hdiag=hdiag)
        R = oracle_problem(g, teleport=teleport, hdiag=hdiag)
        rho = inputs.random_density(g.n, seed=g.n)
        got = Q.to_complex(Q.rhs(P, omega, Q.planar(rho), product=product))
        want = O.rhs_ref(rho, R.H, R.G, R.d, omega)
        assert np.max(np.abs(got - want)) < 1e-12 * max(1.0, np.max(np.abs(want)))
        assert np.array_equal(got, got.conj().T)          # bitwise Hermitian


# -------------------------------------------------------------- RK4 steps
@pytest.mark.parametrize("product", ["dense", "sparse", "fused", "blocksparse"])
@pytest.mark.parametrize("name,steps", [("er16", 60), ("er70", 25), ("ba130", 12)])
def test_rk4_steps_step_locked(Q, name, steps, product):
    g = GRAPHS[name]()
    P = Q.Problem.from_graph(g)
    R = oracle_problem(g)
    omega, dt = 0.8, 0.01
    rho0 = inputs.random_density(g.n, seed=5)
    x = Q.planar(rho0)
    d = Q.rk4_step(P, omega, dt, steps, x, diag=True, product=product)
    got = Q.to_complex(x)
    want = O.rk4_ref(rho0, lambda r: O.rhs_ref(r, R.H, R.G, R.d, omega), dt, steps)
    assert np.max(np.abs(got - want)) < 1e-12
    dd = d.cpu().numpy()
    assert abs(dd[1] - np.trace(want).real) < 1e-12
    assert dd[2] == 0.0 and dd[3] == 0.0


# ---------------------------------------------------------- steady state
@pytest.mark.parametrize("product", ["dense", "sparse", "fused"])
def test_steady_state_er16_matches_oracle(Q, product):
    g = GRAPHS["er16"]()
    P = Q.Problem.from_graph(g)
    R = oracle_problem(g)
    omega, dt, tol = 0.8, 0.01, 1e-10
    f = lambda r: O.rhs_ref(r, R.H, R.G, R.d, omega)
    want, nsteps, res = O.steady_ref(np.eye(16) / 16, f, dt, tol, 100000)
    out = Q.steady_state(P, omega, dt, tol, 100000, product=product)
    got = Q.to_complex(out.rho)
    assert out.stats["steps"] == nsteps
    assert out.stats["converged"] == 1
    assert np.max(np.abs(got - want)) < 1e-10
    assert abs(out.stats["residual"] - res) < 1e-13
    assert out.stats["herm_err"] == 0.0
    assert list(out.rank.cpu().numpy()) == list(O.rank_ref(np.diag(want).real))


@pytest.mark.parametrize("chunk,use_graph", [(7, False), (64, True), (5, True)])
def test_steady_state_graph_and_chunking_do_not_change_result(Q, chunk, use_graph):
    g = GRAPHS["er70"]()
    P = Q.Problem.from_graph(g)
    ref = Q.steady_state(P, 0.5, 0.01, 1e-9, 100000, chunk=64, use_graph=False)
    out = Q.steady_state(P, 0.5, 0.01, 1e-9, 100000, chunk=chunk, use_graph=use_graph)
    assert out.stats["steps"] == ref.stats["steps"]
    assert torch.equal(out.rho, ref.rho)


@pytest.mark.parametrize("product", ["dense", "sparse", "fused", "blocksparse"])
def test_steady_state_ba130_properties_and_oracle(Q, product):
    g = GRAPHS["ba130"]()
    P = Q.Problem.from_graph(g)
    R = oracle_problem(g)
    omega, dt, tol = 0.6, 0.01, 1e-9
    f = lambda r: O.rhs_ref(r, R.H, R.G, R.d, omega)
    want, nsteps, _ = O.steady_ref(np.eye(g.n) / g.n, f, dt, tol, 100000)
    out = Q.steady_state(P, omega, dt, tol, 100000, product=product)
    got = Q.to_complex(out.rho)
    assert out.stats["steps"] == nsteps
    assert np.max(np.abs(got - want)) < 1e-10
    assert np.sqrt(np.sum(np.abs(f(got)) ** 2)) < tol
    assert np.min(np.linalg.eigvalsh(got)) > -1e-12


def test_not_converged_returns_last_state(Q):
    g = GRAPHS["er16"]()
    P = Q.Problem.from_graph(g)
    R = oracle_problem(g)
    out = Q.steady_state(P, 0.8, 0.01, 1e-14, 37, allow_not_converged=True)
    assert out.status == Q.QPR_E_NOT_CONVERGED
    assert out.stats["steps"] == 37
    want = O.rk4_ref(np.eye(16) / 16, lambda r: O.rhs_ref(r, R.H, R.G, R.d, 0.8), 0.01, 37)
    assert np.max(np.abs(Q.to_complex(out.rho) - want)) < 1e-13


def test_error_paths(Q):
    g = GRAPHS["er16"]()
    P = Q.Problem.from_graph(g)
    rho = Q.planar(np.eye(16) / 16)
    with pytest.raises(Q.QprError) as e:
        Q.rhs(P, 1.5, rho)
    assert e.value.status == Q.QPR_E_ARG and "omega" in e.value.message
    with pytest.raises(Q.QprError) as e:
        Q.rk4_step(P, 0.1, 5.0, 1, rho)
    assert e.value.status == Q.QPR_E_UNSTABLE
    bad = rho.clone()
    bad[0, 3, 3] = float("nan")
    with pytest.raises(Q.QprError) as e:
        Q.steady_state(P, 0.8, 0.01, 1e-10, 1000, rho0=bad)
    assert e.value.status == Q.QPR_E_NONFINITE
    with pytest.raises(Q.QprError) as e:
        Q.Problem(4, [0, 1], [1, 9])
    assert e.value.status == Q.QPR_E_ARG


# ------------------------------------------------------ Fehlberg RKF45
@pytest.mark.parametrize("product", ["dense", "sparse", "fused", "blocksparse"])
def test_rkf45_attempts_match_oracle(Q, product):
    """The first attempts of the adaptive Fehlberg integration: same accepted
    and rejected counts and the same state as the oracle's RKF45."""
    g = GRAPHS["ba130"]()
    P = Q.Problem.from_graph(g)
    R = oracle_problem(g)
    omega, h0, tol_step, hmax = 0.7, 0.01, 1e-5, 0.25
    f = lambda r: O.rhs_ref(r, R.H, R.G, R.d, omega)
    attempts = 25
    y, t, acc, rej = O.rkf45_ref(np.eye(g.n) / g.n, f, h0, tol_step, tol_ss=1e-14,
                                 max_steps=attempts, h_max=hmax, raise_on_limit=False)
    out = Q.steady_state(P, omega, h0, 1e-14, attempts, integrator="rkf45", step_tol=tol_step,
                         dt_max=hmax, product=product, allow_not_converged=True, chunk=7)
    assert out.stats["steps"] == acc and out.stats["rejected"] == rej
    assert abs(out.stats["t"] - t) < 1e-12
    assert np.max(np.abs(Q.to_complex(out.rho) - y)) < 1e-12


def test_rkf45_steady_state_matches_rk4_fixed_point(Q):
    """RKF45 and RK4 share the fixed point L(rho) = 0; the adaptive run needs
    far fewer steps."""
    g = GRAPHS["ba300"]()
    P = Q.Problem.from_graph(g)
    R = oracle_problem(g)
    omega, tol = 0.5, 1e-10
    rk4 = Q.steady_state(P, omega, 0.01, tol, 400000)
    rkf = Q.steady_state(P, omega, 0.01, tol, 400000, integrator="rkf45", step_tol=1e-4)
    a, b = Q.to_complex(rkf.rho), Q.to_complex(rk4.rho)
    f = lambda r: O.rhs_ref(r, R.H_sparse, R.G, R.d, omega)
    assert np.sqrt(np.sum(np.abs(f(a)) ** 2)) < tol * (1 + 1e-6)
    assert np.max(np.abs(a - b)) < 1e-9
    assert rkf.stats["steps"] < rk4.stats["steps"] / 4
    assert rkf.stats["herm_err"] == 0.0
    # rankings agree on every pair whose populations differ by more than
    # twice the distance between the two states (closer pairs are ties)
    p = np.diag(b).real
    tau = 2 * np.max(np.abs(a - b))
    pos_f = np.empty(g.n, dtype=int)
    pos_f[rkf.rank.cpu().numpy()] = np.arange(g.n)
    order = rk4.rank.cpu().numpy()
    for i in range(g.n - 1):
        u, v = order[i], order[i + 1]
        if p[u] - p[v] > tau:
            assert pos_f[u] < pos_f[v]


def test_spectral_radius_estimate(Q):
    """h_norm is the power-iteration estimate of rho(H) (a lower bound);
    [h_lo, h_hi] must contain the whole spectrum (rigorous), and with the
    Collatz-Wielandt bound it is close to +-rho(H) even on hub graphs whose
    Gershgorin interval is twice the largest degree wide."""
    for g in (GRAPHS["ba300"](), inputs.ba_digraph(922, 3, seed=0), _hub_and_isolated(),
              inputs.er_digraph(200, 0.01, seed=5)):
        for hdiag in ("zero", "paper"):
            P = Q.Problem.from_graph(g, hdiag=hdiag)
            R = oracle_problem(g, hdiag=hdiag)
            ev = np.linalg.eigvalsh(R.H)
            rho = np.max(np.abs(ev))
            assert 0.97 * rho <= P.p.h_norm <= rho * (1 + 1e-9)
            assert P.p.h_lo <= ev[0] + 1e-12 and ev[-1] <= P.p.h_hi + 1e-12
            if g.n >= 300:      # connected scale-free graphs: the bound is tight
                assert P.p.h_hi - P.p.h_lo <= 2.2 * rho


# ---------------------------------------------------------------- ranking
def test_rank_kernel_with_ties(Q):
    rng = np.random.default_rng(0)
    for n in (1, 7, 256, 1000, 4099):
        p = rng.integers(0, max(2, n // 5), size=n).astype(np.float64) / 7.0  # many ties
        got = Q.rank(torch.from_numpy(p).cuda()).cpu().numpy()
        assert list(got) == list(O.rank_ref(p))


def test_hub_counts_match_oracle(Q):
    rng = np.random.default_rng(1)
    for n in (10, 500, 3000):
        p = rng.dirichlet(np.full(n, 0.3))
        p[:3] = [10.0 / n, 1.0 / n, 10.0 / n + 1e-12]   # boundary values
        got = Q.hub_counts(torch.from_numpy(p).cuda(), 10.0)
        assert got == O.hub_classes_ref(p, 10.0)


# --------------------------------------------------------- full-size cases
@pytest.mark.parametrize("n,m", [(922, 3), (4096, 4)])
def test_rhs_full_size(Q, n, m):
    g = inputs.ba_digraph(n, m, seed=0)
    P = Q.Problem.from_graph(g)
    R = oracle_problem(g)
    rho = inputs.random_density(n, seed=1)
    want = O.rhs_ref(rho, R.H_sparse, R.G, R.d, 0.8)
    for product in ("dense", "sparse", "fused"):
        got = Q.to_complex(Q.rhs(P, 0.8, Q.planar(rho), product=product))
        assert np.max(np.abs(got - want)) < 1e-12 * max(1.0, np.max(np.abs(want)))
    # the H_off pattern the sparse product gathers through
    hp = P.vector("h_ptr").cpu().numpy()
    hi = P.vector("h_idx").cpu().numpy()
    for a in (0, 1, n // 2, n - 1):
        assert list(hi[hp[a]:hp[a + 1]]) == list(np.nonzero(R.H[a] - np.diag(np.diag(R.H))[a])[0])


def _hub_and_isolated(n=200):
    """Node 0 linked to nodes 1..n-11 (a 189-neighbour row: many full groups of
    eight plus a ragged one), a chain 1 -> 2 -> ... -> n-11 and ten isolated
    nodes (empty rows)."""
    src = [0] * (n - 11) + list(range(1, n - 11))
    dst = list(range(1, n - 10)) + list(range(2, n - 10))
    return inputs.Graph(n, np.asarray(src, np.int32), np.asarray(dst, np.int32))


@pytest.mark.parametrize("name", ["er70", "ba130", "hub_isolated", "ba922"])
def test_sparse_variants_bitwise_equal(Q, name):
    """Every sparse-product kernel variant sums each row in the same order, so
    the right-hand side is bitwise the same; it matches the oracle."""
    g = (_hub_and_isolated() if name == "hub_isolated" else
         inputs.ba_digraph(922, 3, seed=0) if name == "ba922" else GRAPHS[name]())
    P = Q.Problem.from_graph(g)
    R = oracle_problem(g)
    rho = inputs.random_density(g.n, seed=11)
    outs = [Q.to_complex(Q.rhs(P, 0.5, Q.planar(rho), product="sparse", sparse_variant=v))
            for v in range(len(Q.SPARSE_VARIANTS))]
    for v in range(1, len(outs)):
        assert np.array_equal(outs[0], outs[v]), Q.SPARSE_VARIANTS[v]
    want = O.rhs_ref(rho, R.H_sparse, R.G, R.d, 0.5)
    assert np.max(np.abs(outs[0] - want)) < 1e-12 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("name", ["hub_isolated", "ba922"])
def test_fused_epilogue_ragged_rows(Q, name):
    """The fused epilogue's gathers on a 189-entry row, empty rows and a ragged
    last tile: the right-hand side and one RK4 step match the oracle, and the
    result is bitwise Hermitian."""
    g = _hub_and_isolated() if name == "hub_isolated" else inputs.ba_digraph(922, 3, seed=0)
    P = Q.Problem.from_graph(g)
    R = oracle_problem(g)
    rho = inputs.random_density(g.n, seed=13)
    got = Q.to_complex(Q.rhs(P, 0.4, Q.planar(rho), product="fused"))
    want = O.rhs_ref(rho, R.H_sparse, R.G, R.d, 0.4)
    assert np.max(np.abs(got - want)) < 1e-12 * max(1.0, np.max(np.abs(want)))
    assert np.array_equal(got, got.conj().T)
    x = Q.planar(rho)
    Q.rk4_step(P, 0.4, 0.01, 1, x, product="fused")
    want1 = O.rk4_ref(rho, lambda r: O.rhs_ref(r, R.H_sparse, R.G, R.d, 0.4), 0.01, 1)
    assert np.max(np.abs(Q.to_complex(x) - want1)) < 1e-12


@pytest.mark.parametrize("name", ["er70", "ba130", "hub_isolated", "ba922"])
def test_fused_equals_sparse_bitwise(Q, name):
    """The fused epilogue sums each gathered row in the separate sparse
    product's order, so the right-hand side, RK4 steps and RKF45 attempts are
    bitwise those of the two-kernel stage."""
    g = (_hub_and_isolated() if name == "hub_isolated" else
         inputs.ba_digraph(922, 3, seed=0) if name == "ba922" else GRAPHS[name]())
    P = Q.Problem.from_graph(g)
    rho = Q.planar(inputs.random_density(g.n, seed=17))
    a = Q.rhs(P, 0.45, rho, product="sparse")
    b = Q.rhs(P, 0.45, rho, product="fused")
    assert torch.equal(a, b)
    xa, xb = rho.clone(), rho.clone()
    Q.rk4_step(P, 0.45, 0.01, 3, xa, product="sparse")
    Q.rk4_step(P, 0.45, 0.01, 3, xb, product="fused")
    assert torch.equal(xa, xb)
    ra = Q.steady_state(P, 0.7, 0.01, 1e-14, 20, integrator="rkf45", product="sparse",
                        allow_not_converged=True, chunk=7)
    rb = Q.steady_state(P, 0.7, 0.01, 1e-14, 20, integrator="rkf45", product="fused",
                        allow_not_converged=True, chunk=7)
    assert torch.equal(ra.rho, rb.rho) and ra.stats["steps"] == rb.stats["steps"]


def test_sparse_variant_out_of_range(Q):
    g = GRAPHS["er16"]()
    P = Q.Problem.from_graph(g)
    rho = Q.planar(inputs.random_density(g.n, seed=1))
    with pytest.raises(Q.QprError):
        Q.rhs(P, 0.5, rho, product="sparse", sparse_variant=len(Q.SPARSE_VARIANTS))


@pytest.mark.parametrize("omega", [0.2, 0.5, 0.8])
def test_steady_state_n922_properties(Q, omega):
    """Config-2 graph at each omega of the workload to 1e-8: residual
    re-measured by the oracle, trace, Hermiticity, positivity, the ranking
    rule, and a step-locked prefix against the oracle's RK4."""
    g = inputs.ba_digraph(922, 3, seed=0)
    P = Q.Problem.from_graph(g)
    R = oracle_problem(g)
    out = Q.steady_state(P, omega, 0.01, 1e-8, 200000)
    rho = Q.to_complex(out.rho)
    res = np.sqrt(np.sum(np.abs(O.rhs_ref(rho, R.H_sparse, R.G, R.d, omega)) ** 2))
    assert res < 1e-8 * (1 + 1e-6)
    assert abs(np.trace(rho).real - 1) < 1e-11
    assert np.array_equal(rho, rho.conj().T)
    assert np.min(np.linalg.eigvalsh(rho)) > -1e-12
    assert np.array_equal(out.rank.cpu().numpy(), O.rank_ref(np.diag(rho).real))
    x = Q.planar(np.eye(922) / 922)
    Q.rk4_step(P, omega, 0.01, 8, x)
    want = O.rk4_ref(np.eye(922) / 922, lambda r: O.rhs_ref(r, R.H_sparse, R.G, R.d, omega),
                     0.01, 8)
    assert np.max(np.abs(Q.to_complex(x) - want)) < 1e-12


@pytest.mark.parametrize("product", ["sparse", "fused", "dense", "blocksparse"])
def test_permutation_equivariance(Q, product):
    """Relabelling the nodes permutes everything: L(P rho P^T) = P L(rho) P^T
    for the relabelled graph, the steady state is the permuted one and the
    ranking is the relabelled ranking (distinct populations here)."""
    g = GRAPHS["ba130"]()
    perm = np.random.default_rng(7).permutation(g.n)
    gp = g.relabel(perm)
    P1, P2 = Q.Problem.from_graph(g), Q.Problem.from_graph(gp)
    rho = inputs.random_density(g.n, seed=31)
    rho_p = np.empty_like(rho)
    rho_p[np.ix_(perm, perm)] = rho                      # rho_p[perm[a], perm[b]] = rho[a, b]
    l1 = Q.to_complex(Q.rhs(P1, 0.6, Q.planar(rho), product=product))
    l2 = Q.to_complex(Q.rhs(P2, 0.6, Q.planar(rho_p), product=product))
    assert np.max(np.abs(l2[np.ix_(perm, perm)] - l1)) < 1e-12
    a = Q.steady_state(P1, 0.6, 0.01, 1e-10, 200000, product=product)
    b = Q.steady_state(P2, 0.6, 0.01, 1e-10, 200000, product=product)
    ra, rb = Q.to_complex(a.rho), Q.to_complex(b.rho)
    assert np.max(np.abs(rb[np.ix_(perm, perm)] - ra)) < 1e-9
    pa = np.diag(ra).real
    if np.min(np.abs(np.diff(np.sort(pa)))) > 1e-8:       # no near-ties
        assert list(b.rank.cpu().numpy()) == list(perm[a.rank.cpu().numpy()])


@pytest.mark.parametrize("product,prec", [("sparse", "fp64"), ("fused", "fp64"),
                                          ("dense", "fp64"), ("fused", "fp32"), ("auto", "fp32")])
def test_runs_are_bitwise_reproducible(Q, product, prec):
    """Fixed-order reductions, no atomics on values: the same solve twice gives
    the same bits (state, steps, residual)."""
    P = Q.Problem.from_graph(GRAPHS["ba130"]())
    a = Q.steady_state(P, 0.45, 0.01, 1e-9, 200000, prec=prec, product=product)
    b = Q.steady_state(P, 0.45, 0.01, 1e-9, 200000, prec=prec, product=product)
    assert torch.equal(a.rho, b.rho) and torch.equal(a.rank, b.rank)
    assert a.stats["steps"] == b.stats["steps"] and a.stats["residual"] == b.stats["residual"]


def _hub_graph_or(name):
    return (_hub_and_isolated() if name == "hub_isolated" else
            inputs.ba_digraph(922, 3, seed=0) if name == "ba922" else
            inputs.ba_digraph(1000, 4, seed=2) if name == "ba1000" else GRAPHS[name]())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["er16", "er70", "ba130", "hub_isolated", "ba922", "ba1000"])
def test_blocksparse_equals_dense(Q, name, prec):
    """The tile-skipping product multiplies only the k-slabs in which a 32-row
    block of H_off has a nonzero; the slabs it skips would only add exact
    zeros, so the right-hand side and RK4 steps equal the dense product's
    (graphs with empty rows, a 189-entry row, ragged tiles, ld = 960 and
    1024 (32 x 64 and 32 x 128 tiles))."""
    g = _hub_graph_or(name)
    P = Q.Problem.from_graph(g)
    rho = Q.planar(inputs.random_density(g.n, seed=41))
    a = Q.rhs(P, 0.55, rho, prec=prec, product="dense")
    b = Q.rhs(P, 0.55, rho, prec=prec, product="blocksparse")
    assert torch.equal(a, b)
    xa, xb = rho.clone(), rho.clone()
    Q.rk4_step(P, 0.55, 0.01, 3, xa, prec=prec, product="dense")
    Q.rk4_step(P, 0.55, 0.01, 3, xb, prec=prec, product="blocksparse")
    assert torch.equal(xa, xb)


def test_blocksparse_rejections(Q):
    P = Q.Problem.from_graph(GRAPHS["ba130"]())
    rho = Q.planar(inputs.random_density(130, seed=2))
    with pytest.raises(Q.QprError):
        Q.rhs(P, 0.5, rho, prec="bf16x3", product="blocksparse")
    with pytest.raises(Q.QprError):
        Q.batch_solve([(P, 0.5)], product="blocksparse", mode="persistent")
