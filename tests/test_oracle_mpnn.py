"""Pins of the FP64 MPNN reference: analytic backward against central finite
differences, invariances of the forward pass, and Adam against its textbook
closed form for a constant gradient."""
import numpy as np
import scipy.sparse as sp

import oracle as O
from paper_2003_04930_amd import inputs


def _batch(seeds=(0, 1), omegas=(0.3, 0.8)):
    Xs, Mi, Mo, seg, pt = [], [], [], [], []
    for g_id, (s, w) in enumerate(zip(seeds, omegas)):
        g = inputs.er_digraph(7 + s, 0.3, seed=s)
        P = O.problem_ref(g.n, g.src, g.dst)
        pr = O.pagerank_power(P.G)
        X, M_in, M_out = O.mpnn_graph_ref(P.A, pr, w)
        Xs.append(X); Mi.append(M_in); Mo.append(M_out)
        seg.append(np.full(g.n, g_id))
        rng = np.random.default_rng(s)
        t = rng.random(g.n) + 0.1
        pt.append(t / t.sum())
    return (np.vstack(Xs), sp.block_diag(Mi).tocsr(), sp.block_diag(Mo).tocsr(),
            np.concatenate(seg), np.concatenate(pt))


def test_backward_matches_central_differences():
    X, Mi, Mo, seg, pt = _batch()
    params = O.mpnn_init_ref(seed=3)
    ph, cache = O.mpnn_forward_ref(params, X, Mi, Mo, seg)
    grads = O.mpnn_backward_ref(params, cache, ph, pt, Mi, Mo, seg)
    rng = np.random.default_rng(0)
    eps = 1e-6
    for name, val in params.items():
        flat = val.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = O.mpnn_loss_ref(O.mpnn_forward_ref(params, X, Mi, Mo, seg)[0], pt, seg)
            flat[idx] = old - eps
            lm = O.mpnn_loss_ref(O.mpnn_forward_ref(params, X, Mi, Mo, seg)[0], pt, seg)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = grads[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (name, idx, fd, an)


def test_forward_is_a_distribution_per_graph_and_permutation_equivariant():
    g = inputs.ba_digraph(20, 2, seed=2)
    P = O.problem_ref(g.n, g.src, g.dst)
    pr = O.pagerank_power(P.G)
    X, Mi, Mo = O.mpnn_graph_ref(P.A, pr, 0.5)
    params = O.mpnn_init_ref(seed=1)
    seg = np.zeros(g.n, dtype=int)
    ph, _ = O.mpnn_forward_ref(params, X, Mi, Mo, seg)
    assert abs(ph.sum() - 1) < 1e-14 and np.all(ph > 0)
    perm = np.random.default_rng(0).permutation(g.n)
    gp = g.relabel(perm)
    Pp = O.problem_ref(gp.n, gp.src, gp.dst)
    Xp, Mip, Mop = O.mpnn_graph_ref(Pp.A, O.pagerank_power(Pp.G), 0.5)
    php, _ = O.mpnn_forward_ref(params, Xp, Mip, Mop, seg)
    assert np.max(np.abs(php[perm] - ph)) < 1e-13


def test_adam_constant_gradient_closed_form():
    # with a constant gradient g, mhat = g and vhat = g^2 exactly, so every
    # step moves the parameter by lr * g / (|g| + eps)
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -0.25])
    m = np.zeros(2); v = np.zeros(2)
    for t in range(1, 6):
        O.adam_ref(p, g, m, v, t, lr=0.01)
    want = np.array([1.0, -2.0]) - 5 * 0.01 * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(p - want)) < 1e-12
