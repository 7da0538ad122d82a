"""Warm-start network kernels (FP32 on the GPU) against the FP64 oracle
(forward, analytic backward, Adam), determinism, and a short training run.

Tolerances: FP32 arithmetic on O(1) activations through three 64-wide layers
gives relative errors ~1e-6..1e-5; predictions are compared at 1e-4 relative
and each gradient block at 1e-3 of its norm (the oracle's own gradient is
pinned to 1e-6 by central differences in test_oracle_mpnn.py).
"""
import numpy as np
import pytest

import oracle as O
from paper_2003_04930_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HID = 64


@pytest.fixture(scope="module")
def Q():
    from paper_2003_04930_amd import qpr
    qpr.lib()
    assert torch.cuda.is_available()
    return qpr


def flat_to_dict(flat):
    """Split the flat parameter vector per the layout in include/qpr.h."""
    flat = np.asarray(flat, dtype=np.float64)
    out, o = {}, 0
    for l, F in enumerate((4, HID, HID)):
        for nm in ("Ws", "Win", "Wout"):
            out[f"{nm}{l}"] = flat[o:o + HID * F].reshape(HID, F)
            o += HID * F
        out[f"b{l}"] = flat[o:o + HID]
        o += HID
    out["w"] = flat[o:o + HID]
    out["c"] = flat[o + HID:o + HID + 1]
    assert o + HID + 1 == flat.size
    return out


def dict_to_flat(d):
    parts = []
    for l in range(3):
        for nm in ("Ws", "Win", "Wout"):
            parts.append(d[f"{nm}{l}"].reshape(-1))
        parts.append(d[f"b{l}"])
    parts += [d["w"], d["c"]]
    return np.concatenate(parts)


def make_items(Q):
    specs = [(inputs.er_digraph(20, 0.2, seed=1), 0.3), (inputs.ba_digraph(35, 2, seed=2), 0.8),
             (inputs.er_digraph(50, 0.08, seed=3), 0.5)]
    items, refs = [], []
    for g, w in specs:
        P = Q.Problem.from_graph(g)
        R = O.problem_ref(g.n, g.src, g.dst)
        items.append((P, w))
        refs.append((R, w))
    return items, refs


def oracle_batch(refs):
    import scipy.sparse as sp
    Xs, Mi, Mo, seg = [], [], [], []
    for gid, (R, w) in enumerate(refs):
        X, M_in, M_out = O.mpnn_graph_ref(R.A, O.pagerank_power(R.G), w)
        Xs.append(X); Mi.append(M_in); Mo.append(M_out)
        seg.append(np.full(R.n, gid))
    return np.vstack(Xs), sp.block_diag(Mi).tocsr(), sp.block_diag(Mo).tocsr(), np.concatenate(seg)


def test_param_count(Q):
    assert Q.mpnn_param_count() == dict_to_flat(O.mpnn_init_ref()).size


def test_forward_backward_adam_match_oracle(Q):
    items, refs = make_items(Q)
    B = Q.MpnnBatch(items)
    X, Mi, Mo, seg = oracle_batch(refs)
    # features agree with the oracle's
    assert np.max(np.abs(B.x.cpu().numpy() - X) / (np.abs(X) + 1e-3)) < 1e-5
    pd = O.mpnn_init_ref(seed=7)
    flat = dict_to_flat(pd)
    params = torch.tensor(flat, dtype=torch.float32, device="cuda")
    ph = Q.mpnn_forward(B, params).cpu().numpy()
    ph_ref, cache = O.mpnn_forward_ref(pd, X, Mi, Mo, seg)
    assert np.max(np.abs(ph - ph_ref) / ph_ref) < 1e-4
    rng = np.random.default_rng(0)
    pt = np.concatenate([rng.dirichlet(np.ones(R.n)) for R, _ in refs])
    grads, loss = Q.mpnn_backward(B, params, torch.tensor(pt, dtype=torch.float32, device="cuda"))
    g_ref = O.mpnn_backward_ref(pd, cache, ph_ref, pt, Mi, Mo, seg)
    assert abs(loss.item() - O.mpnn_loss_ref(ph_ref, pt, seg)) < 1e-5
    g = flat_to_dict(grads.cpu().numpy())
    for k, v in g_ref.items():
        assert np.linalg.norm(g[k] - v) <= 1e-3 * np.linalg.norm(v) + 1e-7, k
    # deterministic: a second backward is bitwise identical
    Q.mpnn_forward(B, params)
    grads2, _ = Q.mpnn_backward(B, params, torch.tensor(pt, dtype=torch.float32, device="cuda"))
    assert torch.equal(grads, grads2)
    # Adam against the textbook update in FP64
    m = torch.zeros_like(params); v = torch.zeros_like(params)
    pr = params.clone()
    Q.mpnn_adam(pr, grads, m, v, 1, lr=1e-2)
    p64 = flat.copy(); m64 = np.zeros_like(p64); v64 = np.zeros_like(p64)
    O.adam_ref(p64, grads.cpu().numpy().astype(np.float64), m64, v64, 1, lr=1e-2)
    assert np.max(np.abs(pr.cpu().numpy() - p64)) < 1e-5


def test_short_training_reduces_loss(Q):
    from paper_2003_04930_amd import warmstart
    graphs = [inputs.batch_graph(k) for k in range(6)]
    items = []
    for g in graphs:
        P = Q.Problem.from_graph(g)
        for w in (0.3, 0.7):
            items.append((P, w))
    targets = warmstart.solve_targets(items, prec="bf16x3", tol=1e-6)
    params, hist = warmstart.train(items, targets, steps=150, batch_graphs=4, lr=3e-3, seed=0)
    assert hist[-1] < 0.5 * hist[0]


def test_trained_weights_gain_over_identity_start(Q):
    """The committed network (trained on 5000 steady states) against rho0 = I/N
    on graphs it never saw: at omega = 0.9 the warm start needs fewer RK4 steps,
    at omega = 0.2 the blended start is I/N itself (no loss), and every solve
    still finishes at the FP64 tolerance at the same steady state."""
    import os
    from paper_2003_04930_amd import warmstart as W
    path = os.path.join(os.path.dirname(W.__file__), "weights", "mpnn_warmstart.npy")
    params = W.load(path)
    assert params.numel() == Q.mpnn_param_count()
    graphs = [inputs.ba_digraph(240, 3, seed=31337), inputs.er_digraph(300, 4.0 / 299, seed=4242)]
    for g in graphs:
        P = Q.Problem.from_graph(g)
        for w in (0.9, 0.2):
            cold = Q.steady_state(P, w, 0.01, 1e-8, 400000)
            rho0 = W.warm_rho0(P, w, params)
            warm = Q.steady_state(P, w, 0.01, 1e-8, 400000, rho0=rho0)
            assert warm.stats["converged"] == 1
            assert float((warm.rho - cold.rho).abs().max()) < 1e-6
            if w == 0.9:
                assert warm.stats["steps"] < cold.stats["steps"], (g, w)
            else:
                assert warm.stats["steps"] == cold.stats["steps"]
    # one batched network pass gives the same start states
    items = [(Q.Problem.from_graph(g), w) for g in graphs for w in (0.9, 0.55)]
    many = W.warm_rho0_batch(items, params)
    for (P, w), r in zip(items, many):
        assert torch.allclose(r, W.warm_rho0(P, w, params), rtol=0, atol=1e-9)


def test_warm_start_gain_on_twenty_unseen_graphs(Q):
    """What the trained network gains, on 20 graphs it never saw (seeds
    20000.., N log-uniform in [50, 1024], ER and BA, the five batch omegas in
    turn), RK4 to 1e-8 in FP64 from I/N, from diag(PageRank) and from the
    omega-blended prediction: where the prediction is used in full (omega >=
    0.7) it needs fewer steps than both other starts on average; at omega <=
    0.3 its start is I/N itself (same steps); every warm solve ends at the
    cold solve's steady state."""
    import os
    from paper_2003_04930_amd import eval_warmstart as E, warmstart as W
    params = W.load(os.path.join(os.path.dirname(W.__file__), "weights", "mpnn_warmstart.npy"))
    items = [(Q.Problem.from_graph(E.test_graph(k, 1024)), inputs.BATCH_OMEGAS[k % 5])
             for k in range(20)]
    cold = Q.batch_solve(items, tol=1e-8)
    pr = Q.batch_solve(items, tol=1e-8, rho0s=[W.pagerank_rho0(P) for P, _ in items])
    warm = Q.batch_solve(items, tol=1e-8, rho0s=W.warm_rho0_batch(items, params))
    ratio_i, ratio_pr = [], []
    for k, (P, w) in enumerate(items):
        sc, sp, sw = (r.stats[k]["steps"] for r in (cold, pr, warm))
        assert warm.stats[k]["converged"] == 1
        assert float((warm.rhos[k] - cold.rhos[k]).abs().max()) < 1e-6
        if w <= 0.3:
            assert sw == sc
        elif w >= 0.7:
            ratio_i.append(sw / sc)
            ratio_pr.append(sw / sp)
    assert len(ratio_i) == 8
    assert np.mean(ratio_i) < 0.97, ratio_i
    assert np.mean(ratio_pr) < 1.0, ratio_pr
