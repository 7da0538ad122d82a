"""FP64 reference of the warm-start message-passing network (forward + backward).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no learned component; this network predicts the steady-state
populations diag(rho_ss) so the integrator can start near the answer.  Its
definition (parity unpinned against the paper, which is silent; pinned here by
central finite differences and by invariances in the tests):

  node features  x_i = [log(1+in_i), log(1+out_i), N * PR_i, omega]
  layer l = 0..2 h'_i = ReLU(Ws h_i + Win mean_{j->i} h_j + Wout mean_{i->j} h_j + b)
                 (an empty neighbourhood contributes a zero mean)
  readout        s_i = w . h_i + c,   p_hat = softmax of s over each graph
  loss           mean over graphs of KL(p || p_hat)

in_i / out_i are the in/out degrees of the deduplicated, loop-free adjacency
and PR the power-iteration PageRank of the Google matrix.  Hidden width 64.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = ["MPNN_HIDDEN", "MPNN_LAYERS", "MPNN_FEATS", "mpnn_init_ref",
           "mpnn_graph_ref", "mpnn_forward_ref", "mpnn_backward_ref",
           "mpnn_loss_ref", "adam_ref"]

MPNN_HIDDEN = 64
MPNN_LAYERS = 3
MPNN_FEATS = 4


def mpnn_init_ref(seed=0, hidden=MPNN_HIDDEN):
    """Deterministic parameter dict (for oracle-only tests)."""
    rng = np.random.default_rng(seed)
    p = {}
    fan_in = MPNN_FEATS
    for l in range(MPNN_LAYERS):
        for nm in ("Ws", "Win", "Wout"):
            p[f"{nm}{l}"] = rng.standard_normal((hidden, fan_in)) / np.sqrt(3 * fan_in)
        p[f"b{l}"] = 0.01 * rng.standard_normal(hidden)
        fan_in = hidden
    p["w"] = rng.standard_normal(hidden) / np.sqrt(hidden)
    p["c"] = np.zeros(1)
    return p


def mpnn_graph_ref(A, pr, omega):
    """Mean-aggregation operators and node features of one graph.

    A[i, j] = 1 iff j links to i.  Returns (X, M_in, M_out) with
    (M_in h)_i = mean over j with j->i of h_j and (M_out h)_i = mean over j
    with i->j of h_j.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    indeg = A.sum(axis=1)
    outdeg = A.sum(axis=0)
    inv_in = np.where(indeg > 0, 1.0 / np.maximum(indeg, 1), 0.0)
    inv_out = np.where(outdeg > 0, 1.0 / np.maximum(outdeg, 1), 0.0)
    M_in = sp.csr_matrix(A * inv_in[:, None])
    M_out = sp.csr_matrix(A.T * inv_out[:, None])
    X = np.stack([np.log1p(indeg), np.log1p(outdeg), n * np.asarray(pr),
                  np.full(n, float(omega))], axis=1)
    return X, M_in, M_out


def _segments(seg):
    seg = np.asarray(seg)
    ids = np.unique(seg)
    return [np.nonzero(seg == g)[0] for g in ids]


def mpnn_forward_ref(params, X, M_in, M_out, seg):
    """Forward pass over a block-diagonal batch.  Returns (p_hat, cache)."""
    H = np.asarray(X, dtype=np.float64)
    cache = []
    for l in range(MPNN_LAYERS):
        ai = M_in @ H
        ao = M_out @ H
        Z = H @ params[f"Ws{l}"].T + ai @ params[f"Win{l}"].T + ao @ params[f"Wout{l}"].T + params[f"b{l}"]
        cache.append((H, ai, ao, Z))
        H = np.maximum(Z, 0.0)
    s = H @ params["w"] + params["c"][0]
    p_hat = np.empty_like(s)
    for idx in _segments(seg):
        e = np.exp(s[idx] - s[idx].max())
        p_hat[idx] = e / e.sum()
    cache.append((H, s))
    return p_hat, cache


def mpnn_loss_ref(p_hat, p_true, seg):
    """Mean over graphs of KL(p_true || p_hat) (terms with p_true = 0 vanish)."""
    segs = _segments(seg)
    tot = 0.0
    for idx in segs:
        pt, ph = p_true[idx], p_hat[idx]
        m = pt > 0
        tot += float(np.sum(pt[m] * (np.log(pt[m]) - np.log(ph[m]))))
    return tot / len(segs)


def mpnn_backward_ref(params, cache, p_hat, p_true, M_in, M_out, seg):
    """Analytic gradient of :func:`mpnn_loss_ref` with respect to every parameter."""
    segs = _segments(seg)
    B = len(segs)
    grads = {}
    H_last, _s = cache[-1]
    ds = (p_hat - p_true) / B
    grads["w"] = H_last.T @ ds
    grads["c"] = np.array([ds.sum()])
    dH = np.outer(ds, params["w"])
    for l in reversed(range(MPNN_LAYERS)):
        H, ai, ao, Z = cache[l]
        dZ = dH * (Z > 0)
        grads[f"Ws{l}"] = dZ.T @ H
        grads[f"Win{l}"] = dZ.T @ ai
        grads[f"Wout{l}"] = dZ.T @ ao
        grads[f"b{l}"] = dZ.sum(axis=0)
        dH = dZ @ params[f"Ws{l}"] + M_in.T @ (dZ @ params[f"Win{l}"]) + M_out.T @ (dZ @ params[f"Wout{l}"])
    return grads


def adam_ref(param, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) in place; step counts from 1."""
    m[...] = b1 * m + (1 - b1) * grad
    v[...] = b2 * v + (1 - b2) * grad * grad
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    param[...] = param - lr * mhat / (np.sqrt(vhat) + eps)
