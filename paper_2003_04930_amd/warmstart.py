"""Learned warm start for the steady-state solve.

A message-passing network (kernels in csrc/qpr_mpnn.hip, layout in
include/qpr.h) predicts the steady-state populations p = diag(rho_ss) of a
graph at a given omega from in/out degree, PageRank and omega.  The solve then
starts from rho0 = diag(p_hat) / sum(p_hat); the FP64-judged integrator still
runs to the tolerance, so the prediction only changes how many steps it takes.

Training data are steady states computed by the solver itself; training runs
on the GPU through the library's forward, backward and Adam kernels.  This
module only orchestrates (batching, the step loop, saving weights).
"""
from __future__ import annotations

import sys

import numpy as np

from . import qpr as Q

HID, FEAT = 64, 4


def _torch():
    import torch
    return torch


def init_params(seed: int = 0):
    """Random initial parameters (flat FP32, layout of include/qpr.h)."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    parts = []
    for F in (FEAT, HID, HID):
        for _ in range(3):
            parts.append(rng.standard_normal(HID * F) / np.sqrt(3.0 * F))
        parts.append(np.zeros(HID))
    parts.append(rng.standard_normal(HID) / np.sqrt(HID))
    parts.append(np.zeros(1))
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == Q.mpnn_param_count()
    return torch.tensor(flat, device="cuda")


def solve_targets(items, prec="bf16x3", tol=1e-8, dt=0.01, max_steps=400000):
    """Steady-state populations (FP32 device tensors) of (Problem, omega) items."""
    torch = _torch()
    out = []
    for P, w in items:
        r = Q.steady_state(P, w, dt, tol, max_steps, prec=prec, want_rank=False)
        out.append(r.rho[0].diagonal().to(torch.float32).clone())
    return out


def make_batches(items, targets, batch_graphs, seed=0):
    torch = _torch()
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(items))
    batches = []
    for i in range(0, len(perm), batch_graphs):
        idx = perm[i:i + batch_graphs]
        B = Q.MpnnBatch([items[j] for j in idx])
        pt = torch.cat([targets[j] for j in idx]).contiguous()
        batches.append((B, pt))
    return batches


def train(items, targets, steps=2000, batch_graphs=32, lr=1e-3, seed=0, params=None,
          lr_final=None, log=None):
    """Adam on the mean per-graph KL divergence; returns (params, loss history).

    lr decays geometrically to lr_final (default lr / 10) over the run.
    """
    torch = _torch()
    batches = make_batches(items, targets, batch_graphs, seed)
    if params is None:
        params = init_params(seed)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    lr_final = lr / 10.0 if lr_final is None else lr_final
    decay = (lr_final / lr) ** (1.0 / max(1, steps - 1))
    losses = []
    for step in range(1, steps + 1):
        B, pt = batches[(step - 1) % len(batches)]
        Q.mpnn_forward(B, params)
        grads, loss = Q.mpnn_backward(B, params, pt)
        Q.mpnn_adam(params, grads, m, v, step, lr=lr * decay ** (step - 1))
        losses.append(loss)
        if log and step % log == 0:
            print(f"[warmstart] step {step} loss {loss.item():.4e}", file=sys.stderr, flush=True)
    return params, [float(x) for x in torch.cat(losses).cpu()]


def evaluate(items, targets, params):
    """Mean KL(p || p_hat) over items (no gradient step)."""
    torch = _torch()
    tot = 0.0
    for (P, w), pt in zip(items, targets):
        B = Q.MpnnBatch([(P, w)])
        Q.mpnn_forward(B, params)
        _, loss = Q.mpnn_backward(B, params, pt)
        tot += float(loss.item())
    return tot / max(1, len(items))


def predict(P, omega, params):
    """Predicted populations (float64 device tensor summing to one)."""
    torch = _torch()
    B = Q.MpnnBatch([(P, omega)])
    p = Q.mpnn_forward(B, params).to(torch.float64)
    return p / p.sum()


def blend_weight(omega, integrator="rk4"):
    """Weight lambda(omega) of the predicted populations in the start state.

    A start state diag(p) has no coherences, and [H, diag(p)] != 0 drives
    coherent modes that the dissipator (strength omega) damps slowly, whereas
    I/N commutes with H.  Integrating from rho0 = (1 - l) I/N + l diag(p_ss),
    with the exact steady-state populations p_ss, takes monotonically more RK4
    steps as l grows for omega <= 0.5 and fewer for omega >= 0.65 (BA and ER
    graphs, N = 40-60): below the crossover no population guess, however good,
    beats I/N.  So for RK4 the prediction is used in full above omega = 0.65,
    not at all below 0.45, and blended linearly in between.

    The adaptive RKF45 integrator takes steps near its stability cap, where
    those coherent modes cost more: on 60 validation graphs (seeds 30000+,
    disjoint from the training and test graphs, N log-uniform in [50, 4096])
    the full prediction took 1.067 / 1.025 / 0.957 / 0.887 / 0.826 times the
    accepted steps of I/N at omega = 0.7 / 0.75 / 0.8 / 0.85 / 0.9, and half of
    it 0.970 at 0.8.  So for RKF45 the prediction is used in full from
    omega = 0.8 and not below 0.75.
    """
    if integrator == "rkf45":
        return float(min(1.0, max(0.0, (omega - 0.75) / 0.05)))
    return float(min(1.0, max(0.0, (omega - 0.45) / 0.2)))


def warm_rho0(P, omega, params, blend=True, integrator="rk4"):
    """rho0 = (1 - l) I/N + l diag(p_hat) as a planar (2, n, n) FP64 tensor,
    l = blend_weight(omega, integrator) (l = 1 if blend is False)."""
    torch = _torch()
    lam = blend_weight(omega, integrator) if blend else 1.0
    rho = torch.zeros((2, P.n, P.n), dtype=torch.float64, device="cuda")
    if lam > 0.0:
        p = predict(P, omega, params)
        rho[0].diagonal().copy_(lam * p + (1.0 - lam) / P.n)
    else:
        rho[0].diagonal().fill_(1.0 / P.n)
    return rho


def warm_rho0_batch(items, params, blend=True, integrator="rk4"):
    """warm_rho0 for many (Problem, omega) pairs with one network pass."""
    torch = _torch()
    lams = [blend_weight(w, integrator) if blend else 1.0 for _, w in items]
    need = [k for k, l in enumerate(lams) if l > 0.0]
    preds = {}
    if need:
        B = Q.MpnnBatch([items[k] for k in need])
        p = Q.mpnn_forward(B, params).to(torch.float64)
        offs = B.graph_ptr.cpu().tolist()
        for j, k in enumerate(need):
            seg = p[offs[j]:offs[j + 1]]
            preds[k] = seg / seg.sum()
    out = []
    for k, (P, _) in enumerate(items):
        rho = torch.zeros((2, P.n, P.n), dtype=torch.float64, device="cuda")
        if k in preds:
            rho[0].diagonal().copy_(lams[k] * preds[k] + (1.0 - lams[k]) / P.n)
        else:
            rho[0].diagonal().fill_(1.0 / P.n)
        out.append(rho)
    return out


def pagerank_rho0(P):
    """rho0 = diag(PageRank of G), the classical guess the network is compared with."""
    torch = _torch()
    pr = P.vector("pagerank").to(torch.float64)
    rho = torch.zeros((2, P.n, P.n), dtype=torch.float64, device="cuda")
    rho[0].diagonal().copy_(pr / pr.sum())
    return rho


def save(params, path):
    np.save(path, params.detach().cpu().numpy().astype(np.float32))


def load(path):
    torch = _torch()
    return torch.tensor(np.load(path).astype(np.float32), device="cuda")
