"""PageRank against quantum PageRank: hub classes and degeneracy.

The results section of the paper classifies nodes by their steady-state
probability p_i against the uniform value 1/N: main hubs p_i > c/N (c = 10)
and secondary hubs 1/N < p_i <= c/N; it reports that the quantum ranking
lifts degeneracies of the classical one (nodes the classical PageRank cannot
tell apart).  This module reports both for the synthetic workload graphs:
hub counts (the library's qpr_hub_counts kernel) for the classical PageRank
vector of G and for diag rho_ss, and tie classes of each ranking.

Tie classes: sort the values; adjacent values closer than tau belong to one
class; a class of two or more nodes is a degeneracy.  The classical vector is
converged to ~1e-15 by power iteration, so its ties are taken at
tau = 1e-12 / N (equal up to rounding); the quantum vector is only known to
the solver's accuracy, so its ties are taken at tau = 2 max|d rho| between two
independent solves (or a given bound), and a classical tie counts as lifted
when the two nodes' quantum values differ by more than that.
"""
from __future__ import annotations

import numpy as np


def tie_classes(p, tau):
    """Classes of nodes whose sorted values chain within tau.  Returns
    (number of classes with >= 2 nodes, nodes in them, largest class)."""
    p = np.asarray(p, dtype=np.float64)
    if p.size < 2:
        return 0, 0, 1 if p.size else 0
    s = np.sort(p)
    close = np.diff(s) <= tau
    classes = nodes = 0
    largest = 1
    run = 1
    for c in close:
        if c:
            run += 1
        else:
            if run >= 2:
                classes += 1
                nodes += run
            largest = max(largest, run)
            run = 1
    if run >= 2:
        classes += 1
        nodes += run
    largest = max(largest, run)
    return int(classes), int(nodes), int(largest)


def lifted_ties(p_classical, p_quantum, tau_c, tau_q):
    """Pairs tied classically (|dp| <= tau_c, chained in sorted order) and how
    many of them the quantum values separate by more than tau_q."""
    p_classical = np.asarray(p_classical, dtype=np.float64)
    p_quantum = np.asarray(p_quantum, dtype=np.float64)
    order = np.argsort(p_classical, kind="stable")
    s = p_classical[order]
    pairs = lifted = 0
    i = 0
    n = s.size
    while i < n:
        j = i
        while j + 1 < n and s[j + 1] - s[j] <= tau_c:
            j += 1
        if j > i:
            members = order[i:j + 1]
            q = p_quantum[members]
            for a in range(len(members)):
                for b in range(a + 1, len(members)):
                    pairs += 1
                    lifted += int(abs(q[a] - q[b]) > tau_q)
        i = j + 1
    return int(pairs), int(lifted)


def hub_study(Q, P, rho, tau_q, c=10.0):
    """Hub classes and degeneracy of PageRank and of diag rho (rho: planar
    (2, n, n) device state) on problem P.  Hub counts come from the library
    (qpr_hub_counts); tie classes from the sorted values."""
    import torch
    n = P.n
    pr = P.vector("pagerank").to(torch.float64)
    pq = rho[0].diagonal().contiguous().to(torch.float64)
    hubs_pr = Q.hub_counts(pr, c)
    hubs_q = Q.hub_counts(pq, c)
    pr_h, pq_h = pr.cpu().numpy(), pq.cpu().numpy()
    tau_c = 1e-12 / n
    pairs, lifted = lifted_ties(pr_h, pq_h, tau_c, tau_q)
    return {
        "n": n, "c": c,
        "pagerank": {"main_hubs": hubs_pr[0], "secondary_hubs": hubs_pr[1],
                     "tie_classes": tie_classes(pr_h, tau_c), "tau": tau_c},
        "quantum": {"main_hubs": hubs_q[0], "secondary_hubs": hubs_q[1],
                    "tie_classes": tie_classes(pq_h, tau_q), "tau": tau_q},
        "classical_tied_pairs": pairs, "lifted_by_quantum": lifted, "tau_classical": tau_c,
        "top10_pagerank": [int(x) for x in np.argsort(-pr_h, kind="stable")[:10]],
        "top10_quantum": [int(x) for x in np.argsort(-pq_h, kind="stable")[:10]],
    }
