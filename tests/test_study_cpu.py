"""Host-side post-processing of the PageRank-versus-quantum-PageRank study:
tie classes and lifted ties against brute force on small vectors."""
import itertools

import numpy as np

from paper_2003_04930_amd import study


def _brute_classes(p, tau):
    # connected components of the "within tau" graph on sorted values (a
    # chain: consecutive sorted values within tau are joined)
    s = sorted(p)
    comps, cur = [], [s[0]]
    for a, b in zip(s, s[1:]):
        if b - a <= tau:
            cur.append(b)
        else:
            comps.append(cur)
            cur = [b]
    comps.append(cur)
    big = [c for c in comps if len(c) >= 2]
    return len(big), sum(len(c) for c in big), max(len(c) for c in comps)


def test_tie_classes_against_brute_force():
    rng = np.random.default_rng(3)
    for _ in range(200):
        n = int(rng.integers(1, 30))
        p = rng.integers(0, 12, size=n) / 11.0 + rng.normal(0, 1e-9, size=n)
        tau = float(rng.choice([1e-12, 1e-8, 0.05]))
        if n == 1:
            assert study.tie_classes(p, tau) == (0, 0, 1)
            continue
        assert study.tie_classes(p, tau) == _brute_classes(list(p), tau)


def test_lifted_ties_counts_pairs():
    pc = np.array([0.1, 0.1, 0.1, 0.3, 0.3, 0.2])
    pq = np.array([0.11, 0.11, 0.12, 0.31, 0.35, 0.2])
    pairs, lifted = study.lifted_ties(pc, pq, 1e-12, 1e-3)
    # classical classes {0,1,2} (3 pairs) and {3,4} (1 pair); the quantum
    # values separate (0,2), (1,2) and (3,4)
    assert pairs == 4 and lifted == 3
    want = sum(1 for a, b in itertools.combinations(range(6), 2) if abs(pc[a] - pc[b]) <= 1e-12)
    assert pairs == want
