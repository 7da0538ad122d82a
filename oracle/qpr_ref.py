"""Plain FP64 reference for the quantum-PageRank steady state.

TEST INFRASTRUCTURE ONLY (see the package docstring): no product code imports
this module.

Model (Tang et al., arXiv:2003.04930, Supplementary Note 1 and Eq. (1)):

    d rho/dt = -(1-omega) i [H, rho]
               + omega * sum_k ( L_k rho L_k^dag - 1/2 {L_k^dag L_k, rho} )

with the adjacency A (A_ij = 1 when j links to i), the Hamiltonian H of
Eq. (S6), the Google matrix G of Eq. (S4) built from the transition matrix and
the long-distance hopping matrix F of Eq. (S2), and one jump operator
L_ij = sqrt(G_ij) |i><j| per ordered pair (i, j).

Readings of garbled or silent passages (each applied where named):

* R-anticommutator  Eq. (1)/(S7) print L_k L_k^dag in the left half of the
  anticommutator but Eq. (2)/(S8) imply L_k^dag L_k; the literal form does not
  preserve the trace, so the standard GKSL form -1/2 {L^dag L, rho} is used.
* R-vec             Eq. (2) prints L^dag (x) L for the gain term; with the
  column-stacking vec that "rho-tilde is the transpose of rho" describes,
  vec(L rho L^dag) = (conj(L) (x) L) vec(rho), which is what is built.
* R-google          Eq. (S4) mixes the generator M with the stochastic F.
  Read as the usual column-stochastic Google matrix G = alpha S + (1-alpha) T:
  S is the out-degree-normalised adjacency, a node with no out-links
  ("dangling") takes the teleport column T_:j, T defaults to F of Eq. (S2)
  (1/(N-1) off the diagonal, 0 on it) and alpha = 0.85.  T = 1/N everywhere is
  kept as an option ("uniform").  d_j, the column sums of G, are computed, not
  assumed to be one.
* R-jumps           Jump operators sqrt(G_ij) |i><j| for every ordered pair,
  i = j included (those only dephase); the paper leaves K unstated.
* R-hamiltonian     Eq. (S6) gives H_ij = -max(A_ij, A_ji), H_jj = -outDeg(j).
  The default ("zero") is the symmetrised adjacency max(A, A^T) with a zero
  diagonal; "paper" is Eq. (S6) literally.
* R-integrator      The classical four-stage Runge-Kutta step of
  Supplementary Note 2 (the commented RK4 form) with a fixed step h.
* R-stop            The paper integrates to a fixed time; the steady state is
  declared at the first step n with ||L(y_n)||_F < tol (absolute Frobenius
  norm of the right-hand side at the current state) and y_n is returned.
* R-rank            Ranking is by descending population, ties broken by the
  smaller node index.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "adjacency", "out_degree", "teleport_matrix", "google_matrix",
    "hamiltonian", "ProblemRef", "problem_ref", "jump_operators",
    "lindblad_rhs_literal", "rhs_ref", "liouvillian_bruteforce", "vec",
    "unvec", "rk4_step_ref", "rk4_ref", "steady_ref", "pagerank_power",
    "rank_ref", "hub_classes_ref", "rkf45_ref", "FEHLBERG", "steady_null_ref",
]


# ---------------------------------------------------------------- graph model
def adjacency(n: int, src, dst) -> np.ndarray:
    """Dense adjacency of Supplementary Note 1: A[i, j] = 1 iff j links to i.

    Duplicate edges collapse to one; self-loops are dropped.
    """
    A = np.zeros((n, n), dtype=np.float64)
    for s, d in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        if not (0 <= s < n and 0 <= d < n):
            raise ValueError(f"edge ({s}->{d}) out of range for n={n}")
        if s != d:
            A[d, s] = 1.0
    return A


def out_degree(A: np.ndarray) -> np.ndarray:
    """outDeg(j) = sum_i A_ij (Supplementary Note 1)."""
    return A.sum(axis=0)


def teleport_matrix(n: int, kind: str = "paper_f") -> np.ndarray:
    """Long-distance hopping matrix.

    "paper_f": Eq. (S2), F_ij = 1/(N-1) for i != j and 0 on the diagonal.
    "uniform": every entry 1/N (the textbook PageRank teleport).
    """
    if kind == "paper_f":
        T = np.full((n, n), 1.0 / (n - 1))
        np.fill_diagonal(T, 0.0)
        return T
    if kind == "uniform":
        return np.full((n, n), 1.0 / n)
    raise ValueError(f"unknown teleport kind {kind!r}")


def google_matrix(A: np.ndarray, alpha: float = 0.85, teleport: str = "paper_f"):
    """Google matrix G = alpha S + (1 - alpha) T (Eq. (S4), reading R-google).

    Column j of S is A[:, j] / outDeg(j), or T[:, j] when node j has no
    out-links.  Returns (G, d) with d_j = sum_i G_ij as computed.
    """
    n = A.shape[0]
    T = teleport_matrix(n, teleport)
    deg = out_degree(A)
    S = np.empty_like(A)
    for j in range(n):
        S[:, j] = A[:, j] / deg[j] if deg[j] > 0 else T[:, j]
    G = alpha * S + (1.0 - alpha) * T
    d = G.sum(axis=0)
    return G, d


def hamiltonian(A: np.ndarray, hdiag: str = "zero") -> np.ndarray:
    """Hamiltonian of the quantum walk (Eq. (S6), reading R-hamiltonian)."""
    sym = np.maximum(A, A.T)
    np.fill_diagonal(sym, 0.0)
    if hdiag == "zero":
        return sym
    if hdiag == "paper":
        H = -sym
        H[np.diag_indices_from(H)] = -out_degree(A)
        return H
    raise ValueError(f"unknown hdiag mode {hdiag!r}")


class ProblemRef:
    """Everything the right-hand side needs, built once per graph."""

    def __init__(self, A, G, d, H):
        self.A, self.G, self.d, self.H = A, G, d, H
        self.n = A.shape[0]
        self._Hs = None

    @property
    def H_sparse(self):
        if self._Hs is None:
            import scipy.sparse as sp
            self._Hs = sp.csr_matrix(self.H)
        return self._Hs

    def rhs(self, rho, omega):
        return rhs_ref(rho, self.H if self.n <= 256 else self.H_sparse,
                       self.G, self.d, omega)


def problem_ref(n, src, dst, alpha=0.85, teleport="paper_f", hdiag="zero") -> ProblemRef:
    A = adjacency(n, src, dst)
    G, d = google_matrix(A, alpha, teleport)
    return ProblemRef(A, G, d, hamiltonian(A, hdiag))


# ------------------------------------------------------------ right-hand side
def jump_operators(G: np.ndarray):
    """Yield sqrt(G_ij) |i><j| for every ordered pair (reading R-jumps)."""
    n = G.shape[0]
    for i in range(n):
        for j in range(n):
            if G[i, j] != 0.0:
                L = np.zeros((n, n), dtype=np.complex128)
                L[i, j] = np.sqrt(G[i, j])
                yield L


def lindblad_rhs_literal(rho, H, G, omega):
    """Eq. (1) summed term by term over explicit jump matrices (tiny N only).

    Uses the GKSL anticommutator {L^dag L, rho} (reading R-anticommutator).
    """
    rho = np.asarray(rho, dtype=np.complex128)
    out = -1j * (1.0 - omega) * (H @ rho - rho @ H)
    diss = np.zeros_like(rho)
    for L in jump_operators(G):
        Ld = L.conj().T
        LdL = Ld @ L
        diss += L @ rho @ Ld - 0.5 * (LdL @ rho + rho @ LdL)
    return out + omega * diss


def rhs_ref(rho, H, G, d, omega):
    """Right-hand side of Eq. (1) with the jump sum in closed form.

    With L_ij = sqrt(G_ij)|i><j|:  sum L rho L^dag = diag(G . diag(rho)) and
    sum L^dag L = diag(d), d_j = sum_i G_ij, so the dissipator is
    diag(G diag rho) - 1/2 (d_a + d_b) rho_ab.  The commutator is two genuine
    matrix products H rho - rho H.  ``H`` may be dense or scipy-sparse.
    """
    rho = np.asarray(rho, dtype=np.complex128)
    Hrho = H @ rho
    rhoH = (H.T @ rho.T).T          # rho @ H, valid for dense and sparse H
    comm = np.asarray(Hrho - rhoH)
    gain = np.diag(G @ np.diag(rho))
    anti = 0.5 * (d[:, None] + d[None, :]) * rho
    return -1j * (1.0 - omega) * comm + omega * (gain - anti)


def vec(rho):
    """Column-stacking vec, i.e. the rows of rho-tilde = rho^T laid end to end."""
    return np.asarray(rho).reshape(-1, order="F")


def unvec(v, n):
    return np.asarray(v).reshape((n, n), order="F")


def liouvillian_bruteforce(H, G, omega):
    """The N^2 x N^2 Liouvillian of Eq. (2), assembled from Kronecker products.

    Commutator part -i(1-omega)(I (x) H - H^T (x) I) as printed; gain part
    conj(L) (x) L (reading R-vec); anticommutator part
    -1/2 (I (x) L^dag L + L^T conj(L) (x) I) as printed.  O(N^6) work: N <= 8.
    """
    n = H.shape[0]
    eye = np.eye(n)
    Lv = -1j * (1.0 - omega) * (np.kron(eye, H) - np.kron(H.T, eye))
    D = np.zeros((n * n, n * n), dtype=np.complex128)
    for L in jump_operators(G):
        LdL = L.conj().T @ L
        D += np.kron(L.conj(), L) - 0.5 * (np.kron(eye, LdL) + np.kron(L.T @ L.conj(), eye))
    return Lv + omega * D


# ------------------------------------------------------------------ integrator
def rk4_step_ref(y, f, h):
    """One classical RK4 step (Supplementary Note 2, reading R-integrator)."""
    k1 = h * f(y)
    k2 = h * f(y + 0.5 * k1)
    k3 = h * f(y + 0.5 * k2)
    k4 = h * f(y + k3)
    return y + k1 / 6.0 + k2 / 3.0 + k3 / 3.0 + k4 / 6.0


def rk4_ref(y0, f, h, nsteps):
    y = np.array(y0, dtype=np.complex128)
    for _ in range(nsteps):
        y = rk4_step_ref(y, f, h)
    return y


def steady_ref(y0, f, h, tol, max_steps, renorm=False):
    """Integrate with RK4 until ||f(y_n)||_F < tol (reading R-stop).

    Returns (y_n, n, residual_n).  ``renorm`` divides the state by its trace
    after every step.  Raises RuntimeError if max_steps is reached.
    """
    y = np.array(y0, dtype=np.complex128)
    for n in range(max_steps + 1):
        k1 = f(y)
        res = float(np.sqrt(np.sum(np.abs(k1) ** 2)))
        if res < tol:
            return y, n, res
        if n == max_steps:
            break
        k1 = h * k1
        k2 = h * f(y + 0.5 * k1)
        k3 = h * f(y + 0.5 * k2)
        k4 = h * f(y + k3)
        y = y + k1 / 6.0 + k2 / 3.0 + k3 / 3.0 + k4 / 6.0
        if renorm:
            y = y / np.trace(y).real
    raise RuntimeError(f"not converged after {max_steps} steps (residual {res:.3e})")


def steady_null_ref(f, n, tol=1e-13, restart=60, maxiter=2000):
    """The steady state by its definition, without time stepping: the unique
    trace-one rho with L(rho) = 0 (the null vector of the Liouvillian of
    Eq. (2), here applied matrix-free through f = L).

    Write rho = I/n + X with tr X = 0.  L maps every matrix to a traceless one,
    so L(X) = -L(I/n) has its right-hand side in the traceless subspace, on
    which L is invertible when the steady state is unique; GMRES started from
    X = 0 (scipy, no preconditioner) stays in that subspace.  Returns
    (rho, ||L(rho)||_F, iterations).
    """
    import scipy.sparse.linalg as spla
    eye = np.eye(n, dtype=np.complex128) / n
    b = -np.asarray(f(eye)).ravel()
    op = spla.LinearOperator((n * n, n * n), dtype=np.complex128,
                             matvec=lambda x: np.asarray(f(x.reshape(n, n))).ravel())
    its = [0]

    def count(_):
        its[0] += 1
    x, info = spla.gmres(op, b, rtol=tol, atol=0.0, restart=restart, maxiter=maxiter,
                         callback=count, callback_type="pr_norm")
    if info != 0:
        raise RuntimeError(f"GMRES did not converge (info={info})")
    rho = eye + x.reshape(n, n)
    res = float(np.sqrt(np.sum(np.abs(f(rho)) ** 2)))
    return rho, res, its[0]


# ---------------------------------------------------------- classical + ranks
def pagerank_power(G, tol=1e-15, max_iter=100000):
    """Stationary vector of the column-stochastic G by power iteration p <- G p."""
    n = G.shape[0]
    p = np.full(n, 1.0 / n)
    for _ in range(max_iter):
        q = G @ p
        q = q / q.sum()
        if np.abs(q - p).sum() < tol:
            return q
        p = q
    return p


def rank_ref(p):
    """Node order by descending p, ties by ascending index (reading R-rank)."""
    p = np.asarray(p, dtype=np.float64)
    return np.lexsort((np.arange(p.size), -p)).astype(np.int32)


def hub_classes_ref(p, c=10.0):
    """Hub classes of the results section: main hubs p > c/N, secondary hubs
    1/N < p <= c/N.  Returns (n_main, n_secondary)."""
    p = np.asarray(p, dtype=np.float64)
    n = p.size
    main = int(np.sum(p > c / n))
    second = int(np.sum((p > 1.0 / n) & (p <= c / n)))
    return main, second


# ---------------------------------------------------------- Fehlberg RKF45
# Runge-Kutta-Fehlberg 4(5) tableau of Supplementary Note 2, Eqs. (S10)-(S12),
# with the two 4101 denominators read as 4104 (with 4101 the fourth-order
# weights do not sum to one and the fifth stage is inconsistent).
FEHLBERG = {
    "c": (0.0, 1 / 4, 3 / 8, 12 / 13, 1.0, 1 / 2),
    "a": (
        (),
        (1 / 4,),
        (3 / 32, 9 / 32),
        (1932 / 2197, -7200 / 2197, 7296 / 2197),
        (439 / 216, -8.0, 3680 / 513, -845 / 4104),
        (-8 / 27, 2.0, -3544 / 2565, 1859 / 4104, -11 / 40),
    ),
    "b4": (25 / 216, 0.0, 1408 / 2565, 2197 / 4104, -1 / 5, 0.0),
    "b5": (16 / 135, 0.0, 6656 / 12825, 28561 / 56430, -9 / 50, 2 / 55),
}


def rkf45_ref(y0, f, h0, tol_step, t_end=None, tol_ss=None, max_steps=100000,
              h_max=None, raise_on_limit=True):
    """Adaptive Fehlberg 4(5) integration (Supplementary Note 2).

    Step factor s = (tol_step * h / (2 |z - y|))^(1/4) (Eq. (S13)); |.| read as
    the max-abs norm.  A step is accepted when |z - y| <= tol_step * h and the
    fourth-order y is kept.  Stops at t_end, or when tol_ss is given at the
    first accepted state with ||f(y)||_F < tol_ss.  Returns (y, t, accepted,
    rejected); after max_steps attempts it raises, or with raise_on_limit=False
    returns the state reached.
    """
    y = np.array(y0, dtype=np.complex128)
    t, h = 0.0, h0
    acc = rej = 0
    a, b4, b5 = FEHLBERG["a"], FEHLBERG["b4"], FEHLBERG["b5"]
    while acc + rej < max_steps:
        if tol_ss is not None:
            if float(np.sqrt(np.sum(np.abs(f(y)) ** 2))) < tol_ss:
                return y, t, acc, rej
        if t_end is not None:
            if t >= t_end:
                return y, t, acc, rej
            h = min(h, t_end - t)
        k = []
        for s in range(6):
            ys = y.copy()
            for j, coef in enumerate(a[s]):
                ys = ys + coef * k[j]
            k.append(h * f(ys))
        y4 = y + sum(b * kk for b, kk in zip(b4, k))
        y5 = y + sum(b * kk for b, kk in zip(b5, k))
        err = float(np.max(np.abs(y5 - y4)))
        if err <= tol_step * h:
            y, t = y4, t + h
            acc += 1
        else:
            rej += 1
        s_fac = (tol_step * h / (2.0 * err)) ** 0.25 if err > 0 else 4.0
        h = h * min(4.0, max(0.1, s_fac))
        if h_max is not None:
            h = min(h, h_max)
    if raise_on_limit:
        raise RuntimeError("rkf45: step limit reached")
    return y, t, acc, rej
