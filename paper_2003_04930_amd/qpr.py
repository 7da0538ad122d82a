"""Python binding of libqpr (ctypes).  Argument marshalling only.

Every numerical step runs in the HIP library; PyTorch supplies device memory
(problem arenas, workspaces, density matrices) and the current stream.  The
library is loaded on first use and a missing library raises
:class:`QprError` -- there is no CPU fallback.

Density matrices are planar float64 tensors of shape (2, n, n) on the GPU:
``rho[0] = Re rho``, ``rho[1] = Im rho`` (row-major, rho_ab = <a|rho|b>).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqpr.so")

QPR_OK, QPR_E_ARG, QPR_E_HIP, QPR_E_NOT_CONVERGED = 0, -1, -2, -3
QPR_E_NONFINITE, QPR_E_UNSTABLE, QPR_E_WORKSPACE = -4, -5, -6
STATUS_NAMES = {0: "QPR_OK", -1: "QPR_E_ARG", -2: "QPR_E_HIP", -3: "QPR_E_NOT_CONVERGED",
                -4: "QPR_E_NONFINITE", -5: "QPR_E_UNSTABLE", -6: "QPR_E_WORKSPACE"}
TELEPORT = {"paper_f": 0, "uniform": 1}
HDIAG = {"zero": 0, "paper": 1}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
PRODUCT = {"auto": 0, "dense": 1, "sparse": 2, "fused": 3, "blocksparse": 4}
INTEGRATOR = {"rk4": 0, "rkf45": 1}

# every symbol include/qpr.h declares
EXPORTS = (
    "qpr_problem_bytes", "qpr_build_google", "qpr_workspace_bytes", "qpr_rhs",
    "qpr_rk4_step", "qpr_steady_state", "qpr_steady_state_many", "qpr_rank", "qpr_last_error",
    "qpr_version",
    "qpr_time_kernels", "qpr_product_configs", "qpr_product_config_name",
    "qpr_mpnn_param_count", "qpr_mpnn_workspace_bytes", "qpr_mpnn_features",
    "qpr_mpnn_forward", "qpr_mpnn_backward", "qpr_mpnn_adam", "qpr_autotune",
    "qpr_load_tuning", "qpr_batch_workspace_bytes", "qpr_batch_solve", "qpr_hub_counts",
    "qpr_sparse_variants", "qpr_sparse_variant_name", "qpr_rk4_step_noalloc",
)


class QprError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class qpr_problem(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("ld", C.c_int32), ("n_edges_in", C.c_int64), ("nnz_a", C.c_int64),
        ("nnz_h", C.c_int64), ("n_self_loops", C.c_int32), ("n_dangling", C.c_int32),
        ("alpha", C.c_double), ("teleport", C.c_int32), ("hdiag", C.c_int32),
        ("h_lo", C.c_double), ("h_hi", C.c_double), ("h_norm", C.c_double),
        ("pagerank_iters", C.c_int32),
        ("reserved", C.c_int32),
        ("h_off", C.c_void_p), ("h_off_f32", C.c_void_p), ("h_off_bf16", C.c_void_p),
        ("h_diag", C.c_void_p), ("d", C.c_void_p), ("inv_outdeg", C.c_void_p),
        ("dangling", C.c_void_p), ("outdeg", C.c_void_p), ("indeg", C.c_void_p),
        ("in_ptr", C.c_void_p), ("in_idx", C.c_void_p), ("out_ptr", C.c_void_p),
        ("out_idx", C.c_void_p), ("pagerank", C.c_void_p), ("h_ptr", C.c_void_p),
        ("h_idx", C.c_void_p), ("arena", C.c_void_p),
        ("arena_bytes", C.c_size_t),
    ]


class qpr_stats(C.Structure):
    _fields_ = [
        ("steps", C.c_int64), ("rhs_evals", C.c_int64), ("rhs_evals_fp64", C.c_int64),
        ("folds", C.c_int64), ("t", C.c_double), ("residual", C.c_double),
        ("trace_err", C.c_double), ("herm_err", C.c_double), ("min_diag", C.c_double),
        ("seconds", C.c_double), ("converged", C.c_int32), ("status", C.c_int32),
        ("rejected", C.c_int64), ("last_step", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class qpr_mpnn_batch(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_graphs", C.c_int32), ("x", C.c_void_p),
                ("in_ptr", C.c_void_p), ("in_idx", C.c_void_p), ("out_ptr", C.c_void_p),
                ("out_idx", C.c_void_p), ("inv_in", C.c_void_p), ("inv_out", C.c_void_p),
                ("graph_ptr", C.c_void_p)]


class qpr_opts(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("use_graph", C.c_int32), ("fold_every", C.c_int32),
                ("renorm", C.c_int32), ("gemm_cfg", C.c_int32), ("product", C.c_int32),
                ("integrator", C.c_int32), ("sparse_variant", C.c_int32),
                ("batch_mode", C.c_int32), ("batch_workers", C.c_int32), ("step_tol", C.c_double),
                ("dt_max", C.c_double), ("delta_state", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def lib():
    """Load libqpr.so (raises QprError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise QprError(QPR_E_HIP, f"{LIB_PATH} is missing; build it with "
                                  "`python -m paper_2003_04930_amd.build`")
    # torch first: the library then binds to the HIP runtime torch loaded (the
    # one that owns the device memory and streams passed in), not to a second
    # copy found on the library path
    _torch()
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    P = C.POINTER(qpr_problem)
    sig = {
        "qpr_problem_bytes": (sz, [i32, i64]),
        "qpr_build_google": (i32, [i32, i64, vp, vp, dbl, i32, i32, vp, sz, P, vp]),
        "qpr_workspace_bytes": (sz, [i32, i32, i32]),
        "qpr_rhs": (i32, [P, dbl, vp, vp, i32, C.POINTER(qpr_opts), vp, sz, vp]),
        "qpr_rk4_step": (i32, [P, dbl, dbl, i32, vp, i32, vp, C.POINTER(qpr_opts), vp, sz, vp]),
        "qpr_rk4_step_noalloc": (i32, [P, dbl, dbl, i32, vp, i32, vp, C.POINTER(qpr_opts), vp]),
        "qpr_steady_state": (i32, [P, dbl, dbl, dbl, i64, i32, vp, vp, C.POINTER(qpr_stats),
                                   C.POINTER(qpr_opts), vp, sz, vp]),
        "qpr_steady_state_many": (i32, [i32, vp, vp, dbl, dbl, i64, i32, vp, vp,
                                        C.POINTER(qpr_stats), C.POINTER(qpr_opts), i32, vp, vp,
                                        vp]),
        "qpr_rank": (i32, [i32, vp, vp, vp]),
        "qpr_hub_counts": (i32, [i32, vp, dbl, vp, vp]),
        "qpr_time_kernels": (i32, [P, dbl, i32, i32, i32, vp, C.POINTER(C.c_double), vp, sz, vp]),
        "qpr_product_configs": (i32, [i32]),
        "qpr_autotune": (i32, [P, i32, i32, C.c_char_p, C.POINTER(i32), C.POINTER(C.c_double), vp,
                               sz, vp]),
        "qpr_load_tuning": (i32, [C.c_char_p]),
        "qpr_batch_workspace_bytes": (sz, [i32, vp, i32, C.POINTER(qpr_opts)]),
        "qpr_batch_solve": (i32, [i32, vp, vp, dbl, dbl, i64, i32, vp, vp, C.POINTER(qpr_stats),
                                  C.POINTER(qpr_opts), C.POINTER(i32), C.c_char_p, vp, sz, vp]),
        "qpr_product_config_name": (C.c_char_p, [i32, i32]),
        "qpr_sparse_variants": (i32, []),
        "qpr_sparse_variant_name": (C.c_char_p, [i32]),
        "qpr_mpnn_param_count": (i32, []),
        "qpr_mpnn_workspace_bytes": (sz, [i32, i32]),
        "qpr_mpnn_features": (i32, [P, dbl, vp, vp, vp, vp]),
        "qpr_mpnn_forward": (i32, [C.POINTER(qpr_mpnn_batch), vp, vp, vp, sz, vp]),
        "qpr_mpnn_backward": (i32, [C.POINTER(qpr_mpnn_batch), vp, vp, vp, vp, vp, sz, vp]),
        "qpr_mpnn_adam": (i32, [vp, vp, vp, vp, i32, i32, C.c_float, C.c_float, C.c_float,
                                C.c_float, vp]),
        "qpr_last_error": (C.c_char_p, []),
        "qpr_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int, allow=()):
    if status != QPR_OK and status not in allow:
        raise QprError(status, lib().qpr_last_error().decode())
    return status


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def version() -> str:
    return lib().qpr_version().decode()


# ------------------------------------------------------------------ problem
class Problem:
    """A built problem (qpr_build_google) owning its device arena."""

    def __init__(self, n, src, dst, alpha=0.85, teleport="paper_f", hdiag="zero", device="cuda"):
        torch = _torch()
        L = lib()
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        if src.shape != dst.shape:
            raise ValueError("src and dst must have the same length")
        nbytes = L.qpr_problem_bytes(int(n), int(src.size))
        if nbytes == 0:
            raise QprError(QPR_E_ARG, f"invalid problem size n={n}, E={src.size}")
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.arena.data_ptr()) % 256
        self._base = self.arena.data_ptr() + off
        self.p = qpr_problem()
        _check(L.qpr_build_google(int(n), int(src.size), src.ctypes.data_as(C.c_void_p),
                                  dst.ctypes.data_as(C.c_void_p), float(alpha),
                                  TELEPORT[teleport], HDIAG[hdiag], C.c_void_p(self._base),
                                  nbytes, C.byref(self.p), _stream()))
        self.alpha, self.teleport, self.hdiag = alpha, teleport, hdiag

    @classmethod
    def from_graph(cls, g, **kw):
        return cls(g.n, g.src, g.dst, **kw)

    @property
    def n(self):
        return self.p.n

    @property
    def ld(self):
        return self.p.ld

    def _view(self, ptr, count, dtype):
        torch = _torch()
        item = torch.empty((), dtype=dtype).element_size()
        off = ptr - self.arena.data_ptr()
        return self.arena[off:off + count * item].view(dtype)

    def h_off(self):
        torch = _torch()
        return self._view(self.p.h_off, self.ld * self.ld, torch.float64).view(self.ld, self.ld)

    def vector(self, name):
        torch = _torch()
        if name in ("h_diag", "d", "inv_outdeg", "pagerank"):
            return self._view(getattr(self.p, name), self.n, torch.float64)
        if name in ("dangling", "outdeg", "indeg"):
            return self._view(getattr(self.p, name), self.n, torch.int32)
        if name in ("in_ptr", "out_ptr", "h_ptr"):
            return self._view(getattr(self.p, name), self.n + 1, torch.int32)
        if name == "h_idx":
            return self._view(self.p.h_idx, self.p.nnz_h, torch.int32)
        if name in ("in_idx", "out_idx"):
            return self._view(getattr(self.p, name), self.p.nnz_a, torch.int32)
        raise KeyError(name)


def workspace_bytes(n, prec="fp64", integrator="rk4"):
    nbytes = lib().qpr_workspace_bytes(int(n), PREC[prec], INTEGRATOR[integrator])
    if nbytes == 0:
        raise QprError(QPR_E_ARG, f"invalid workspace request n={n} prec={prec} "
                                  f"integrator={integrator}")
    return nbytes


class Workspace:
    """Device workspace of at least `nbytes` bytes (256-byte aligned)."""

    def __init__(self, nbytes, device="cuda"):
        torch = _torch()
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self.ptr = self.buf.data_ptr() + (-self.buf.data_ptr()) % 256
        self.nbytes = nbytes


_ws_cache = {}


def workspace(n, prec="fp64", integrator="rk4"):
    """The workspace of (prec, current stream), grown when a call needs more.
    Calls on one stream run in order and share it (a larger buffer serves any
    smaller problem); each other stream gets its own, so solves on concurrent
    streams never share scratch memory.  A buffer that is replaced goes back
    to torch's stream-ordered allocator, so work still queued on the stream
    finishes with it before its memory is reused."""
    need = workspace_bytes(n, prec, integrator)
    key = (prec, _stream().value)
    ws = _ws_cache.get(key)
    if ws is None or ws.nbytes < need:
        _ws_cache.pop(key, None)
        ws = _ws_cache[key] = Workspace(need)
    return ws


# ----------------------------------------------------------- conversions
def planar(rho, device="cuda"):
    """complex numpy/torch (n,n) -> planar float64 (2,n,n) device tensor."""
    torch = _torch()
    if isinstance(rho, np.ndarray):
        rho = torch.from_numpy(np.ascontiguousarray(rho, dtype=np.complex128))
    if rho.is_complex():
        out = torch.stack([rho.real, rho.imag]).to(torch.float64)
    else:
        out = rho.to(torch.float64)
    return out.to(device).contiguous()


def to_complex(rho_planar) -> np.ndarray:
    r = rho_planar.detach().cpu().numpy()
    return r[0] + 1j * r[1]


def _planar_arg(rho, n):
    torch = _torch()
    if not (isinstance(rho, torch.Tensor) and rho.dtype == torch.float64 and rho.is_cuda
            and rho.is_contiguous() and tuple(rho.shape) == (2, n, n)):
        raise ValueError(f"rho must be a contiguous float64 CUDA tensor of shape (2,{n},{n})")
    return rho


# --------------------------------------------------------------- entry points


def sparse_variants():
    """Names of the sparse-product kernel variants (index v: sparse_variant=v)."""
    L = lib()
    return [L.qpr_sparse_variant_name(v).decode() for v in range(L.qpr_sparse_variants())]


def __getattr__(name):
    if name == "SPARSE_VARIANTS":
        return tuple(sparse_variants())
    raise AttributeError(name)


BATCH_MODE = {"auto": 0, "persistent": 1, "concurrent": 2}


DELTA_STATE = {"auto": 0, "fp64": 1, "fp32": 2}


def make_opts(chunk=64, use_graph=True, fold_every=0, renorm=1, gemm_cfg=-1, product="auto",
              integrator="rk4", step_tol=1e-4, dt_max=0.0, sparse_variant=-1, batch_mode="auto",
              batch_workers=0, delta_state="auto"):
    return qpr_opts(int(chunk), int(bool(use_graph)), int(fold_every), int(renorm),
                    int(gemm_cfg), PRODUCT[product], INTEGRATOR[integrator],
                    int(sparse_variant) + 1, BATCH_MODE[batch_mode], int(batch_workers),
                    float(step_tol), float(dt_max), DELTA_STATE[delta_state], 0)


def rhs(P: Problem, omega, rho, prec="fp64", out=None, product="auto", gemm_cfg=-1,
        sparse_variant=-1):
    torch = _torch()
    rho = _planar_arg(rho, P.n)
    if out is None:
        out = torch.empty_like(rho)
    ws = workspace(P.n, prec)
    op = make_opts(gemm_cfg=gemm_cfg, product=product, sparse_variant=sparse_variant)
    _check(lib().qpr_rhs(C.byref(P.p), float(omega), _ptr(rho), _ptr(out), PREC[prec],
                         C.byref(op), C.c_void_p(ws.ptr), ws.nbytes, _stream()))
    return out


def rk4_step(P: Problem, omega, dt, nsteps, rho, prec="fp64", diag=False, product="auto",
             gemm_cfg=-1):
    """nsteps RK4 steps in place; returns [res^2, trace, herm, nonfinite] if diag."""
    torch = _torch()
    rho = _planar_arg(rho, P.n)
    ws = workspace(P.n, prec)
    d = torch.zeros(4, dtype=torch.float64, device=rho.device) if diag else None
    op = make_opts(gemm_cfg=gemm_cfg, product=product)
    _check(lib().qpr_rk4_step(C.byref(P.p), float(omega), float(dt), int(nsteps), _ptr(rho),
                              PREC[prec], _ptr(d), C.byref(op), C.c_void_p(ws.ptr), ws.nbytes,
                              _stream()))
    return d


def rk4_step_noalloc(P: Problem, omega, dt, nsteps, rho, diag=None, product="auto"):
    """qpr_rk4_step_noalloc: nsteps FP64 RK4 steps in place, the workspace in the
    library's static device array (n <= 1024).  `diag`, if given, is a device
    float64 tensor of 4 that receives [res^2, trace, herm, nonfinite]."""
    rho = _planar_arg(rho, P.n)
    op = make_opts(product=product)
    _check(lib().qpr_rk4_step_noalloc(C.byref(P.p), float(omega), float(dt), int(nsteps),
                                      _ptr(rho), PREC["fp64"], _ptr(diag), C.byref(op),
                                      _stream()))
    return diag


@dataclass
class SolveResult:
    rho: "object"
    rank: "object"
    stats: dict
    status: int


def steady_state(P: Problem, omega, dt=0.01, tol=1e-8, max_steps=200000, prec="fp64", rho0=None,
                 want_rank=True, chunk=64, use_graph=True, fold_every=0, renorm=1, gemm_cfg=-1,
                 allow_not_converged=False, product="auto", integrator="rk4", step_tol=1e-4,
                 dt_max=0.0, delta_state="auto"):
    torch = _torch()
    n = P.n
    if rho0 is None:
        rho = torch.zeros((2, n, n), dtype=torch.float64, device="cuda")
        rho[0].diagonal().fill_(1.0 / n)
    else:
        rho = _planar_arg(rho0, n).clone()
    rank = torch.empty(n, dtype=torch.int32, device="cuda") if want_rank else None
    st = qpr_stats()
    op = make_opts(chunk, use_graph, fold_every, renorm, gemm_cfg, product, integrator, step_tol,
                   dt_max, delta_state=delta_state)
    ws = workspace(n, prec, integrator)
    status = lib().qpr_steady_state(C.byref(P.p), float(omega), float(dt), float(tol),
                                    int(max_steps), PREC[prec], _ptr(rho), _ptr(rank),
                                    C.byref(st), C.byref(op), C.c_void_p(ws.ptr), ws.nbytes,
                                    _stream())
    _check(status, allow=(QPR_E_NOT_CONVERGED,) if allow_not_converged else ())
    return SolveResult(rho, rank, st.as_dict(), status)


_stream_pool = []


def _pool_streams(k):
    """The first k streams of a pool kept for the life of the process (their
    cached workspaces are reused from call to call)."""
    torch = _torch()
    while len(_stream_pool) < k:
        _stream_pool.append(torch.cuda.Stream())
    return _stream_pool[:k]


def steady_state_many(items, dt=0.01, tol=1e-8, max_steps=200000, prec="fp64", rho0s=None,
                      want_rank=True, chunk=64, use_graph=True, fold_every=0, renorm=1,
                      gemm_cfg=-1, allow_not_converged=False, product="auto", integrator="rk4",
                      step_tol=1e-4, dt_max=0.0, workers=8, delta_state="auto"):
    """Solve [(Problem, omega), ...] concurrently with qpr_steady_state_many: a
    pool of min(workers, len(items)) host threads, each with its own stream and
    workspace; each result is bitwise what steady_state returns."""
    torch = _torch()
    k = len(items)
    nw = max(1, min(int(workers), k))
    streams = _pool_streams(nw)
    cur = torch.cuda.current_stream()
    rhos, ranks = [], []
    for i, (P, _) in enumerate(items):
        if rho0s is None or rho0s[i] is None:
            r = torch.zeros((2, P.n, P.n), dtype=torch.float64, device="cuda")
            r[0].diagonal().fill_(1.0 / P.n)
        else:
            r = _planar_arg(rho0s[i], P.n).clone()
        rhos.append(r)
        ranks.append(torch.empty(P.n, dtype=torch.int32, device="cuda") if want_rank else None)
    nmax = max(P.n for P, _ in items)
    wss = []
    for s in streams:
        with torch.cuda.stream(s):
            wss.append(workspace(nmax, prec, integrator))
        s.wait_stream(cur)   # the initial states are written on the current stream
    op = make_opts(chunk, use_graph, fold_every, renorm, gemm_cfg, product, integrator, step_tol,
                   dt_max, delta_state=delta_state)
    probs = (C.POINTER(qpr_problem) * k)(*[C.pointer(P.p) for P, _ in items])
    omegas = (C.c_double * k)(*[float(w) for _, w in items])
    rho_ptrs = (C.c_void_p * k)(*[r.data_ptr() for r in rhos])
    rank_ptrs = (C.c_void_p * k)(*[(r.data_ptr() if r is not None else None) for r in ranks])
    ws_ptrs = (C.c_void_p * nw)(*[w.ptr for w in wss])
    ws_bytes = (C.c_size_t * nw)(*[w.nbytes for w in wss])
    handles = (C.c_void_p * nw)(*[s.cuda_stream for s in streams])
    stats = (qpr_stats * k)()
    status = lib().qpr_steady_state_many(k, probs, omegas, float(dt), float(tol), int(max_steps),
                                         PREC[prec], rho_ptrs, rank_ptrs, stats, C.byref(op), nw,
                                         ws_ptrs, ws_bytes, handles)
    _check(status, allow=(QPR_E_NOT_CONVERGED,) if allow_not_converged else ())
    return [SolveResult(r, rk, st.as_dict(), st.status) for r, rk, st in zip(rhos, ranks, stats)]


def hub_counts(p, c=10.0):
    """(main hubs, secondary hubs) of the populations p, counted on the GPU."""
    torch = _torch()
    p = p.to(torch.float64).contiguous()
    out = torch.zeros(2, dtype=torch.int32, device=p.device)
    _check(lib().qpr_hub_counts(int(p.numel()), _ptr(p), float(c), _ptr(out), _stream()))
    a, b = out.cpu().tolist()
    return int(a), int(b)


def rank(p):
    """Order of nodes by descending p (ties: ascending index), on the GPU."""
    torch = _torch()
    p = p.to(torch.float64).contiguous()
    order = torch.empty(p.numel(), dtype=torch.int32, device=p.device)
    _check(lib().qpr_rank(int(p.numel()), _ptr(p), _ptr(order), _stream()))
    return order


def time_kernels(P: Problem, omega, rho, prec="fp64", cfg=-1, reps=50):
    """Mean ms per launch of (product, RK4-stage epilogue over the four stages), timed with HIP
    events; cfg -2 / -3 - v pick the sparse product (see qpr_time_kernels)."""
    rho = _planar_arg(rho, P.n)
    ws = workspace(P.n, prec)
    out = (C.c_double * 2)()
    _check(lib().qpr_time_kernels(C.byref(P.p), float(omega), PREC[prec], int(cfg), int(reps),
                                  _ptr(rho), out, C.c_void_p(ws.ptr), ws.nbytes, _stream()))
    return float(out[0]), float(out[1])


def product_configs(prec="fp64"):
    L = lib()
    return [L.qpr_product_config_name(PREC[prec], i).decode()
            for i in range(L.qpr_product_configs(PREC[prec]))]


# ------------------------------------------------------- learned warm start
def mpnn_param_count() -> int:
    return int(lib().qpr_mpnn_param_count())


class MpnnBatch:
    """Block-diagonal batch of (problem, omega) pairs for the warm-start network.

    Features come from qpr_mpnn_features on each built problem; the CSR
    arrays are the problems' own in/out link lists shifted by node offsets.
    """

    def __init__(self, items):
        torch = _torch()
        xs, ii, oo, ip, ix, op, ox, offs = [], [], [], [], [], [], [], [0]
        base = nnz_in = nnz_out = 0
        for P, omega in items:
            n = P.n
            x = torch.empty((n, 4), dtype=torch.float32, device="cuda")
            inv_in = torch.empty(n, dtype=torch.float32, device="cuda")
            inv_out = torch.empty(n, dtype=torch.float32, device="cuda")
            _check(lib().qpr_mpnn_features(C.byref(P.p), float(omega), _ptr(x), _ptr(inv_in),
                                           _ptr(inv_out), _stream()))
            xs.append(x)
            ii.append(inv_in)
            oo.append(inv_out)
            ip.append(P.vector("in_ptr")[:-1].to(torch.int64) + nnz_in)
            ix.append(P.vector("in_idx").to(torch.int64) + base)
            op.append(P.vector("out_ptr")[:-1].to(torch.int64) + nnz_out)
            ox.append(P.vector("out_idx").to(torch.int64) + base)
            nnz_in += int(P.p.nnz_a)
            nnz_out += int(P.p.nnz_a)
            base += n
            offs.append(base)
        nnz = sum(int(t.numel()) for t in ix)
        i32 = torch.int32
        self.x = torch.cat(xs).contiguous()
        self.inv_in = torch.cat(ii).contiguous()
        self.inv_out = torch.cat(oo).contiguous()
        self.in_ptr = torch.cat(ip + [torch.tensor([nnz], device="cuda")]).to(i32).contiguous()
        self.in_idx = torch.cat(ix).to(i32).contiguous() if nnz else torch.zeros(1, dtype=i32, device="cuda")
        self.out_ptr = torch.cat(op + [torch.tensor([nnz], device="cuda")]).to(i32).contiguous()
        self.out_idx = torch.cat(ox).to(i32).contiguous() if nnz else torch.zeros(1, dtype=i32, device="cuda")
        self.graph_ptr = torch.tensor(offs, dtype=i32, device="cuda")
        self.n_nodes, self.n_graphs = base, len(items)
        self.c = qpr_mpnn_batch(self.n_nodes, self.n_graphs, self.x.data_ptr(),
                                self.in_ptr.data_ptr(), self.in_idx.data_ptr(),
                                self.out_ptr.data_ptr(), self.out_idx.data_ptr(),
                                self.inv_in.data_ptr(), self.inv_out.data_ptr(),
                                self.graph_ptr.data_ptr())
        nbytes = lib().qpr_mpnn_workspace_bytes(self.n_nodes, self.n_graphs)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        self.ws_ptr = self.ws.data_ptr() + (-self.ws.data_ptr()) % 256
        self.ws_bytes = nbytes


def mpnn_forward(batch: MpnnBatch, params):
    torch = _torch()
    p_hat = torch.empty(batch.n_nodes, dtype=torch.float32, device="cuda")
    _check(lib().qpr_mpnn_forward(C.byref(batch.c), _ptr(params), _ptr(p_hat),
                                  C.c_void_p(batch.ws_ptr), batch.ws_bytes, _stream()))
    return p_hat


def mpnn_backward(batch: MpnnBatch, params, p_true):
    """Gradient and loss after mpnn_forward on the same batch."""
    torch = _torch()
    grads = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(lib().qpr_mpnn_backward(C.byref(batch.c), _ptr(params), _ptr(p_true), _ptr(grads),
                                   _ptr(loss), C.c_void_p(batch.ws_ptr), batch.ws_bytes,
                                   _stream()))
    return grads, loss


def mpnn_adam(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    _check(lib().qpr_mpnn_adam(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), int(params.numel()),
                               int(step), float(lr), float(b1), float(b2), float(eps), _stream()))


def autotune(P: Problem, prec="fp64", reps=20, cache_path=None):
    """Time every dense-product tile configuration; returns (best_cfg, {name: us})."""
    ws = workspace(P.n, prec)
    L = lib()
    ncfg = L.qpr_product_configs(PREC[prec])
    us = (C.c_double * ncfg)()
    best = C.c_int32(-1)
    path = cache_path.encode() if cache_path else None
    _check(L.qpr_autotune(C.byref(P.p), PREC[prec], int(reps), path, C.byref(best), us,
                          C.c_void_p(ws.ptr), ws.nbytes, _stream()))
    names = product_configs(prec)
    return int(best.value), {names[i]: float(us[i]) for i in range(ncfg)}


def load_tuning(cache_path):
    _check(lib().qpr_load_tuning(cache_path.encode()))


@dataclass
class BatchResult:
    rhos: list
    ranks: list
    stats: list
    status: int
    tuned_cfg: int
    seconds: float


def batch_solve(items, dt=0.01, tol=1e-8, max_steps=400000, prec="fp64", rho0s=None,
                want_rank=True, chunk=0, use_graph=True, gemm_cfg=-1, product="auto",
                allow_not_converged=False, integrator="rk4", step_tol=1e-4, dt_max=0.0,
                mode="auto", workers=0, delta_state="auto", tune_cache=None):
    """Solve [(Problem, omega), ...] together with qpr_batch_solve (mode "auto" or
    "concurrent": a pool of worker streams; "persistent": shared launches).
    chunk 0 takes the library's default for the mode."""
    torch = _torch()
    import time as _time
    nsys = len(items)
    ns = (C.c_int32 * nsys)(*[P.n for P, _ in items])
    op = make_opts(chunk, use_graph, 0, 1, gemm_cfg, product, integrator, step_tol, dt_max,
                   batch_mode=mode, batch_workers=workers, delta_state=delta_state)
    nbytes = lib().qpr_batch_workspace_bytes(nsys, ns, PREC[prec], C.byref(op))
    if nbytes == 0:
        raise QprError(QPR_E_ARG, "invalid batch request")
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr() + (-buf.data_ptr()) % 256
    rhos, ranks = [], []
    for k, (P, _) in enumerate(items):
        if rho0s is None or rho0s[k] is None:
            r = torch.zeros((2, P.n, P.n), dtype=torch.float64, device="cuda")
            r[0].diagonal().fill_(1.0 / P.n)
        else:
            r = _planar_arg(rho0s[k], P.n).clone()
        rhos.append(r)
        ranks.append(torch.empty(P.n, dtype=torch.int32, device="cuda") if want_rank else None)
    probs = (C.POINTER(qpr_problem) * nsys)(*[C.pointer(P.p) for P, _ in items])
    omegas = (C.c_double * nsys)(*[float(w) for _, w in items])
    rho_ptrs = (C.c_void_p * nsys)(*[r.data_ptr() for r in rhos])
    rank_ptrs = (C.c_void_p * nsys)(*[(r.data_ptr() if r is not None else None) for r in ranks])
    stats = (qpr_stats * nsys)()
    tuned = C.c_int32(-1)
    t0 = _time.perf_counter()
    status = lib().qpr_batch_solve(nsys, probs, omegas, float(dt), float(tol), int(max_steps),
                                   PREC[prec], rho_ptrs, rank_ptrs, stats, C.byref(op),
                                   C.byref(tuned), tune_cache.encode() if tune_cache else None,
                                   C.c_void_p(base), nbytes, _stream())
    secs = _time.perf_counter() - t0
    _check(status, allow=(QPR_E_NOT_CONVERGED,) if allow_not_converged else ())
    return BatchResult(rhos, ranks, [s.as_dict() for s in stats], status, int(tuned.value), secs)
