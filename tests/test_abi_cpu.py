"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, the ctypes structs match the C layout, and argument checks
that precede any device work return the documented status codes."""
import ctypes as C
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from paper_2003_04930_amd import qpr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qpr.h")


def _lib():
    if not os.path.exists(qpr.LIB_PATH):
        pytest.fail("libqpr.so is not built (run __graft_entry__.build())")
    return qpr.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qpr_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = _lib()
    names = declared_functions()
    assert "qpr_steady_state" in names and len(names) >= 9
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(qpr.EXPORTS)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "lay.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "qpr.h"
int main(void){
  printf("%zu %zu %zu\n", sizeof(qpr_problem), sizeof(qpr_stats), sizeof(qpr_opts));
  printf("%zu %zu %zu\n", offsetof(qpr_problem, h_off), offsetof(qpr_problem, pagerank), offsetof(qpr_problem, arena_bytes));
  printf("%zu %zu\n", offsetof(qpr_stats, seconds), offsetof(qpr_stats, status));
  return 0;
}''')
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    got = [int(x) for x in out]
    want = [C.sizeof(qpr.qpr_problem), C.sizeof(qpr.qpr_stats), C.sizeof(qpr.qpr_opts),
            qpr.qpr_problem.h_off.offset, qpr.qpr_problem.pagerank.offset,
            qpr.qpr_problem.arena_bytes.offset, qpr.qpr_stats.seconds.offset,
            qpr.qpr_stats.status.offset]
    assert got == want


def test_size_queries_and_version():
    L = _lib()
    assert L.qpr_problem_bytes(1, 0) == 0
    b922 = L.qpr_problem_bytes(922, 3031)
    assert b922 > 960 * 960 * (8 + 4 + 2)
    assert L.qpr_workspace_bytes(1, 0, 0) == 0
    assert L.qpr_workspace_bytes(922, 7, 0) == 0
    assert L.qpr_workspace_bytes(922, 0, 9) == 0        # unknown integrator
    assert L.qpr_workspace_bytes(922, 1, 1) == 0        # RKF45 is FP64 only
    w64 = L.qpr_workspace_bytes(922, 0, 0)
    packed = (30 * 31 // 2) * 2 * 32 * 32 * 8   # one Hermitian-packed tile-pair array
    assert w64 >= 8 * 960 * 960 * 8 + packed   # y_n, two stage states, X; accumulator packed
    assert w64 < 10 * 960 * 960 * 8
    rkf = L.qpr_workspace_bytes(922, 0, 1)
    assert rkf >= w64 + 2 * 960 * 960 * 8 + 5 * packed   # + candidate, packed K_1..K_5
    assert L.qpr_workspace_bytes(922, 2, 0) >= 14 * 960 * 960 * 8
    assert b"gfx950" in L.qpr_version()


def _build(n, src, dst, alpha=0.85, teleport=0, hdiag=0, arena=C.c_void_p(256), nbytes=1 << 40):
    L = _lib()
    src = np.asarray(src, dtype=np.int32)
    dst = np.asarray(dst, dtype=np.int32)
    P = qpr.qpr_problem()
    return L.qpr_build_google(n, src.size, src.ctypes.data_as(C.c_void_p),
                              dst.ctypes.data_as(C.c_void_p), alpha, teleport, hdiag, arena,
                              nbytes, C.byref(P), None)


@pytest.mark.parametrize("kw,needle", [
    (dict(n=1, src=[], dst=[]), "n must be"),
    (dict(n=4, src=[0], dst=[1], alpha=1.5), "alpha"),
    (dict(n=4, src=[0], dst=[1], teleport=7), "teleport"),
    (dict(n=4, src=[0], dst=[1], hdiag=3), "hdiag"),
    (dict(n=4, src=[0, 5], dst=[1, 2]), "out of range"),
    (dict(n=4, src=[0], dst=[-1]), "out of range"),
    (dict(n=4, src=[0], dst=[1], arena=C.c_void_p(0)), "NULL"),
    (dict(n=4, src=[0], dst=[1], arena=C.c_void_p(8)), "aligned"),
])
def test_build_argument_errors(kw, needle):
    assert _build(**kw) == qpr.QPR_E_ARG
    assert needle in _lib().qpr_last_error().decode()


def test_build_arena_too_small():
    assert _build(4, [0], [1], nbytes=16) == qpr.QPR_E_WORKSPACE


def test_solver_argument_errors_before_device_work():
    L = _lib()
    st = qpr.qpr_stats()
    assert L.qpr_rhs(None, 0.5, None, None, 0, None, None, 0, None) == qpr.QPR_E_ARG
    assert L.qpr_steady_state(None, 0.5, 0.01, 1e-8, 10, 0, None, None, C.byref(st), None, None,
                              0, None) == qpr.QPR_E_ARG
    assert L.qpr_rank(0, None, None, None) == qpr.QPR_E_ARG
    # a fake problem with bad ld is rejected before any HIP call
    P = qpr.qpr_problem()
    P.n, P.ld = 10, 10
    assert L.qpr_rk4_step(C.byref(P), 0.5, 0.01, 1, C.c_void_p(256), 0, None, None,
                          C.c_void_p(256), 1 << 30, None) == qpr.QPR_E_ARG
    assert "built problem" in L.qpr_last_error().decode()


def test_concurrent_solve_argument_errors_before_device_work():
    L = _lib()
    two = lambda t: (t * 2)()
    probs, omegas = two(C.c_void_p), (C.c_double * 2)(0.5, 0.5)
    rhos, ws, wsb = two(C.c_void_p), two(C.c_void_p), (C.c_size_t * 2)(1, 1)
    head = (0.01, 1e-8, 10, 0, rhos, None, None, None)
    many = L.qpr_steady_state_many
    assert many(0, probs, omegas, *head, 2, ws, wsb, two(C.c_void_p)) == qpr.QPR_E_ARG
    assert many(2, probs, omegas, *head, 0, ws, wsb, two(C.c_void_p)) == qpr.QPR_E_ARG
    assert many(2, probs, omegas, *head, 65, ws, wsb, two(C.c_void_p)) == qpr.QPR_E_ARG
    assert many(2, None, omegas, *head, 2, ws, wsb, two(C.c_void_p)) == qpr.QPR_E_ARG
    same = (C.c_void_p * 2)(4096, 4096)
    assert many(2, probs, omegas, *head, 2, ws, wsb, same) == qpr.QPR_E_ARG
    assert "share a stream" in L.qpr_last_error().decode()
    assert many(2, probs, omegas, *head, 2, ws, wsb, (C.c_void_p * 2)(4096, 8192)) == qpr.QPR_E_ARG
    assert "probs[0] is NULL" in L.qpr_last_error().decode()
    # a built-looking problem whose workspaces are too small
    P = qpr.qpr_problem()
    P.n, P.ld = 100, 128
    ps = (C.c_void_p * 2)(C.addressof(P), C.addressof(P))
    bad = (C.c_void_p * 2)(256, 512)
    assert many(2, ps, omegas, *head, 2, bad, wsb, (C.c_void_p * 2)(4096, 8192)) == \
        qpr.QPR_E_WORKSPACE


def test_batch_workspace_query_and_mode_check():
    """Host-side: the concurrent form needs one single-system workspace of
    the largest system per worker; the persistent form more; an unknown
    batch_mode is rejected before any device work."""
    L = _lib()
    ns = (C.c_int32 * 3)(40, 922, 75)
    one = L.qpr_workspace_bytes(922, 0, 0)
    for workers, want in ((0, 3), (2, 2), (100, 3)):   # 0 = min(nsys, 8); capped at nsys
        op = qpr.make_opts(batch_workers=workers)
        assert L.qpr_batch_workspace_bytes(3, ns, 0, C.byref(op)) == want * one
    # RKF45 workers carry the Fehlberg planes, RK4 workers do not
    op = qpr.make_opts(batch_workers=2, integrator="rkf45")
    assert L.qpr_batch_workspace_bytes(3, ns, 0, C.byref(op)) == 2 * L.qpr_workspace_bytes(922, 0, 1)
    pers = L.qpr_batch_workspace_bytes(3, ns, 0, C.byref(qpr.make_opts(batch_mode="persistent")))
    assert pers > 0 and pers != 3 * one
    assert L.qpr_batch_workspace_bytes(3, ns, 2, None) == 0      # no BF16x3 batch
    # AUTO: FP32 batches of eight or more systems take the persistent form
    # (unless the defect is forced to FP64 or a product is named)
    n8 = (C.c_int32 * 8)(*([40, 922, 75] * 3)[:8])
    n7 = (C.c_int32 * 7)(*([40, 922, 75] * 3)[:7])
    one32 = L.qpr_workspace_bytes(922, 1, 0)
    persist8 = L.qpr_batch_workspace_bytes(8, n8, 1, C.byref(qpr.make_opts(batch_mode="persistent")))
    assert L.qpr_batch_workspace_bytes(8, n8, 1, C.byref(qpr.make_opts())) == persist8
    assert L.qpr_batch_workspace_bytes(8, n8, 1, None) == persist8
    assert L.qpr_batch_workspace_bytes(7, n7, 1, C.byref(qpr.make_opts())) == 7 * one32
    assert L.qpr_batch_workspace_bytes(8, n8, 0, C.byref(qpr.make_opts())) == 8 * one
    for kw in (dict(delta_state="fp64"), dict(product="fused")):
        assert L.qpr_batch_workspace_bytes(8, n8, 1, C.byref(qpr.make_opts(**kw))) == 8 * one32
    P = qpr.qpr_problem()
    P.n, P.ld, P.h_off = 100, 128, C.c_void_p(256)
    op = qpr.make_opts()
    op.batch_mode = 5
    st = L.qpr_batch_solve(1, (C.c_void_p * 1)(C.addressof(P)), (C.c_double * 1)(0.5), 0.01,
                           1e-8, 10, 0, (C.c_void_p * 1)(256), None, None, C.byref(op), None,
                           None, C.c_void_p(256), 1 << 20, None)
    assert st == qpr.QPR_E_ARG and "batch_mode" in L.qpr_last_error().decode()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(qpr, "_lib", None)
    monkeypatch.setattr(qpr, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(qpr.QprError):
        qpr.lib()


def test_load_tuning_parses_every_entry_kind(tmp_path):
    """Dense tiles (precision codes 0-2), the sparse-product variant (10) and
    the stage form (11) load; malformed or out-of-range lines are skipped and
    a cache with none left is an error."""
    L = _lib()
    good = tmp_path / "tune.txt"
    good.write_text("0 960 1 139.2 f64_32x32_w16x16_k16\n"
                    "10 960 4 11.9 row128\n"
                    "11 960 0 24.4 product+epilogue\n"
                    "11 4096 1 401.0 fused_epilogue\n")
    assert L.qpr_load_tuning(str(good).encode()) == qpr.QPR_OK
    bad = tmp_path / "bad.txt"
    bad.write_text("10 960 99 1.0 none\n11 960 7 1.0 none\n3 960 0 1.0 none\n0 100 0 1.0 odd\n")
    assert L.qpr_load_tuning(str(bad).encode()) == qpr.QPR_E_ARG
    assert L.qpr_load_tuning(str(tmp_path / "absent.txt").encode()) == qpr.QPR_E_ARG


def test_product_configuration_tables():
    """Host-side tables of the dense-product tile configurations: names are
    unique per precision, and the BF16x3 table holds both MFMA families (the
    32 x 32 x 16 ones named _m32_), whose results agree only within the
    family (the GPU test checks the values)."""
    _lib()
    counts = {}
    for prec in ("fp64", "fp32", "bf16x3"):
        names = qpr.product_configs(prec)
        assert len(names) == len(set(names)) and len(names) >= 6, prec
        assert all(n.startswith(prec.replace("fp", "f")) or n.startswith(prec) for n in names)
        counts[prec] = names
    bf = counts["bf16x3"]
    assert any("_m32_" in n for n in bf) and any("_m32_" not in n for n in bf)
    assert qpr.lib().qpr_product_configs(99) == 0
    assert qpr.lib().qpr_product_config_name(99, 0) == b"?"
    assert qpr.lib().qpr_product_config_name(0, 10 ** 6) == b"?"
