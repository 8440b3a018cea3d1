"""The C-ABI library loads and exports every entry point declared in
include/cbgmres.h; host-only size queries agree with the oracle's storage
definitions; argument errors are reported before any device work (CPU only)."""
import ctypes as C
import os
import re
import subprocess

import pytest

import oracle
import paper_2409_15468_amd as cb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cbgmres.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set()
    for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b([a-z][a-z0-9_]*)\s*\(", text, flags=re.M):
        line = m.group(0)
        if line.lstrip().startswith(("typedef", "#")):
            continue
        names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 25
    L = cb.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", cb.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert set(names) <= exported
    assert set(names) == set(cb.SIGNATURES)


def test_size_queries_match_storage_definitions():
    for n in (1, 31, 32, 33, 1000, 1 << 20, 1000003):
        assert cb.frsz2_exponent_words(n) == (n + 31) // 32
        for bits in (16, 21, 32):
            assert cb.frsz2_value_words(n, bits) == bits * ((n + 31) // 32)
        for fmt in oracle.FORMATS:
            stride = cb.cb_basis_column_bytes(fmt, n)
            data = oracle.col_bytes(fmt, n)
            assert stride % 256 == 0 and data <= stride < data + 256
            V = cb.Basis(cb.FORMATS[fmt], n, 1, None, None)
            assert V.column_data_bytes() == data
            ew = cb.cb_basis_exponent_words(fmt, n)
            assert ew == ((n + 31) // 32 if fmt.startswith("frsz2") else 0)
    for l in range(3, 33):
        assert cb.frsz2_value_words(1000, l) == l * 32
        f = cb.frsz2_bits_format(l)
        assert cb.cb_basis_column_bytes(f, 1000) == (l * 32 * 4 + 255) // 256 * 256
        assert cb.cb_basis_exponent_words(f, 1000) == 32
        assert oracle.col_bytes(f, 1000) == l * 32 * 4
    assert cb.frsz2_value_words(10, 2) == -1 and cb.frsz2_value_words(10, 33) == -1
    assert cb.cb_basis_column_bytes(9, 10) == -1
    assert cb.cb_basis_column_bytes(cb.CB_FRSZ2_GENERIC_BASE + 2, 10) == -1
    assert cb.cb_basis_column_bytes(cb.CB_FRSZ2_GENERIC_BASE + 33, 10) == -1
    assert cb.cbgmres_batch_workspace_bytes(1000, 30, cb.frsz2_bits_format(12)) == -1
    assert cb.cbgmres_workspace_bytes(1000, 10, "frsz2_32") > 11 * cb.cb_basis_column_bytes("frsz2_32", 1000)
    assert cb.Server.request_bytes(1000, 5000, 10, "float32") > cb.cbgmres_workspace_bytes(1000, 10, "float32")


def test_argument_errors_without_device_work():
    L = cb.lib()
    for bad_bits in (2, 33, 0, -1):
        assert L.frsz2_compress(None, 10, bad_bits, None, None, None, None) == cb.CB_ERR_UNSUPPORTED_BITS
        assert L.frsz2_decompress(None, None, 10, bad_bits, None, None) == cb.CB_ERR_UNSUPPORTED_BITS
    assert b"3 to 32" in L.cb_last_error()
    assert L.frsz2_compress(None, 10, 32, None, None, None, None) == cb.CB_ERR_INVALID_ARG
    assert L.frsz2_compress(None, 10, 17, None, None, None, None) == cb.CB_ERR_INVALID_ARG
    assert L.frsz2_decompress(None, None, 0, 16, None, None) == cb.CB_ERR_INVALID_ARG
    A = cb.cb_csr(10, 0, None, None, None)
    res = cb.cb_result()
    st = L.cbgmres_solve(C.byref(A), None, None, 10, 1e-8, 5, None, None, 0, None, 0, C.byref(res), None)
    assert st == cb.CB_ERR_INVALID_ARG
    V = cb.cb_basis(5, 100, 4, 0, None, None)
    assert L.cb_basis_load(C.byref(V), 0, None, None) == cb.CB_ERR_INVALID_ARG
    V = cb.cb_basis(9, 100, 4, 0, 1, 1)  # 9: no such format
    assert L.cb_basis_load(C.byref(V), 0, 1, None) == cb.CB_ERR_INVALID_ARG
    for s in range(10):
        assert L.cb_status_string(s)


def test_column_count_limits_without_device_work():
    """The projection, update and combine take at most 513 columns (their
    per-column sums and coefficients live in LDS); more is rejected before any
    launch.  Pointers here are never dereferenced."""
    L = cb.lib()
    V = cb.cb_basis(5, 100, 600, 0, 256, 256)
    assert L.cb_cgs_project(C.byref(V), 514, 256, 256, 256, 1 << 30, None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_cgs_subtract(C.byref(V), 514, 256, 256, None, None, 0, None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_basis_combine(C.byref(V), 514, 256, 256, None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_cgs_project_noalloc(C.byref(V), 514, 256, 256, None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_cgs_project_noalloc(C.byref(V), 0, 256, 256, None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_cgs_project_noalloc(C.byref(V), 4, 256, None, None) == cb.CB_ERR_INVALID_ARG


def test_noalloc_scratch_size():
    """The fixed scratch of the allocation-free projection holds the ticket
    counters and 512 workgroup partials for each of 513 columns, the most any
    valid call writes."""
    assert cb.cb_cgs_project_noalloc_max_bytes() == 8192 + 8 * 512 * 513


def test_batch_arguments_without_device_work():
    L = cb.lib()
    assert cb.cbgmres_batch_max_n() >= 16384 and cb.cbgmres_batch_max_restart() >= 100
    assert cb.cbgmres_batch_workspace_bytes(0, 10, "float64") == -1
    assert cb.cbgmres_batch_workspace_bytes(100, 0, "float64") == -1
    assert cb.cbgmres_batch_workspace_bytes(100, 10, 9) == -1
    need = cb.cbgmres_batch_workspace_bytes(1000, 30, "frsz2_21")
    assert need >= 31 * cb.cb_basis_column_bytes("frsz2_21", 1000) + 2 * 8 * 1000
    res = (cb.cb_result * 1)()
    item = (cb.cb_batch_item * 1)()
    item[0].A = cb.cb_csr(1000, 5000, 256, 256, 256)
    item[0].b, item[0].x, item[0].workspace = 256, 256, 256
    item[0].workspace_bytes = need
    item[0].m, item[0].format, item[0].tol = 30, 4, 1e-8
    item[0].m = cb.cbgmres_batch_max_restart() + 1
    assert L.cbgmres_solve_batch(item, 1, None, res, None) == cb.CB_ERR_INVALID_ARG
    item[0].m = 30
    item[0].workspace_bytes = need - 1
    assert L.cbgmres_solve_batch(item, 1, None, res, None) == cb.CB_ERR_WORKSPACE
    item[0].workspace_bytes = need
    item[0].workspace = 257  # not 256-byte aligned
    assert L.cbgmres_solve_batch(item, 1, None, res, None) == cb.CB_ERR_WORKSPACE
    item[0].workspace = 256
    item[0].tol = 0.0
    assert L.cbgmres_solve_batch(item, 1, None, res, None) == cb.CB_ERR_INVALID_ARG
    assert L.cbgmres_solve_batch(item, 0, None, res, None) == cb.CB_OK


def test_auto_solve_arguments_without_device_work():
    """cbgmres_solve_auto rejects bad candidate lists, probe lengths and
    workspaces before any device work.  Pointers here are never dereferenced."""
    L = cb.lib()
    res = cb.cb_auto_result()
    A = cb.cb_csr(1000, 5000, 256, 256, 256)
    need = cb.cbgmres_auto_workspace_bytes(1000, 30, 10, ["frsz2_32", "float16"])
    assert need >= max(cb.cbgmres_workspace_bytes(1000, 30, f) for f in ("frsz2_32", "float16")) + 3 * 8 * 1000
    assert cb.cbgmres_auto_workspace_bytes(1000, 30, 0, ["frsz2_32"]) == -1
    assert cb.cbgmres_auto_workspace_bytes(1000, 30, 10, [9]) == -1
    assert cb.cbgmres_auto_workspace_bytes(1000, 30, 10, ["float64"] * 9) == -1

    def call(cands, probe, ws_bytes=need, m=30, tol=1e-8):
        fm = (C.c_int32 * max(1, len(cands)))(*cands)
        return L.cbgmres_solve_auto(C.byref(A), 256, 256, m, tol, C.cast(fm, C.c_void_p), len(cands), probe,
                                    None, 256, ws_bytes, None, 0, C.byref(res), None)
    assert call([], 10) == cb.CB_ERR_INVALID_ARG
    assert call([5] * 9, 10) == cb.CB_ERR_INVALID_ARG
    assert call([5, 9], 10) == cb.CB_ERR_INVALID_ARG
    assert call([5, 2], 0) == cb.CB_ERR_INVALID_ARG
    assert call([5, 2], 513) == cb.CB_ERR_INVALID_ARG
    assert call([5, 2], 10, m=0) == cb.CB_ERR_INVALID_ARG
    assert call([5, 2], 10, tol=0.0) == cb.CB_ERR_INVALID_ARG
    assert call([5, 2], 10, ws_bytes=need - 1) == cb.CB_ERR_WORKSPACE


def test_precond_arguments_without_device_work():
    """cbgmres_solve_precond and cb_jacobi_setup reject bad arguments before
    any device work.  Pointers here are never dereferenced."""
    L = cb.lib()
    res = cb.cb_result()
    A = cb.cb_csr(1000, 5000, 256, 256, 256)
    need = cb.cbgmres_precond_workspace_bytes(1000, 5000, 30, "frsz2_16")
    assert need >= cb.cbgmres_workspace_bytes(1000, 30, "frsz2_16") + 8 * 5000
    assert cb.cbgmres_precond_workspace_bytes(0, 5000, 30, "frsz2_16") == -1
    assert cb.cbgmres_precond_workspace_bytes(1000, 5000, 30, 9) == -1

    def call(kind, diag, ws_bytes=need, m=30):
        M = cb.cb_precond(kind, 0, diag)
        return L.cbgmres_solve_precond(C.byref(A), 256, 256, m, 1e-8, 3, C.byref(M), None, 256, ws_bytes,
                                       None, 0, C.byref(res), None)
    assert call(7, 256) == cb.CB_ERR_INVALID_ARG
    assert call(cb.CB_PRECOND_JACOBI, None) == cb.CB_ERR_INVALID_ARG
    assert call(cb.CB_PRECOND_JACOBI, 256, m=513) == cb.CB_ERR_INVALID_ARG
    assert call(cb.CB_PRECOND_JACOBI, 256, ws_bytes=need - 1) == cb.CB_ERR_WORKSPACE
    assert L.cb_jacobi_setup(None, 256, None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_jacobi_setup(C.byref(cb.cb_csr(0, 0, 256, None, None)), 256, None) == cb.CB_ERR_INVALID_ARG


def test_misaligned_pointers_rejected_without_device_work():
    """Basis values and the vectors the row kernels access in 16-byte pieces
    must be 16-byte aligned; a misaligned pointer is an argument error, caught
    before any launch.  Pointers here are never dereferenced."""
    L = cb.lib()
    V = cb.cb_basis(5, 1000, 4, 0, 256 + 8, 256)
    assert L.cb_basis_load(C.byref(V), 0, 256, None) == cb.CB_ERR_INVALID_ARG
    V = cb.cb_basis(5, 1000, 4, 0, 256, 258)
    assert L.cb_basis_load(C.byref(V), 0, 256, None) == cb.CB_ERR_INVALID_ARG
    V = cb.cb_basis(5, 1000, 4, 0, 256, 256)
    assert L.cb_basis_load(C.byref(V), 0, 264, None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_basis_store(C.byref(V), 0, 264, None, None, None, None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_basis_store(C.byref(V), 0, 256, None, 264, None, None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_cgs_project(C.byref(V), 2, 264, 256, 256, 1 << 30, None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_cgs_subtract(C.byref(V), 2, 256, 264, None, None, 0, None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_basis_combine(C.byref(V), 2, 256, 264, None) == cb.CB_ERR_INVALID_ARG
    assert L.frsz2_compress(264, 1000, 16, 256, 256, None, None) == cb.CB_ERR_INVALID_ARG
    assert L.frsz2_compress(256, 1000, 16, 256, 264, None, None) == cb.CB_ERR_INVALID_ARG
    assert L.frsz2_decompress(256, 264, 1000, 21, 256, None) == cb.CB_ERR_INVALID_ARG
    A = cb.cb_csr(1000, 5000, 256, 256, 256)
    res = cb.cb_result()
    assert L.cbgmres_solve(C.byref(A), 256, 264, 10, 1e-8, 5, None, None, 0, None, 0, C.byref(res),
                           None) == cb.CB_ERR_INVALID_ARG
    assert L.cbgmres_solve(C.byref(A), 260, 256, 10, 1e-8, 5, None, None, 0, None, 0, C.byref(res),
                           None) == cb.CB_ERR_INVALID_ARG


def test_row_count_limit_without_device_work():
    """n may not exceed 2^31 - 4096: every 32-bit row index a kernel forms,
    padding to 2048-row groups included, stays below 2^31.  Pointers here are
    never dereferenced."""
    L = cb.lib()
    nmax = (1 << 31) - 4096
    assert cb.cb_basis_column_bytes("frsz2_32", nmax) > 0
    assert cb.cbgmres_workspace_bytes(nmax, 10, "float64") > 0
    assert cb.cbgmres_workspace_bytes(nmax + 1, 10, "float64") == -1
    assert cb.cb_reduce_workspace_bytes(nmax + 1, 4) == -1
    assert cb.cb_intensity_groups(nmax + 1) == -1
    V = cb.cb_basis(5, nmax + 1, 4, 0, 256, 256)
    assert L.cb_basis_load(C.byref(V), 0, 256, None) == cb.CB_ERR_INVALID_ARG
    assert L.frsz2_compress(256, nmax + 1, 21, 256, 256, None, None) == cb.CB_ERR_INVALID_ARG
    A = cb.cb_csr(nmax + 1, 5000, 256, 256, 256)
    res = cb.cb_result()
    assert L.cbgmres_solve(C.byref(A), 256, 256, 10, 1e-8, 5, None, None, 0, None, 0, C.byref(res),
                           None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_jacobi_setup(C.byref(A), 256, None) == cb.CB_ERR_INVALID_ARG


def test_header_is_plain_c(tmp_path):
    """include/cbgmres.h compiles as C99 (no C++ or HIP types in the ABI)."""
    src = tmp_path / "use.c"
    src.write_text('#include "cbgmres.h"\n'
                   'int f(cb_csr* A, const double* b, double* x, void* s) {\n'
                   '    cb_result r;\n'
                   '    return cbgmres_solve(A, b, x, 30, 1e-8, CB_FRSZ2_BITS(12), 0, 0, 0, 0, 0, &r, s);\n'
                   '}\n')
    out = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-fsyntax-only",
                          "-I", os.path.dirname(HEADER), str(src)], capture_output=True, text=True)
    assert out.returncode == 0, out.stderr


def test_ir_arguments_without_device_work():
    """cbgmres_ir_solve checks its workspace (size, 256-byte alignment) and
    scalars before any device work.  Pointers here are never dereferenced."""
    L = cb.lib()
    res = cb.cb_result()
    A = cb.cb_csr(1000, 5000, 256, 256, 256)
    need = cb.cbgmres_ir_workspace_bytes(1000, 100, "frsz2_16")
    assert need >= cb.cbgmres_workspace_bytes(1000, 100, "frsz2_16") + 2 * 8 * 1000
    assert cb.cbgmres_ir_workspace_bytes(0, 100, "frsz2_16") == -1
    assert cb.cbgmres_ir_workspace_bytes(1000, 513, "frsz2_16") == -1
    assert cb.cbgmres_ir_workspace_bytes(1000, 100, 9) == -1

    def call(ws=256, ws_bytes=need, inner_tol=1e-4, max_outer=10):
        return L.cbgmres_ir_solve(C.byref(A), 256, 256, 100, inner_tol, 1e-12, 3, max_outer, ws, ws_bytes,
                                  C.byref(res), None)
    assert call(ws_bytes=need - 1) == cb.CB_ERR_WORKSPACE
    assert call(ws=256 + 16) == cb.CB_ERR_INVALID_ARG
    assert call(inner_tol=0.0) == cb.CB_ERR_INVALID_ARG
    assert call(max_outer=0) == cb.CB_ERR_INVALID_ARG


def test_batch_rejects_b_not_16_byte_aligned():
    """The batched solver reads b in 16-byte pieces, so an 8-byte-offset b is
    an argument error before any launch.  Pointers are never dereferenced."""
    L = cb.lib()
    need = cb.cbgmres_batch_workspace_bytes(1000, 30, "frsz2_21")
    res = (cb.cb_result * 1)()
    item = (cb.cb_batch_item * 1)()
    item[0].A = cb.cb_csr(1000, 5000, 256, 256, 256)
    item[0].b, item[0].x, item[0].workspace = 256 + 8, 256, 256
    item[0].workspace_bytes = need
    item[0].m, item[0].format, item[0].tol = 30, 4, 1e-8
    assert L.cbgmres_solve_batch(item, 1, None, res, None) == cb.CB_ERR_INVALID_ARG
    item[0].b = 256
    item[0].x = 256 + 8
    assert L.cbgmres_solve_batch(item, 1, None, res, None) == cb.CB_ERR_INVALID_ARG
