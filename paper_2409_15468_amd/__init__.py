"""Python binding of libcbgmres.so: restarted GMRES with an FRSZ2-compressed
(or low-precision) Krylov basis on an MI355X GPU.

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Device buffers are torch tensors on the HIP device (PyTorch provides
memory and streams); each function passes their data pointers and the current
stream to the C entry point of the same name and raises CbError on a non-zero
status.  There is no CPU fallback: without the built library, importing the
bindings' functions raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbgmres.so")

CB_OK, CB_ERR_INVALID_ARG, CB_ERR_UNSUPPORTED_BITS, CB_ERR_NONFINITE = 0, 1, 2, 3
CB_ERR_NOT_CONVERGED, CB_ERR_WORKSPACE, CB_ERR_OVER_BUDGET, CB_ERR_HIP = 4, 5, 6, 7
CB_PENDING, CB_ERR_NOT_FOUND = 8, 9

FORMATS = {"float64": 0, "float32": 1, "float16": 2, "frsz2_16": 3, "frsz2_21": 4, "frsz2_32": 5}
FORMAT_NAMES = {v: k for k, v in FORMATS.items()}


class CbError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class cb_basis(C.Structure):
    _fields_ = [("format", C.c_int32), ("n", C.c_int32), ("ncols", C.c_int32),
                ("reserved", C.c_int32), ("values", C.c_void_p), ("exps", C.c_void_p)]


class cb_csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class cb_options(C.Structure):
    _fields_ = [("eta", C.c_double), ("max_iters", C.c_int32), ("max_cycles", C.c_int32),
                ("literal_breakdown", C.c_int32), ("fuse_updates", C.c_int32)]


class cb_result(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("reorths", C.c_int32),
                ("breakdowns", C.c_int32), ("converged", C.c_int32), ("status", C.c_int32),
                ("rel_residual", C.c_double), ("implicit_rel_residual", C.c_double),
                ("seconds", C.c_double), ("basis_bytes", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


CB_PRECOND_NONE, CB_PRECOND_JACOBI = 0, 1


class cb_precond(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("diag_inv", C.c_void_p)]


CB_AUTO_MAX_CANDIDATES = 8


class cb_auto_result(C.Structure):
    _K = CB_AUTO_MAX_CANDIDATES
    _fields_ = [("chosen", C.c_int32), ("chosen_format", C.c_int32), ("probed", C.c_int32),
                ("status", C.c_int32), ("rel_residual0", C.c_double),
                ("probe_steps", C.c_int32 * _K), ("probe_rel_residual", C.c_double * _K),
                ("probe_seconds", C.c_double * _K), ("probe_rate", C.c_double * _K),
                ("seconds", C.c_double), ("solve", cb_result)]

    def as_dict(self) -> dict:
        k = self.probed
        return {"chosen": self.chosen, "chosen_format": self.chosen_format, "probed": k,
                "status": self.status, "rel_residual0": self.rel_residual0,
                "probe_steps": list(self.probe_steps[:k]),
                "probe_rel_residual": list(self.probe_rel_residual[:k]),
                "probe_seconds": list(self.probe_seconds[:k]), "probe_rate": list(self.probe_rate[:k]),
                "seconds": self.seconds, "solve": self.solve.as_dict()}


class cb_batch_item(C.Structure):
    _fields_ = [("A", cb_csr), ("b", C.c_void_p), ("x", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("m", C.c_int32), ("format", C.c_int32),
                ("tol", C.c_double)]


# name -> (restype, argtypes); the full C ABI of include/cbgmres.h
_P, _I32, _I64, _D, _SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
SIGNATURES = {
    "cb_status_string": (C.c_char_p, [C.c_int]),
    "cb_last_error": (C.c_char_p, []),
    "frsz2_exponent_words": (_I64, [_I64]),
    "frsz2_value_words": (_I64, [_I64, C.c_int]),
    "frsz2_compress": (C.c_int, [_P, _I64, C.c_int, _P, _P, _P, _P]),
    "frsz2_decompress": (C.c_int, [_P, _P, _I64, C.c_int, _P, _P]),
    "cb_basis_column_bytes": (_I64, [C.c_int, _I64]),
    "cb_basis_exponent_words": (_I64, [C.c_int, _I64]),
    "cb_basis_store": (C.c_int, [C.POINTER(cb_basis), _I32, _P, _P, _P, _P, _P]),
    "cb_basis_load": (C.c_int, [C.POINTER(cb_basis), _I32, _P, _P]),
    "cb_reduce_workspace_bytes": (_I64, [_I32, _I32]),
    "cb_cgs_project": (C.c_int, [C.POINTER(cb_basis), _I32, _P, _P, _P, _SZ, _P]),
    "cb_cgs_project_noalloc": (C.c_int, [C.POINTER(cb_basis), _I32, _P, _P, _P]),
    "cb_cgs_project_noalloc_max_bytes": (_I64, []),
    "cb_cgs_subtract": (C.c_int, [C.POINTER(cb_basis), _I32, _P, _P, _P, _P, _SZ, _P]),
    "cb_cgs_subtract_project": (C.c_int, [C.POINTER(cb_basis), _I32, _P, _P, _P, _P, _SZ, _P]),
    "cb_basis_combine": (C.c_int, [C.POINTER(cb_basis), _I32, _P, _P, _P]),
    "cb_spmv_workspace_bytes": (_I64, [_I32, _I32]),
    "cb_spmv": (C.c_int, [C.POINTER(cb_csr), _P, _P, _P, _P, _SZ, _P]),
    "cb_residual": (C.c_int, [C.POINTER(cb_csr), _P, _P, _P, _P, _P, _SZ, _P]),
    "cbgmres_workspace_bytes": (_I64, [_I32, _I32, C.c_int]),
    "cbgmres_solve": (C.c_int, [C.POINTER(cb_csr), _P, _P, _I32, _D, C.c_int, C.POINTER(cb_options),
                                _P, _SZ, _P, _I64, C.POINTER(cb_result), _P]),
    "cbgmres_ir_workspace_bytes": (_I64, [_I32, _I32, C.c_int]),
    "cbgmres_ir_solve": (C.c_int, [C.POINTER(cb_csr), _P, _P, _I32, _D, _D, C.c_int, _I32, _P, _SZ,
                                   C.POINTER(cb_result), _P]),
    "cb_jacobi_setup": (C.c_int, [C.POINTER(cb_csr), _P, _P]),
    "cbgmres_precond_workspace_bytes": (_I64, [_I32, _I32, _I32, C.c_int]),
    "cbgmres_solve_precond": (C.c_int, [C.POINTER(cb_csr), _P, _P, _I32, _D, C.c_int, C.POINTER(cb_precond),
                                        C.POINTER(cb_options), _P, _SZ, _P, _I64, C.POINTER(cb_result), _P]),
    "cb_auto_pick": (_I32, [_D, _P, _P, _I32]),
    "cbgmres_auto_workspace_bytes": (_I64, [_I32, _I32, _I32, _P, _I32]),
    "cbgmres_solve_auto": (C.c_int, [C.POINTER(cb_csr), _P, _P, _I32, _D, _P, _I32, _I32,
                                     C.POINTER(cb_options), _P, _SZ, _P, _I64,
                                     C.POINTER(cb_auto_result), _P]),
    "cbgmres_batch_max_n": (_I32, []),
    "cbgmres_batch_max_restart": (_I32, []),
    "cbgmres_batch_workspace_bytes": (_I64, [_I32, _I32, C.c_int]),
    "cbgmres_solve_batch": (C.c_int, [C.POINTER(cb_batch_item), _I32, C.POINTER(cb_options),
                                      C.POINTER(cb_result), _P]),
    "cb_intensity_groups": (_I32, [_I64]),
    "cb_intensity_run": (C.c_int, [C.POINTER(cb_basis), _I32, _I32, _D, _D, _P, _P]),
    "cb_server_create": (_P, [_SZ, C.c_int, C.c_int]),
    "cb_server_request_bytes": (_I64, [_I32, _I32, _I32, C.c_int]),
    "cb_server_submit": (C.c_int, [_P, _I32, _I32, _P, _P, _P, _P, _P, _I32, _D, C.c_int,
                                   C.POINTER(C.c_uint64)]),
    "cb_server_poll": (C.c_int, [_P, C.c_uint64, _P, C.POINTER(cb_result), _P]),
    "cb_server_stats": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "cb_server_ring_stats": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "cb_server_destroy": (None, [_P]),
}

_lib = None


def lib() -> C.CDLL:
    """The loaded library.  Raises if it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c "
                               f"'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int, where: str) -> int:
    if st not in (CB_OK,):
        raise CbError(st, where, lib().cb_last_error().decode() or lib().cb_status_string(st).decode())
    return st


CB_FRSZ2_GENERIC_BASE = 64
CB_FRSZ2_B64_GENERIC_BASE = 128
CB_FRSZ2_16_B64, CB_FRSZ2_32_B64 = 6, 7
FORMATS_B64 = {"frsz2b64_16": CB_FRSZ2_16_B64, "frsz2b64_32": CB_FRSZ2_32_B64}


def frsz2_bits_format(l: int, block: int = 32) -> int:
    """CB_FRSZ2_BITS(l) (block 32) or CB_FRSZ2_B64_BITS(l) (block 64): FRSZ2
    with l bits (3 <= l <= 32) on the generic codec."""
    if not 3 <= l <= 32 or block not in (32, 64):
        raise ValueError("l must lie in [3, 32] and the block size be 32 or 64")
    return (CB_FRSZ2_GENERIC_BASE if block == 32 else CB_FRSZ2_B64_GENERIC_BASE) + l


def format_bits(f: int) -> int:
    """FRSZ2 l of format number f (0 for the float formats)."""
    return {3: 16, 4: 21, 5: 32, 6: 16, 7: 32}.get(f, f & 63 if f > 64 else 0)


def format_block(f: int) -> int:
    """FRSZ2 block size of format number f (32 for the float formats)."""
    return 64 if f in (6, 7) or f > CB_FRSZ2_B64_GENERIC_BASE else 32


def _fmt(fmt) -> int:
    """A format name or number: the names of FORMATS and FORMATS_B64,
    "frsz2_<l>" for any other l in [3, 32], "frsz2g_<l>" for the generic codec
    at any l; "frsz2b64_<l>" / "frsz2b64g_<l>" likewise with blocks of 64."""
    if not isinstance(fmt, str):
        return int(fmt)
    if fmt in FORMATS:
        return FORMATS[fmt]
    if fmt in FORMATS_B64:
        return FORMATS_B64[fmt]
    if fmt.startswith("frsz2b64_") or fmt.startswith("frsz2b64g_"):
        return frsz2_bits_format(int(fmt.split("_")[1]), 64)
    if fmt.startswith("frsz2_") or fmt.startswith("frsz2g_"):
        return frsz2_bits_format(int(fmt.split("_")[1]))
    raise KeyError(fmt)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype, name):
    import torch
    if t is None:
        return
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on the GPU")


# ---------------------------------------------------------------- FRSZ2 codec
def frsz2_exponent_words(n: int) -> int:
    return int(lib().frsz2_exponent_words(n))


def frsz2_value_words(n: int, bits: int) -> int:
    return int(lib().frsz2_value_words(n, bits))


def frsz2_compress(x, bits: int, exps=None, words=None, nonfinite_flag=None, stream=None):
    """Compress the float64 device vector x; returns (exps, words) device
    tensors of 32-bit words (int32 storage of the uint32 words; allocated here
    unless given)."""
    import torch
    _dev(x, torch.float64, "x")
    n = x.numel()
    nw = frsz2_value_words(n, bits)
    if nw < 0:
        _check(CB_ERR_UNSUPPORTED_BITS, f"frsz2_compress(bits={bits})")
    if exps is None:
        exps = torch.empty(frsz2_exponent_words(n), dtype=torch.int32, device=x.device)
    if words is None:
        words = torch.empty(nw, dtype=torch.int32, device=x.device)
    if exps.numel() < frsz2_exponent_words(n) or words.numel() < nw:
        raise ValueError("exps/words too small")
    _check(lib().frsz2_compress(_ptr(x), n, bits, _ptr(exps), _ptr(words), _ptr(nonfinite_flag),
                                _stream(stream)), "frsz2_compress")
    return exps, words


def frsz2_decompress(exps, words, n: int, bits: int, x=None, stream=None):
    import torch
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=words.device)
    _dev(x, torch.float64, "x")
    if exps.numel() < frsz2_exponent_words(n) or words.numel() < frsz2_value_words(n, bits):
        raise ValueError("exps/words too small")
    _check(lib().frsz2_decompress(_ptr(exps), _ptr(words), n, bits, _ptr(x), _stream(stream)),
           "frsz2_decompress")
    return x


# ---------------------------------------------------------------- basis
def cb_basis_column_bytes(fmt, n: int) -> int:
    return int(lib().cb_basis_column_bytes(_fmt(fmt), n))


def cb_basis_exponent_words(fmt, n: int) -> int:
    return int(lib().cb_basis_exponent_words(_fmt(fmt), n))


@dataclass
class Basis:
    """A device basis of `ncols` columns over n rows in one storage format."""
    fmt: int
    n: int
    ncols: int
    values: "object"  # torch.uint8 tensor, ncols * column_bytes
    exps: "object"    # torch.int32 tensor holding the uint32 exponent words, or None

    @staticmethod
    def empty(fmt, n: int, ncols: int, device="cuda") -> "Basis":
        import torch
        f = _fmt(fmt)
        cb = cb_basis_column_bytes(f, n)
        ew = cb_basis_exponent_words(f, n)
        vals = torch.zeros(ncols * cb, dtype=torch.uint8, device=device)
        ex = torch.zeros(max(ncols * ew, 1), dtype=torch.int32, device=device) if ew else None
        return Basis(f, n, ncols, vals, ex)

    def desc(self) -> cb_basis:
        return cb_basis(self.fmt, self.n, self.ncols, 0, self.values.data_ptr(),
                        self.exps.data_ptr() if self.exps is not None else None)

    def column_bytes(self) -> int:
        return cb_basis_column_bytes(self.fmt, self.n)

    def column_data_bytes(self) -> int:
        bits, bs = format_bits(self.fmt), format_block(self.fmt)
        if not bits:
            return (self.n + 31) // 32 * 32 * (8, 4, 2)[self.fmt]
        return (self.n + bs - 1) // bs * (bs // 32) * bits * 4

    def column(self, c: int):
        """The stored bytes of column c (without the stride padding)."""
        cb = self.column_bytes()
        return self.values[c * cb:c * cb + self.column_data_bytes()]

    def column_exps(self, c: int):
        ew = cb_basis_exponent_words(self.fmt, self.n)
        return None if not ew else self.exps[c * ew:(c + 1) * ew]


def cb_basis_store(V: Basis, col: int, w, divisor=None, v_out=None, nonfinite_flag=None, stream=None):
    import torch
    _dev(w, torch.float64, "w")
    if w.numel() < V.n or not (0 <= col < V.ncols):
        raise ValueError("bad w size or column")
    d = V.desc()
    _check(lib().cb_basis_store(C.byref(d), col, _ptr(w), _ptr(divisor), _ptr(v_out),
                                _ptr(nonfinite_flag), _stream(stream)), "cb_basis_store")


def cb_basis_load(V: Basis, col: int, x=None, stream=None):
    import torch
    if x is None:
        x = torch.empty(V.n, dtype=torch.float64, device=V.values.device)
    if not (0 <= col < V.ncols) or x.numel() < V.n:
        raise ValueError("bad column or x size")
    d = V.desc()
    _check(lib().cb_basis_load(C.byref(d), col, _ptr(x), _stream(stream)), "cb_basis_load")
    return x


def cb_reduce_workspace_bytes(n: int, ncols: int) -> int:
    return int(lib().cb_reduce_workspace_bytes(n, ncols))


def _work(n: int, ncols: int, device):
    import torch
    nbytes = cb_reduce_workspace_bytes(n, ncols)
    return torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=device), nbytes


def cb_cgs_project(V: Basis, j: int, w, h=None, work=None, stream=None):
    import torch
    _dev(w, torch.float64, "w")
    if not (1 <= j <= V.ncols) or w.numel() < V.n:
        raise ValueError("bad j or w size")
    if h is None:
        h = torch.empty(j, dtype=torch.float64, device=w.device)
    if work is None:
        work, nbytes = _work(V.n, j, w.device)
    else:
        nbytes = work.numel() * work.element_size()
    d = V.desc()
    _check(lib().cb_cgs_project(C.byref(d), j, _ptr(w), _ptr(h), _ptr(work), nbytes, _stream(stream)),
           "cb_cgs_project")
    return h


def cb_cgs_project_noalloc(V: Basis, j: int, w, h, stream=None):
    """cb_cgs_project with the library's fixed device scratch as the reduction
    workspace: nothing is allocated (h is the caller's float64[j] device
    tensor)."""
    import torch
    _dev(w, torch.float64, "w")
    _dev(h, torch.float64, "h")
    if not (1 <= j <= V.ncols) or w.numel() < V.n or h.numel() < j:
        raise ValueError("bad j, w or h size")
    d = V.desc()
    _check(lib().cb_cgs_project_noalloc(C.byref(d), j, _ptr(w), _ptr(h), _stream(stream)),
           "cb_cgs_project_noalloc")
    return h


def cb_cgs_project_noalloc_max_bytes() -> int:
    return int(lib().cb_cgs_project_noalloc_max_bytes())


def cb_cgs_subtract_project(V: Basis, j: int, h, w, out=None, work=None, stream=None):
    """w -= D(V[:, :j]) h, then out[:j] = D(V[:, :j])^T w and out[j] = ||w||^2
    (the first update fused with the second projection)."""
    import torch
    _dev(w, torch.float64, "w")
    _dev(h, torch.float64, "h")
    if not (1 <= j <= V.ncols) or w.numel() < V.n or h.numel() < j:
        raise ValueError("bad j, w or h size")
    if out is None:
        out = torch.empty(j + 1, dtype=torch.float64, device=w.device)
    if work is None:
        work, nbytes = _work(V.n, j + 1, w.device)
    else:
        nbytes = work.numel() * work.element_size()
    d = V.desc()
    _check(lib().cb_cgs_subtract_project(C.byref(d), j, _ptr(h), _ptr(w), _ptr(out), _ptr(work), nbytes,
                                         _stream(stream)), "cb_cgs_subtract_project")
    return out


def cb_cgs_subtract(V: Basis, j: int, h, w, norm2=None, work=None, stream=None):
    import torch
    _dev(w, torch.float64, "w")
    _dev(h, torch.float64, "h")
    if not (1 <= j <= V.ncols) or w.numel() < V.n or h.numel() < j:
        raise ValueError("bad j, w or h size")
    if norm2 is not None and work is None:
        work, nbytes = _work(V.n, 1, w.device)
    else:
        nbytes = 0 if work is None else work.numel() * work.element_size()
    d = V.desc()
    _check(lib().cb_cgs_subtract(C.byref(d), j, _ptr(h), _ptr(w), _ptr(norm2), _ptr(work), nbytes,
                                 _stream(stream)), "cb_cgs_subtract")
    return w


def cb_basis_combine(V: Basis, j: int, y, x, stream=None):
    import torch
    _dev(x, torch.float64, "x")
    _dev(y, torch.float64, "y")
    if not (1 <= j <= V.ncols) or x.numel() < V.n or y.numel() < j:
        raise ValueError("bad j, x or y size")
    d = V.desc()
    _check(lib().cb_basis_combine(C.byref(d), j, _ptr(y), _ptr(x), _stream(stream)), "cb_basis_combine")
    return x


# ---------------------------------------------------------------- sparse matrix
@dataclass
class DeviceCSR:
    n: int
    nnz: int
    row_ptr: "object"
    col: "object"
    val: "object"

    @staticmethod
    def from_host(row_ptr, col, val, device="cuda") -> "DeviceCSR":
        import torch
        rp = torch.as_tensor(row_ptr, dtype=torch.int32).to(device)
        ci = torch.as_tensor(col, dtype=torch.int32).to(device)
        va = torch.as_tensor(val, dtype=torch.float64).to(device)
        n = rp.numel() - 1
        if int(rp[-1]) != ci.numel() or ci.numel() != va.numel():
            raise ValueError("inconsistent CSR arrays")
        return DeviceCSR(n, ci.numel(), rp, ci, va)

    def desc(self) -> cb_csr:
        return cb_csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                      self.val.data_ptr())


def cb_spmv_workspace_bytes(n: int, nnz: int) -> int:
    return int(lib().cb_spmv_workspace_bytes(n, nnz))


def _spmv_work(A: DeviceCSR, device, plan=True):
    """The SpMV workspace: with plan, large enough for the windowed long-row
    gather; without, only the norm's partial sums."""
    import torch
    nbytes = max(8 * (A.n + 1), cb_spmv_workspace_bytes(A.n, A.nnz)) if plan else 8 * (A.n + 1)
    return torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=device), nbytes


def cb_spmv(A: DeviceCSR, x, y=None, norm2=None, stream=None, plan=True):
    import torch
    _dev(x, torch.float64, "x")
    if y is None:
        y = torch.empty(A.n, dtype=torch.float64, device=x.device)
    work, nbytes = _spmv_work(A, x.device, plan)
    d = A.desc()
    _check(lib().cb_spmv(C.byref(d), _ptr(x), _ptr(y), _ptr(norm2), _ptr(work), nbytes, _stream(stream)),
           "cb_spmv")
    return y


def cb_residual(A: DeviceCSR, b, x, r=None, norm2=None, stream=None, plan=True):
    import torch
    _dev(x, torch.float64, "x")
    _dev(b, torch.float64, "b")
    if r is None:
        r = torch.empty(A.n, dtype=torch.float64, device=x.device)
    work, nbytes = _spmv_work(A, x.device, plan)
    d = A.desc()
    _check(lib().cb_residual(C.byref(d), _ptr(b), _ptr(x), _ptr(r), _ptr(norm2), _ptr(work), nbytes,
                             _stream(stream)), "cb_residual")
    return r


# ---------------------------------------------------------------- solver
def cbgmres_workspace_bytes(n: int, m: int, fmt) -> int:
    return int(lib().cbgmres_workspace_bytes(n, m, _fmt(fmt)))


def cb_jacobi_setup(A: DeviceCSR, stream=None):
    """The Jacobi preconditioner's diag_inv (device float64[n]): 1 / a_ii."""
    import torch
    d = torch.empty(A.n, dtype=torch.float64, device="cuda")
    desc = A.desc()
    _check(lib().cb_jacobi_setup(C.byref(desc), _ptr(d), _stream(stream)), "cb_jacobi_setup")
    return d


def cbgmres_precond_workspace_bytes(n: int, nnz: int, m: int, fmt) -> int:
    return int(lib().cbgmres_precond_workspace_bytes(n, nnz, m, _fmt(fmt)))


def cbgmres_solve(A: DeviceCSR, b, x, m: int, tol: float, fmt="frsz2_32", eta: float = 0.0,
                  max_iters: int = 0, max_cycles: int = 0, literal_breakdown: bool = False,
                  workspace=None, history_cap: int = 0, stream=None, check: bool = True,
                  fuse_updates: int = 0, diag_inv=None):
    """Solve A x = b in place on x (x holds x0).  Returns (result dict,
    history numpy array of implicit relative residuals).  Solver outcomes
    (converged, not converged, non-finite) come back in result["status"];
    argument and runtime errors raise CbError.  diag_inv (device float64[n],
    e.g. from cb_jacobi_setup) selects the Jacobi right preconditioner
    M^-1 = diag(diag_inv) (cbgmres_solve_precond)."""
    import numpy as np
    import torch
    _dev(x, torch.float64, "x")
    _dev(b, torch.float64, "b")
    if x.numel() != A.n or b.numel() != A.n:
        raise ValueError("x and b must have n entries")
    opt = cb_options(eta, max_iters, max_cycles, int(literal_breakdown), int(fuse_updates))
    res = cb_result()
    hist = np.zeros(max(history_cap, 1), np.float64)
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    d = A.desc()
    if diag_inv is None:
        st = lib().cbgmres_solve(C.byref(d), _ptr(b), _ptr(x), m, tol, _fmt(fmt), C.byref(opt),
                                 _ptr(workspace), nbytes, hist.ctypes.data_as(C.c_void_p), history_cap,
                                 C.byref(res), _stream(stream))
    else:
        _dev(diag_inv, torch.float64, "diag_inv")
        if diag_inv.numel() != A.n:
            raise ValueError("diag_inv must have n entries")
        M = cb_precond(CB_PRECOND_JACOBI, 0, diag_inv.data_ptr())
        st = lib().cbgmres_solve_precond(C.byref(d), _ptr(b), _ptr(x), m, tol, _fmt(fmt), C.byref(M),
                                         C.byref(opt), _ptr(workspace), nbytes,
                                         hist.ctypes.data_as(C.c_void_p), history_cap, C.byref(res),
                                         _stream(stream))
    if check and st not in (CB_OK, CB_ERR_NOT_CONVERGED, CB_ERR_NONFINITE):
        _check(st, "cbgmres_solve")
    out = res.as_dict()
    out["status"] = st
    return out, hist[:min(history_cap, res.iterations)]


def cbgmres_ir_workspace_bytes(n: int, m: int, fmt) -> int:
    return int(lib().cbgmres_ir_workspace_bytes(n, m, _fmt(fmt)))


def cbgmres_ir_solve(A: DeviceCSR, b, x, m: int, inner_tol: float, tol: float, fmt="frsz2_16",
                     max_outer: int = 100, workspace=None, stream=None, check: bool = True):
    """Iterative refinement in place on x; workspace (optional device tensor
    of at least cbgmres_ir_workspace_bytes) keeps the call allocation-free."""
    import torch
    _dev(x, torch.float64, "x")
    _dev(b, torch.float64, "b")
    res = cb_result()
    d = A.desc()
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    st = lib().cbgmres_ir_solve(C.byref(d), _ptr(b), _ptr(x), m, inner_tol, tol, _fmt(fmt), max_outer,
                                _ptr(workspace), nbytes, C.byref(res), _stream(stream))
    if check and st not in (CB_OK, CB_ERR_NOT_CONVERGED, CB_ERR_NONFINITE):
        _check(st, "cbgmres_ir_solve")
    out = res.as_dict()
    out["status"] = st
    return out


def cb_auto_pick(rel0: float, rel, seconds) -> int:
    """Index of the first candidate with the highest convergence rate
    ln(rel0 / rel[i]) / seconds[i] (host-only rule)."""
    import numpy as np
    r = np.ascontiguousarray(rel, np.float64)
    s = np.ascontiguousarray(seconds, np.float64)
    if r.size != s.size:
        raise ValueError("rel and seconds differ in length")
    return int(lib().cb_auto_pick(rel0, r.ctypes.data_as(C.c_void_p), s.ctypes.data_as(C.c_void_p), r.size))


def _formats_array(candidates):
    fm = (C.c_int32 * max(1, len(candidates)))(*[_fmt(c) for c in candidates])
    return fm


def cbgmres_auto_workspace_bytes(n: int, m: int, probe_steps: int, candidates) -> int:
    fm = _formats_array(candidates)
    return int(lib().cbgmres_auto_workspace_bytes(n, m, probe_steps, C.cast(fm, C.c_void_p), len(candidates)))


def cbgmres_solve_auto(A: DeviceCSR, b, x, m: int, tol: float,
                       candidates=("frsz2_32", "float32", "float16"), probe_steps: int = 20,
                       eta: float = 0.0, max_iters: int = 0, max_cycles: int = 0,
                       literal_breakdown: bool = False, fuse_updates: int = 0, workspace=None,
                       history_cap: int = 0, stream=None, check: bool = True):
    """Solve A x = b in place on x with the basis format picked by probing
    each candidate for probe_steps Arnoldi steps from x0.  Returns (result
    dict with the probes and the continuation under "solve", history of the
    continuation's implicit relative residuals)."""
    import numpy as np
    import torch
    _dev(x, torch.float64, "x")
    _dev(b, torch.float64, "b")
    if x.numel() != A.n or b.numel() != A.n:
        raise ValueError("x and b must have n entries")
    fm = _formats_array(candidates)
    opt = cb_options(eta, max_iters, max_cycles, int(literal_breakdown), int(fuse_updates))
    res = cb_auto_result()
    hist = np.zeros(max(history_cap, 1), np.float64)
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    d = A.desc()
    st = lib().cbgmres_solve_auto(C.byref(d), _ptr(b), _ptr(x), m, tol, C.cast(fm, C.c_void_p), len(candidates),
                                  probe_steps, C.byref(opt), _ptr(workspace), nbytes,
                                  hist.ctypes.data_as(C.c_void_p), history_cap, C.byref(res), _stream(stream))
    if check and st not in (CB_OK, CB_ERR_NOT_CONVERGED, CB_ERR_NONFINITE):
        _check(st, "cbgmres_solve_auto")
    out = res.as_dict()
    out["status"] = st
    return out, hist[:min(history_cap, res.solve.iterations)]


def cbgmres_batch_max_n() -> int:
    return int(lib().cbgmres_batch_max_n())


def cbgmres_batch_max_restart() -> int:
    return int(lib().cbgmres_batch_max_restart())


def cbgmres_batch_workspace_bytes(n: int, m: int, fmt) -> int:
    return int(lib().cbgmres_batch_workspace_bytes(n, m, _fmt(fmt)))


def cbgmres_solve_batch(systems, eta: float = 0.0, max_iters: int = 0, literal_breakdown: bool = False,
                        workspaces=None, stream=None, check: bool = True):
    """Solve several small systems in one launch, one workgroup each.
    systems: list of (A: DeviceCSR, b, x, m, tol, fmt); x is updated in place.
    workspaces: optional list of uint8 device tensors (one per system, at least
    cbgmres_batch_workspace_bytes); allocated here when None.  Returns the
    list of result dicts (status per system)."""
    import torch
    count = len(systems)
    items = (cb_batch_item * max(count, 1))()
    keep = []
    for i, (A, b, x, m, tol, fmt) in enumerate(systems):
        _dev(x, torch.float64, "x")
        _dev(b, torch.float64, "b")
        if x.numel() != A.n or b.numel() != A.n:
            raise ValueError("x and b must have n entries")
        nbytes = cbgmres_batch_workspace_bytes(A.n, m, fmt)
        if workspaces is None:
            ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=x.device)
        else:
            ws = workspaces[i]
        keep.append(ws)
        items[i].A = A.desc()
        items[i].b = b.data_ptr()
        items[i].x = x.data_ptr()
        items[i].workspace = ws.data_ptr()
        items[i].workspace_bytes = ws.numel()
        items[i].m = m
        items[i].format = _fmt(fmt)
        items[i].tol = tol
    opt = cb_options(eta, max_iters, 0, int(literal_breakdown), 0)
    res = (cb_result * max(count, 1))()
    st = lib().cbgmres_solve_batch(items, count, C.byref(opt), res, _stream(stream))
    if check and st not in (CB_OK, CB_ERR_NOT_CONVERGED, CB_ERR_NONFINITE):
        _check(st, "cbgmres_solve_batch")
    out = []
    for i in range(count):
        d = res[i].as_dict()
        out.append(d)
    return out


# ---------------------------------------------------------------- intensity sweep
def cb_intensity_groups(n: int) -> int:
    return int(lib().cb_intensity_groups(n))


def cb_intensity_run(V: Basis, col: int, ops: int, a: float, b: float, partials=None, stream=None):
    """Read column col through its decoder, apply ops steps y <- y*a + b to
    every value, return the per-workgroup sums (device tensor)."""
    import torch
    if partials is None:
        partials = torch.empty(cb_intensity_groups(V.n), dtype=torch.float64, device=V.values.device)
    d = V.desc()
    _check(lib().cb_intensity_run(C.byref(d), col, ops, a, b, _ptr(partials), _stream(stream)), "cb_intensity_run")
    return partials


# ---------------------------------------------------------------- serving
class Server:
    """Continuous-batching solve server (cb_server_*)."""

    def __init__(self, hbm_budget_bytes: int, device: int = 0, lanes: int = 8):
        h = lib().cb_server_create(hbm_budget_bytes, device, lanes)
        if not h:
            raise CbError(CB_ERR_INVALID_ARG, "cb_server_create", lib().cb_last_error().decode())
        self._h = C.c_void_p(h)

    @staticmethod
    def request_bytes(n: int, nnz: int, m: int, fmt) -> int:
        return int(lib().cb_server_request_bytes(n, nnz, m, _fmt(fmt)))

    def submit(self, row_ptr, col, val, b, m: int, tol: float, fmt, x0=None) -> int:
        import numpy as np
        rp = np.ascontiguousarray(row_ptr, np.int32)
        ci = np.ascontiguousarray(col, np.int32)
        va = np.ascontiguousarray(val, np.float64)
        bb = np.ascontiguousarray(b, np.float64)
        x0p = None if x0 is None else np.ascontiguousarray(x0, np.float64)
        t = C.c_uint64()
        _check(lib().cb_server_submit(self._h, rp.size - 1, ci.size, rp.ctypes.data_as(C.c_void_p),
                                      ci.ctypes.data_as(C.c_void_p), va.ctypes.data_as(C.c_void_p),
                                      bb.ctypes.data_as(C.c_void_p),
                                      None if x0p is None else x0p.ctypes.data_as(C.c_void_p),
                                      m, tol, _fmt(fmt), C.byref(t)), "cb_server_submit")
        return int(t.value)

    def poll(self, ticket: int, n: int):
        """None while pending, else (x, result dict, (t_submit, t_start, t_end))."""
        import numpy as np
        x = np.empty(n, np.float64)
        res = cb_result()
        times = np.zeros(3, np.float64)
        st = lib().cb_server_poll(self._h, ticket, x.ctypes.data_as(C.c_void_p), C.byref(res),
                                  times.ctypes.data_as(C.c_void_p))
        if st == CB_PENDING:
            return None
        if st == CB_ERR_NOT_FOUND:
            _check(st, "cb_server_poll")
        out = res.as_dict()
        out["status"] = st
        return x, out, tuple(times)

    def stats(self):
        cb_, q, r = C.c_int64(), C.c_int32(), C.c_int32()
        _check(lib().cb_server_stats(self._h, C.byref(cb_), C.byref(q), C.byref(r)), "cb_server_stats")
        return int(cb_.value), int(q.value), int(r.value)

    def ring_stats(self):
        """(published, joined_running, launches) of the device-resident loop
        for small requests."""
        p, j, n = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().cb_server_ring_stats(self._h, C.byref(p), C.byref(j), C.byref(n)), "cb_server_ring_stats")
        return int(p.value), int(j.value), int(n.value)

    def close(self):
        if self._h:
            lib().cb_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
