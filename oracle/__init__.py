"""Python view of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  The
oracle shares no code with the HIP library.

Basis format numbers: 0 float64, 1 float32, 2 float16, 3 frsz2_16, 4 frsz2_21,
5 frsz2_32.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FORMATS = {"float64": 0, "float32": 1, "float16": 2, "frsz2_16": 3, "frsz2_21": 4, "frsz2_32": 5}
# FRSZ2 with blocks of 64 values (6, 7), and any l with blocks of 32 (64 + l) or 64 (128 + l)
FORMATS_B64 = {"frsz2b64_16": 6, "frsz2b64_32": 7}
FRSZ2_BITS = {3: 16, 4: 21, 5: 32, 6: 16, 7: 32, **{64 + l: l for l in range(3, 33)},
              **{128 + l: l for l in range(3, 33)}}


def block_size(fmt) -> int:
    f = _fmt(fmt)
    return 64 if f in (6, 7) or 128 + 3 <= f <= 128 + 32 else 32


def build() -> str:
    """Compile oracle.c with gcc (no fast-math, no FP contraction)."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                    "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32, d = C.c_int64, C.c_int, C.c_double
        sig = {
            "or_frsz2_encode": (i32, [P, i64, i32, P, P]),
            "or_frsz2_decode": (None, [P, P, i64, i32, P]),
            "or_frsz2_decode_value": (d, [P, P, i64, i32]),
            "or_frsz2_encode_bs": (i32, [P, i64, i32, i32, P, P]),
            "or_frsz2_decode_bs": (None, [P, P, i64, i32, i32, P]),
            "or_frsz2_decode_value_bs": (d, [P, P, i64, i32, i32]),
            "or_basis_exp_words": (i64, [i32, i64]),
            "or_f16_from_f64": (C.c_uint16, [d]),
            "or_f64_from_f16": (d, [C.c_uint16]),
            "or_basis_col_bytes": (i64, [i32, i64]),
            "or_basis_encode": (i32, [i32, P, i64, P, P]),
            "or_basis_decode": (None, [i32, P, P, i64, P]),
            "or_dot": (d, [i64, P, P]),
            "or_nrm2": (d, [i64, P]),
            "or_spmv": (None, [i64, P, P, P, P, P]),
            "or_cgs_project": (None, [i64, i32, P, i64, P, P]),
            "or_cgs_subtract": (None, [i64, i32, P, i64, P, P]),
            "or_gmres": (i32, [i64, P, P, P, P, P, i32, d, i32, P, P, P, i64]),
            "or_gmres_cycle": (None, [i64, P, P, P, P, d, i32, i32, d, i32, d, i32, P, P, P, P,
                                      P, P, P, P, P]),
            "or_ir_solve": (i32, [i64, P, P, P, P, P, i32, d, d, i32, i32, P]),
            "or_gmres_pc": (i32, [i64, P, P, P, P, P, P, i32, d, i32, P, P, P, i64]),
            "or_jacobi_diag_inv": (None, [i64, P, P, P, P]),
            "or_dense_solve": (i32, [i32, P, P]),
            "or_rounding_is_nearest": (i32, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def frsz2_any(l: int) -> int:
    """Format number of FRSZ2 with l bits, 3 <= l <= 32 (64 + l)."""
    if not 3 <= l <= 32:
        raise ValueError("l must lie in [3, 32]")
    return 64 + l


def _fmt(fmt) -> int:
    """A format name or number: the names above, "frsz2_<l>" for any other l
    in [3, 32], "frsz2g_<l>" for the number 64 + l of any l; with blocks of 64,
    "frsz2b64_<l>" (128 + l unless l is 16 or 32) and "frsz2b64g_<l>" (128 + l)."""
    if not isinstance(fmt, str):
        return int(fmt)
    if fmt in FORMATS:
        return FORMATS[fmt]
    if fmt in FORMATS_B64:
        return FORMATS_B64[fmt]
    if fmt.startswith("frsz2b64_") or fmt.startswith("frsz2b64g_"):
        return 64 + frsz2_any(int(fmt.split("_")[1]))
    if fmt.startswith("frsz2_") or fmt.startswith("frsz2g_"):
        return frsz2_any(int(fmt.split("_")[1]))
    raise KeyError(fmt)


def nblocks(n: int) -> int:
    return (n + 31) // 32


# ---------------------------------------------------------------- FRSZ2 codec
def frsz2_encode(x: np.ndarray, bits: int, bs: int = 32):
    """Blocks of bs (32 or 64) values.  Returns (exps uint32[ceil(n/bs)],
    words uint32[(bs/32)*bits*ceil(n/bs)], nonfinite)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    nb = (x.size + bs - 1) // bs
    exps = np.zeros(nb, np.uint32)
    words = np.zeros(nb * bits * (bs // 32), np.uint32)
    if bs == 32:
        bad = lib().or_frsz2_encode(_p(x), x.size, bits, _p(exps), _p(words))
    else:
        bad = lib().or_frsz2_encode_bs(_p(x), x.size, bits, bs, _p(exps), _p(words))
    return exps, words, bool(bad)


def frsz2_decode(exps: np.ndarray, words: np.ndarray, n: int, bits: int, bs: int = 32) -> np.ndarray:
    exps = np.ascontiguousarray(exps, dtype=np.uint32)
    words = np.ascontiguousarray(words, dtype=np.uint32)
    out = np.empty(n, np.float64)
    if bs == 32:
        lib().or_frsz2_decode(_p(exps), _p(words), n, bits, _p(out))
    else:
        lib().or_frsz2_decode_bs(_p(exps), _p(words), n, bits, bs, _p(out))
    return out


def frsz2_decode_value(exps: np.ndarray, words: np.ndarray, i: int, bits: int, bs: int = 32) -> float:
    exps = np.ascontiguousarray(exps, dtype=np.uint32)
    words = np.ascontiguousarray(words, dtype=np.uint32)
    if bs == 32:
        return lib().or_frsz2_decode_value(_p(exps), _p(words), i, bits)
    return lib().or_frsz2_decode_value_bs(_p(exps), _p(words), i, bits, bs)


# ---------------------------------------------------------------- casts
def f16_bits(x: float) -> int:
    return int(lib().or_f16_from_f64(float(x)))


def f16_value(h: int) -> float:
    return float(lib().or_f64_from_f16(int(h)))


# ---------------------------------------------------------------- basis columns
def col_bytes(fmt, n: int) -> int:
    return int(lib().or_basis_col_bytes(_fmt(fmt), n))


def exp_words(fmt, n: int) -> int:
    return int(lib().or_basis_exp_words(_fmt(fmt), n))


def basis_encode(fmt, x: np.ndarray):
    """Q(x) for one column.  Returns (values as uint8 bytes, exps uint32, nonfinite)."""
    f = _fmt(fmt)
    x = np.ascontiguousarray(x, dtype=np.float64)
    vals = np.zeros(col_bytes(f, x.size), np.uint8)
    exps = np.zeros(max(1, exp_words(f, x.size)), np.uint32)
    bad = lib().or_basis_encode(f, _p(x), x.size, _p(vals), _p(exps))
    return vals, exps[:exp_words(f, x.size)] if exp_words(f, x.size) else exps, bool(bad)


def basis_decode(fmt, vals: np.ndarray, exps: np.ndarray, n: int) -> np.ndarray:
    f = _fmt(fmt)
    vals = np.ascontiguousarray(vals)
    exps = np.ascontiguousarray(exps, dtype=np.uint32)
    out = np.empty(n, np.float64)
    lib().or_basis_decode(f, _p(vals), _p(exps), n, _p(out))
    return out


# ---------------------------------------------------------------- FP64 kernels
def dot(a, b) -> float:
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    return lib().or_dot(a.size, _p(a), _p(b))


def nrm2(a) -> float:
    a = np.ascontiguousarray(a, np.float64)
    return lib().or_nrm2(a.size, _p(a))


def spmv(A, x) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    y = np.empty(A.n, np.float64)
    lib().or_spmv(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(x), _p(y))
    return y


def cgs_project(Vdec: np.ndarray, w: np.ndarray) -> np.ndarray:
    """h = V^T w for the columns of Vdec (n x j, Fortran order)."""
    V = np.asfortranarray(Vdec, np.float64)
    w = np.ascontiguousarray(w, np.float64)
    n, j = V.shape
    h = np.empty(j, np.float64)
    lib().or_cgs_project(n, j, _p(V), n, _p(w), _p(h))
    return h


def cgs_subtract(Vdec: np.ndarray, h: np.ndarray, w: np.ndarray) -> np.ndarray:
    V = np.asfortranarray(Vdec, np.float64)
    h = np.ascontiguousarray(h, np.float64)
    out = np.array(w, dtype=np.float64, copy=True)
    n, j = V.shape
    lib().or_cgs_subtract(n, j, _p(V), n, _p(h), _p(out))
    return out


# ---------------------------------------------------------------- solvers
class _Stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("reorths", C.c_int32),
                ("breakdowns", C.c_int32), ("converged", C.c_int32), ("status", C.c_int32),
                ("rel_residual", C.c_double), ("implicit_rel_residual", C.c_double)]


class _Options(C.Structure):
    _fields_ = [("eta", C.c_double), ("max_iters", C.c_int32), ("max_cycles", C.c_int32),
                ("literal_breakdown", C.c_int32)]


class _IRStats(C.Structure):
    _fields_ = [("outer", C.c_int32), ("iterations", C.c_int32), ("converged", C.c_int32),
                ("status", C.c_int32), ("rel_residual", C.c_double)]


class _CycleInfo(C.Structure):
    _fields_ = [("steps", C.c_int32), ("reorths", C.c_int32), ("breakdown", C.c_int32),
                ("status", C.c_int32), ("gabs", C.c_double)]


@dataclass
class Cycle:
    steps: int
    reorths: int
    breakdown: bool
    status: int
    gabs: float
    enc: np.ndarray      # uint8[(m+1), col_bytes]: Q(v_i) per column
    exps: np.ndarray     # uint32[(m+1), ceil(n/32)]
    Vdec: np.ndarray     # float64 n x (m+1), Fortran order: D(Q(v_i))
    R: np.ndarray        # (m+1) x m rotated Hessenberg (upper triangle valid)
    Hraw: np.ndarray     # (m+1) x m unrotated Hessenberg
    Vfp: np.ndarray      # float64 n x (m+1), Fortran order: the FP64 v_i (SpMV input, Q's input)
    y: np.ndarray        # least-squares solution, length steps
    gabs_hist: np.ndarray


def gmres_cycle(A, r, beta: float, m: int, fmt="float64", eta: float = 0.7071067811865476,
                literal_breakdown: bool = False, tol_abs: float = 0.0,
                max_steps: int = 1 << 30) -> Cycle:
    """One GMRES cycle (Fig. 1 steps 1-17) starting from residual r."""
    f = _fmt(fmt)
    r = np.ascontiguousarray(r, np.float64)
    n = A.n
    cb = col_bytes(f, n)
    enc = np.zeros((m + 1, cb), np.uint8)
    exps = np.zeros((m + 1, max(1, nblocks(n))), np.uint32)
    Vdec = np.zeros((n, m + 1), np.float64, order="F")
    R = np.zeros((m + 1, m), np.float64, order="F")
    Hraw = np.zeros((m + 1, m), np.float64, order="F")
    Vfp = np.zeros((n, m + 1), np.float64, order="F")
    y = np.zeros(m, np.float64)
    hist = np.zeros(m, np.float64)
    ci = _CycleInfo()
    lib().or_gmres_cycle(n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(r), beta, m, f, eta,
                         int(literal_breakdown), tol_abs, max_steps, _p(enc), _p(exps),
                         _p(Vdec), _p(R), _p(Hraw), _p(Vfp), _p(y), _p(hist), C.byref(ci))
    return Cycle(ci.steps, ci.reorths, bool(ci.breakdown), ci.status, ci.gabs, enc, exps,
                 Vdec, R, Hraw, Vfp, y[:ci.steps].copy(), hist[:ci.steps].copy())


@dataclass
class GmresResult:
    x: np.ndarray
    iterations: int
    restarts: int
    reorths: int
    breakdowns: int
    converged: bool
    status: int
    rel_residual: float
    implicit_rel_residual: float
    history: np.ndarray


def gmres(A, b, m: int, tol: float, fmt="float64", x0=None, eta: float = 0.7071067811865476,
          max_iters: int = 20000, max_cycles: int = 0, literal_breakdown: bool = False,
          hist_cap: int = 0, dinv=None) -> GmresResult:
    """Restarted GMRES(m); dinv (optional) is the Jacobi right preconditioner
    M^-1 = diag(dinv) of Fig. 1 steps 3 and 17."""
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros(A.n, np.float64) if x0 is None else np.array(x0, np.float64, copy=True)
    st = _Stats()
    opt = _Options(eta, max_iters, max_cycles, int(literal_breakdown))
    hist = np.zeros(max(hist_cap, 1), np.float64)
    dv = None if dinv is None else np.ascontiguousarray(dinv, np.float64)
    lib().or_gmres_pc(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), None if dv is None else _p(dv), _p(b),
                      _p(x), m, tol, _fmt(fmt), C.byref(opt), C.byref(st), _p(hist), hist_cap)
    return GmresResult(x, st.iterations, st.restarts, st.reorths, st.breakdowns,
                       bool(st.converged), st.status, st.rel_residual,
                       st.implicit_rel_residual, hist[:min(hist_cap, st.iterations)])


def jacobi(A) -> np.ndarray:
    """dinv[i] = 1 / a_ii (1 where the diagonal is missing, zero or not finite)."""
    out = np.empty(A.n, np.float64)
    lib().or_jacobi_diag_inv(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(out))
    return out


@dataclass
class IRResult:
    x: np.ndarray
    outer: int
    iterations: int
    converged: bool
    status: int
    rel_residual: float


def ir_solve(A, b, m: int, inner_tol: float, tol: float, fmt="frsz2_16", x0=None,
             max_outer: int = 100) -> IRResult:
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros(A.n, np.float64) if x0 is None else np.array(x0, np.float64, copy=True)
    st = _IRStats()
    lib().or_ir_solve(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(b), _p(x), m, inner_tol,
                      tol, _fmt(fmt), max_outer, C.byref(st))
    return IRResult(x, st.outer, st.iterations, bool(st.converged), st.status, st.rel_residual)


def dense_solve(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    A = np.array(a, dtype=np.float64, order="F", copy=True)
    x = np.array(b, dtype=np.float64, copy=True)
    if lib().or_dense_solve(A.shape[0], _p(A), _p(x)):
        raise np.linalg.LinAlgError("singular")
    return x


# ---------------------------------------------------------------- format chosen by probing
# The autotuning named in the paper's conclusions (Section VIII): run each
# candidate method for a short probe, measure its convergence per unit time,
# continue with the best.  The reading used here: a probe is a GMRES(p) run
# from x0 capped at p Arnoldi steps; its rate is the natural-log decrease of
# the explicit relative residual per second of wall time; the first candidate
# with the highest rate wins; a probe that met the tolerance wins outright.
def auto_rate(rel0: float, rel: float, seconds: float) -> float:
    """ln(rel0 / rel) / seconds; -inf when the probe did not lower the
    residual or produced Inf/NaN; +inf when it reached a zero residual."""
    import math
    if not math.isfinite(rel) or rel < 0.0 or not rel < rel0:
        return -math.inf
    if rel == 0.0 or not seconds > 0.0:
        return math.inf
    return math.log(rel0 / rel) / seconds


def auto_pick(rel0: float, rel, seconds) -> int:
    """Index of the first candidate with the highest auto_rate."""
    rates = [auto_rate(rel0, r, t) for r, t in zip(rel, seconds)]
    best = 0
    for i, r in enumerate(rates):
        if r > rates[best]:
            best = i
    return best


def auto_probe(A, b, x0, fmt, probe_steps: int, tol: float, eta: float = 0.7071067811865476,
               literal_breakdown: bool = False) -> GmresResult:
    """One candidate's probe: GMRES(probe_steps) from x0, at most probe_steps
    Arnoldi steps; rel_residual is the explicit residual after it."""
    return gmres(A, b, probe_steps, tol, fmt, x0=x0, eta=eta, max_iters=probe_steps,
                 literal_breakdown=literal_breakdown)
