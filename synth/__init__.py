"""Seeded synthetic inputs shared by the GPU path's tests, the bench and the
oracle's checks.

This module builds *inputs* only: sparse matrices, right-hand sides, tall-skinny
test bases and serving request streams.  It holds none of the method's
arithmetic (no compression, no Gram-Schmidt, no GMRES).  The one product it
forms, b = A x*, uses scipy's CSR mat-vec as a library primitive so that both
sides receive identical bytes.

The paper evaluates on SuiteSparse CFD matrices (Section V-B, Table 1).  Those
are not available here; the convection-diffusion stencils below stand in for
them (a 7-point 3D stencil has 6.94 nonzeros per row, the same density as the
atmosmod matrices of Table 1).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class CSR:
    """CSR matrix with int32 indices and float64 values (row-major, sorted
    columns within each row)."""
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.row_ptr, self.col, self.val):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def _from_coo(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds 32-bit indexing")
    return CSR(n, row_ptr.astype(np.int32), cols.astype(np.int32),
               np.ascontiguousarray(vals, dtype=np.float64))


def convection_diffusion(N: int, dim: int, beta, nu: float = 1.0) -> CSR:
    """-nu*Laplace(u) + beta . grad(u) on the unit square (dim=2) or cube
    (dim=3) with N interior points per side, h = 1/(N+1), zero Dirichlet
    boundary, central differences, every row scaled by h^2.

    Row index has x fastest.  Coefficients: diagonal 2*dim*nu; the +x/-x
    neighbours get -nu +/- beta_x*h/2 (likewise y, z); neighbours on the
    boundary are dropped.  nnz = 5N^2-4N (2D) or 7N^3-6N^2 (3D).
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    beta = tuple(float(b) for b in beta)
    if len(beta) != dim:
        raise ValueError("beta must have dim entries")
    h = 1.0 / (N + 1)
    n = N ** dim
    idx = np.arange(n, dtype=np.int64)
    coords = [(idx // N ** a) % N for a in range(dim)]
    # the stencil's entries in increasing column order: -z, -y, -x, the
    # diagonal, +x, +y, +z (strides N^2, N, 1), so each row comes out sorted
    # without a sort
    offsets = [(a, -1) for a in reversed(range(dim))] + [None] + [(a, 1) for a in range(dim)]
    k = len(offsets)
    cols = np.empty((n, k), dtype=np.int64)
    vals = np.empty((n, k), dtype=np.float64)
    keep = np.empty((n, k), dtype=bool)
    for t, off in enumerate(offsets):
        if off is None:
            cols[:, t] = idx
            vals[:, t] = 2.0 * dim * nu
            keep[:, t] = True
        else:
            a, sgn = off
            cols[:, t] = idx + sgn * N ** a
            vals[:, t] = -nu + sgn * beta[a] * h / 2.0
            keep[:, t] = (coords[a] + sgn >= 0) & (coords[a] + sgn < N)
    counts = keep.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds 32-bit indexing")
    flat = keep.ravel()
    return CSR(n, row_ptr.astype(np.int32), cols.ravel()[flat].astype(np.int32),
               np.ascontiguousarray(vals.ravel()[flat]))


def rhs_from_solution(A: CSR, x_star: np.ndarray) -> np.ndarray:
    """b = A x* with scipy's CSR mat-vec (input construction only)."""
    return np.ascontiguousarray(A.scipy() @ x_star, dtype=np.float64)


@dataclass
class LinearSystem:
    A: CSR
    b: np.ndarray
    x_star: np.ndarray
    name: str


def plain_2d(N: int = 64, seed: int = 0) -> LinearSystem:
    """2D convection-diffusion, 5-point stencil, diffusion 1, convection 20
    along x; x* ~ U(-1,1) from default_rng(seed); b = A x*."""
    A = convection_diffusion(N, 2, (20.0, 0.0))
    x = np.random.default_rng(seed).uniform(-1.0, 1.0, A.n)
    return LinearSystem(A, rhs_from_solution(A, x), x, f"cd2d_N{N}")


def sweep_3d(N: int = 100, seed: int = 1) -> LinearSystem:
    """3D convection-diffusion, 7-point stencil on N^3, convection (10,5,2);
    x* ~ U(-1,1) from default_rng(seed); b = A x*."""
    A = convection_diffusion(N, 3, (10.0, 5.0, 2.0))
    x = np.random.default_rng(seed).uniform(-1.0, 1.0, A.n)
    return LinearSystem(A, rhs_from_solution(A, x), x, f"cd3d_N{N}")


def column_scaled(base: LinearSystem, decades: float = 3.0, seed: int = 6) -> LinearSystem:
    """The system of `base` with column j of A multiplied by 10^u_j,
    u ~ U(-decades, decades) from default_rng(seed): A' = A S, x*' = S^-1 x*,
    b unchanged.  Badly scaled unknowns, as a diagonal (Jacobi) preconditioner
    is meant to fix."""
    A = base.A
    s = 10.0 ** np.random.default_rng(seed).uniform(-decades, decades, A.n)
    val = np.ascontiguousarray(A.val * s[A.col], dtype=np.float64)
    As = CSR(A.n, A.row_ptr.copy(), A.col.copy(), val)
    xs = base.x_star / s
    return LinearSystem(As, rhs_from_solution(As, xs), xs, base.name + f"_colscaled{decades:g}")


def banded_random(n: int = 1 << 22, per_row: int = 27, half_band: int = 1000,
                  diag_factor: float = 1.2, seed: int = 3) -> LinearSystem:
    """Random nonsymmetric banded matrix: the diagonal plus per_row-1 distinct
    columns drawn uniformly from [i-half_band, i+half_band] intersected with
    [0, n) minus {i}; off-diagonals U(-1,1); diagonal = diag_factor times the
    absolute off-diagonal row sum (strictly diagonally dominant).

    One stream default_rng(seed), in this order: column draws (with
    duplicate rows redrawn in passes until every row is distinct), the
    off-diagonal values, then x* ~ U(-1,1).  b = A x*.
    """
    k = per_row - 1
    if n < 2 * k:
        raise ValueError("matrix too small for the requested row count")
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(0, i - half_band)
    hi = np.minimum(n - 1, i + half_band)
    cnt = hi - lo  # candidates excluding the diagonal
    if np.any(cnt < k):
        raise ValueError("band too narrow for the requested row count")

    def draw(rows_sel: np.ndarray, m: int) -> np.ndarray:
        u = rng.random((rows_sel.size, m))
        off = np.floor(u * cnt[rows_sel, None]).astype(np.int64)
        c = lo[rows_sel, None] + off
        return c + (c >= i[rows_sel, None])

    cols = draw(i, k)
    while True:
        cols.sort(axis=1)
        dup = np.zeros_like(cols, dtype=bool)
        dup[:, 1:] = cols[:, 1:] == cols[:, :-1]
        bad_rows = np.nonzero(dup.any(axis=1))[0]
        if bad_rows.size == 0:
            break
        r, c = np.nonzero(dup[bad_rows])
        fresh = draw(bad_rows[r], 1)[:, 0]
        cols[bad_rows[r], c] = fresh
    offv = rng.uniform(-1.0, 1.0, (n, k))
    diag = diag_factor * np.abs(offv).sum(axis=1)
    rows = np.concatenate([np.repeat(i, k), i])
    allc = np.concatenate([cols.ravel(), i])
    allv = np.concatenate([offv.ravel(), diag])
    A = _from_coo(n, rows, allc, allv)
    x = rng.uniform(-1.0, 1.0, n)
    return LinearSystem(A, rhs_from_solution(A, x), x, f"banded_n{n}")


def basis_columns(n: int = 1 << 24, ncols: int = 101, seed: int = 2):
    """Tall-skinny test basis, yielded one float64 column at a time: one
    stream default_rng(seed); per column z ~ N(0,1)^n, u ~ U(-8,0) per
    32-value block, column = z/sqrt(n) * 10^u (block-wise)."""
    if n % 32:
        raise ValueError("n must be a multiple of 32")
    rng = np.random.default_rng(seed)
    for _ in range(ncols):
        z = rng.standard_normal(n)
        u = rng.uniform(-8.0, 0.0, n // 32)
        z /= np.sqrt(n)
        z *= np.repeat(10.0 ** u, 32)
        yield z


def basis_probe_vector(n: int = 1 << 24, seed: int = 2) -> np.ndarray:
    """The vector w that the tall-skinny basis is projected against:
    drawn after the basis columns from a separate stream default_rng(seed+1000),
    w ~ N(0,1)/sqrt(n)."""
    return np.random.default_rng(seed + 1000).standard_normal(n) / np.sqrt(n)


FORMATS = ("float64", "float32", "float16", "frsz2_16", "frsz2_21", "frsz2_32")


@dataclass
class Request:
    rid: int
    arrival_s: float
    dim: int
    N: int
    fmt: str
    tol: float
    m: int
    seed: int

    @property
    def n(self) -> int:
        return self.N ** self.dim

    def system(self) -> LinearSystem:
        beta = (20.0, 0.0) if self.dim == 2 else (10.0, 5.0, 2.0)
        A = convection_diffusion(self.N, self.dim, beta)
        x = np.random.default_rng(self.seed).uniform(-1.0, 1.0, A.n)
        return LinearSystem(A, rhs_from_solution(A, x), x, f"req{self.rid}")


def serving_requests(count: int = 512, rate_per_s: float = 200.0, seed: int = 4,
                     n_min: int = 32 ** 2, n_max: int = 128 ** 3,
                     formats=("float32", "frsz2_16", "frsz2_21", "frsz2_32")) -> list:
    """Seeded solve-request stream: Poisson arrivals (exponential gaps at
    rate_per_s); dim 2 or 3 with p=1/2; target n log-uniform in [n_min, n_max]
    and grid side round(n^(1/dim)) (at least 4); basis format uniform over
    formats; tol log-uniform in [1e-12, 1e-8]; restart m uniform in 30..100;
    x* drawn from default_rng(1000 + id)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, count)
    arrivals = np.cumsum(gaps) - gaps[0]
    dims = rng.integers(2, 4, count)
    logn = rng.uniform(np.log(n_min), np.log(n_max), count)
    fmts = rng.integers(0, len(formats), count)
    logtol = rng.uniform(np.log(1e-12), np.log(1e-8), count)
    ms = rng.integers(30, 101, count)
    out = []
    for r in range(count):
        d = int(dims[r])
        N = max(4, int(round(np.exp(logn[r] / d))))
        out.append(Request(r, float(arrivals[r]), d, N, formats[int(fmts[r])],
                           float(np.exp(logtol[r])), int(ms[r]), 1000 + r))
    return out
