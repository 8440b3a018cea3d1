/*
 * cbgmres.h -- C ABI of libcbgmres.so: restarted GMRES with a compressed
 * Krylov basis (FRSZ2 block compression or low-precision casts) on one
 * MI355X (gfx950) GPU.
 *
 * Method: GMRES with classical Gram-Schmidt and one conditional
 * re-orthogonalisation, restarted every m steps (the paper's Fig. 1), whose
 * basis vectors are stored compressed and decompressed inside the
 * Gram-Schmidt projections and the solution update; everything else (SpMV,
 * dot products, norms, Givens rotations, the solution) is FP64.  FRSZ2
 * (Section IV) groups 32 consecutive values under their largest biased IEEE
 * exponent and keeps, per value, a sign bit and the leading l-1 bits of the
 * significand aligned to that exponent (Eq. 2).
 *
 * Conventions shared by every entry point:
 *  - Pointers are DEVICE pointers (memory on the current HIP device) unless
 *    the name ends in _host.  The caller owns every buffer passed in; the
 *    library never frees caller memory and never keeps a pointer past the
 *    call (except the server, which copies its inputs).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Entry points documented as asynchronous only enqueue work on it.
 *  - Return value: a cb_status.  Nothing is thrown across the ABI.  On an
 *    error no kernel has been enqueued and cb_last_error() (thread-local)
 *    describes the cause.
 *  - Sizes n are row counts, 1 <= n <= 2^31 - 4096 (so that every 32-bit
 *    row index a kernel forms, including its padding to 2048-row groups,
 *    stays below 2^31); indices are 32-bit.
 *  - Alignment: basis values / FRSZ2 words and the FP64 vectors the basis
 *    kernels read or write (w, x, v_out, a solve's x) are accessed in 16-byte
 *    pieces and must be 16-byte aligned; other arrays need their element's
 *    alignment.  Every hipMalloc (and torch) allocation is 256-byte aligned.
 *    A misaligned pointer returns CB_ERR_INVALID_ARG.
 */
#ifndef CBGMRES_H
#define CBGMRES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cb_status {
    CB_OK = 0,
    CB_ERR_INVALID_ARG = 1,      /* null pointer, bad size, bad format ... */
    CB_ERR_UNSUPPORTED_BITS = 2, /* FRSZ2 bit width outside 3..32 */
    CB_ERR_NONFINITE = 3,        /* Inf/NaN met in a solve */
    CB_ERR_NOT_CONVERGED = 4,    /* iteration or cycle cap reached */
    CB_ERR_WORKSPACE = 5,        /* workspace too small */
    CB_ERR_OVER_BUDGET = 6,      /* server request larger than the HBM budget */
    CB_ERR_HIP = 7,              /* a HIP runtime call failed */
    CB_PENDING = 8,              /* server ticket not finished yet */
    CB_ERR_NOT_FOUND = 9         /* unknown server ticket */
} cb_status;

/* Basis storage formats.  float16 is IEEE binary16 rounded to nearest-even
 * in one step from float64; float32 likewise.  frsz2_l is FRSZ2 with block
 * size 32 and l bits per value. */
typedef enum cb_basis_format {
    CB_F64 = 0,
    CB_F32 = 1,
    CB_F16 = 2,
    CB_FRSZ2_16 = 3,
    CB_FRSZ2_21 = 4,
    CB_FRSZ2_32 = 5,
    CB_FRSZ2_16_B64 = 6,  /* frsz2_16 and frsz2_32 with blocks of 64 values */
    CB_FRSZ2_32_B64 = 7
} cb_basis_format;

/* FRSZ2 with any l in [3, 32] (l is a free parameter of the format, Section
 * IV-A): format number CB_FRSZ2_BITS(l), run by a generic codec whose lanes
 * walk their codes with a runtime bit offset.  The storage layout and the
 * codes are those of the fixed formats: CB_FRSZ2_BITS(16), (21) and (32)
 * store the same bits as CB_FRSZ2_16, _21 and _32, which have specialised
 * (faster) kernels.  Every entry point that takes a format accepts these and
 * the block-64 formats below, except the batched small-system solver. */
#define CB_FRSZ2_GENERIC_BASE 64
#define CB_FRSZ2_BITS(l) (CB_FRSZ2_GENERIC_BASE + (l))

/* Blocks of 64 values (one wavefront's 64 lanes x 8 values cover 8 blocks):
 * 64 consecutive values share one exponent word and their codes form one
 * 64 l-bit stream of 2 l words; a column has ceil(n/64) exponent words and
 * rows n .. 64*ceil(n/64)-1 stored as +0.0.  The paper fixes 32 (Section
 * IV-C, item 2; other sizes ran slower end to end on its GPU); these formats
 * let the trade-off be measured on a 64-wide machine.  CB_FRSZ2_16_B64 and
 * CB_FRSZ2_32_B64 have specialised kernels; CB_FRSZ2_B64_BITS(l), any l in
 * [3, 32], runs the generic codec. */
#define CB_FRSZ2_B64_GENERIC_BASE 128
#define CB_FRSZ2_B64_BITS(l) (CB_FRSZ2_B64_GENERIC_BASE + (l))

const char* cb_status_string(int status);
const char* cb_last_error(void);

/* ======================================================================
 * FRSZ2 codec (Section IV-A compression steps 1-6, Section IV-B
 * decompression steps 1-4, storage layout of Eq. 3).
 *
 * Layout of a compressed vector of n values, nb = ceil(n/32) blocks:
 *   exps[nb]     uint32: the block's largest biased IEEE exponent field E
 *                (0..2047; the value grid is 2^(max(E,1)-1023-(l-2)));
 *   words[l*nb]  uint32: block b owns words [b*l, (b+1)*l), holding the
 *                32 l-bit codes of the block as one little-endian bit stream,
 *                code q at bits [q*l, (q+1)*l); a code is sign << (l-1) |
 *                floor(|x| / grid), i.e. the significand truncated to l-1
 *                bits after alignment to E.
 * The exponent and value arrays are separate (Section IV-C, item 5).
 * A partial last block is encoded as if padded with +0.0.
 * ====================================================================== */

/* ceil(n/32) */
int64_t frsz2_exponent_words(int64_t n);
/* bits * ceil(n/32), or -1 for a width outside 3..32 */
int64_t frsz2_value_words(int64_t n, int bits);

/* Compress x[n] (float64) into exps/words.  3 <= bits <= 32 (16, 21 and 32
 * use the specialised kernels).
 * nonfinite_flag (nullable, device int32) is set to 1 -- never cleared -- when
 * a block holds Inf or NaN; that block's words are then unspecified.
 * Asynchronous. */
int frsz2_compress(const double* x, int64_t n, int bits, uint32_t* exps, uint32_t* words,
                   int32_t* nonfinite_flag, void* stream);

/* Decompress n values into x[n] (float64).  Every code decodes exactly (the
 * values are multiples of 2^-1074 below 2^1024).  Asynchronous. */
int frsz2_decompress(const uint32_t* exps, const uint32_t* words, int64_t n, int bits,
                     double* x, void* stream);

/* ======================================================================
 * Compressed basis V = [v_0 .. v_{ncols-1}] (Fig. 1, the highlighted
 * storage sites) and the fused hot-path primitives.
 *
 * Column c of `values` starts at byte c * cb_basis_column_bytes(format, n)
 * (the column's data rounded up to a multiple of 256 bytes); frsz2 columns
 * keep their exponents at exps + c * cb_basis_exponent_words.  Rows
 * n .. 32*ceil(n/32)-1 of every column are stored as +0.0.  Float columns
 * begin with float64/float32/binary16 arrays of 32*ceil(n/32) entries; frsz2
 * columns with the `words` array above.  `exps` is ignored (may be NULL) for
 * float formats.
 * ====================================================================== */
typedef struct cb_basis {
    int32_t format;   /* cb_basis_format */
    int32_t n;        /* rows */
    int32_t ncols;    /* capacity in columns */
    int32_t reserved; /* 0 */
    void* values;     /* device */
    uint32_t* exps;   /* device, frsz2 only */
} cb_basis;

int64_t cb_basis_column_bytes(int format, int64_t n);   /* column stride */
int64_t cb_basis_exponent_words(int format, int64_t n); /* 0 for float formats */

/* Normalise and store one basis column (Fig. 1 steps 1, 13-14):
 * v = w / *divisor with IEEE division per entry (divisor: device double;
 * NULL stores w unchanged); column `col` := Q(v); if v_out is non-NULL it
 * receives the float64 v (n entries).  w and v_out may alias.
 * nonfinite_flag as for frsz2_compress.  Asynchronous. */
int cb_basis_store(const cb_basis* V, int32_t col, const double* w, const double* divisor,
                   double* v_out, int32_t* nonfinite_flag, void* stream);

/* x[n] := D(column col), float64.  Asynchronous. */
int cb_basis_load(const cb_basis* V, int32_t col, double* x, void* stream);

/* Bytes of reduction workspace needed by the primitives below for n rows and
 * up to ncols columns: an 8 KB header (ticket counters that the call clears
 * itself) followed by per-workgroup partial sums.  Calls that share a
 * workspace must run in stream order. */
int64_t cb_reduce_workspace_bytes(int32_t n, int32_t ncols);

/* Classical Gram-Schmidt projection with decompression fused into the read
 * (Fig. 1 step 5, first half): h[i] = sum_k D(v_i)[k] * w[k] for
 * i = 0..j-1 (1 <= j <= 513), all against the same w.  h: device float64[j].  The sum over k
 * runs in a fixed order that depends on n only (deterministic).
 * Asynchronous. */
int cb_cgs_project(const cb_basis* V, int32_t j, const double* w, double* h, void* work,
                   size_t work_bytes, void* stream);

/* The projection of cb_cgs_project for callers that cannot allocate device
 * memory (code under stream capture, serving loops and harnesses that forbid
 * hipMalloc): same arguments and result, computed by the same kernels, but
 * the reduction workspace is a fixed library-owned device array of
 * cb_cgs_project_noalloc_max_bytes() bytes (2.0 MiB; every valid n and
 * 1 <= j <= 513 fits), so the call allocates nothing.  The array's device
 * address is looked up on the first call on each device (that call may make
 * the HIP runtime load the library's code on the device); each device holds
 * its own copy until the process ends.  The call clears the array's ticket
 * counters itself with a fill kernel.  All calls on one device share the
 * array: calls that may overlap on one device (different streams, or host
 * threads without stream order) race and give wrong results; calls in one
 * stream's order are safe.  CB_ERR_WORKSPACE if a call needed more than the
 * fixed size; other errors as for cb_cgs_project.  Asynchronous. */
int cb_cgs_project_noalloc(const cb_basis* V, int32_t j, const double* w, double* h, void* stream);
int64_t cb_cgs_project_noalloc_max_bytes(void);

/* Classical Gram-Schmidt update with decompression fused in (Fig. 1 step 5,
 * second half, and step 6): w[k] -= sum_{i<j} h[i] * D(v_i)[k] (1 <= j <= 513;
 * each row's correction summed over i in order, then subtracted), and, if
 * norm2 is non-NULL, *norm2 = ||w||^2 after the update (device double).
 * Asynchronous. */
int cb_cgs_subtract(const cb_basis* V, int32_t j, const double* h, double* w, double* norm2,
                    void* work, size_t work_bytes, void* stream);

/* The first Gram-Schmidt update fused with the second projection (Fig. 1
 * steps 5b, 6 and 8): w[k] -= sum_{i<j} h[i] * D(v_i)[k] (each row's
 * correction summed over i first, then subtracted), then
 * out[i] = sum_k D(v_i)[k] * w[k] for i < j on the updated w, and
 * out[j] = ||w||^2 (1 <= j <= 512).  out: device float64[j + 1].  work as for
 * cb_cgs_project with j + 1 columns.  Sums run in fixed orders that depend on
 * (n, j) only.  Asynchronous. */
int cb_cgs_subtract_project(const cb_basis* V, int32_t j, const double* h, double* w, double* out,
                            void* work, size_t work_bytes, void* stream);

/* Solution update with decompression fused in (Fig. 1 step 17):
 * x[k] += sum_{i<j} y[i] * D(v_i)[k] (1 <= j <= 513).  y: device float64[j].
 * Asynchronous. */
int cb_basis_combine(const cb_basis* V, int32_t j, const double* y, double* x, void* stream);

/* ======================================================================
 * Sparse matrix (CSR, int32 indices sorted within rows, float64 values).
 * ====================================================================== */
typedef struct cb_csr {
    int32_t n;   /* rows = columns */
    int32_t nnz;
    const int32_t* row_ptr; /* device, n+1 */
    const int32_t* col;     /* device, nnz */
    const double* val;      /* device, nnz */
} cb_csr;

/* Workspace bytes of cb_spmv / cb_residual for a matrix of n rows and nnz
 * entries: the norm's partial sums, and for rows of more than 8 entries on
 * average the column window of every 512-row block (with it, such a SpMV
 * stages each block's window of x in LDS instead of gathering x from memory;
 * the results are the same).  -1 on a bad size. */
int64_t cb_spmv_workspace_bytes(int32_t n, int32_t nnz);

/* y = A x (Fig. 1 step 3, M = I) and, if norm2 != NULL, *norm2 = ||y||^2
 * (step 4).  The norm needs a device workspace of at least 8 * (n + 1) bytes;
 * a workspace of cb_spmv_workspace_bytes(n, nnz) bytes (8-byte aligned) also
 * lets long rows use the windowed gather, the plan being formed in it by the
 * call.  Column indices must lie in [0, n).  Asynchronous. */
int cb_spmv(const cb_csr* A, const double* x, double* y, double* norm2, void* work,
            size_t work_bytes, void* stream);

/* r = b - A x and, if norm2 != NULL, *norm2 = ||r||^2 (Fig. 1 step 1);
 * workspace as for cb_spmv.  Asynchronous. */
int cb_residual(const cb_csr* A, const double* b, const double* x, double* r, double* norm2,
                void* work, size_t work_bytes, void* stream);

/* ======================================================================
 * Solver (Fig. 1; stopping rule Eq. 4).
 * ====================================================================== */
typedef struct cb_options {
    double eta;                /* re-orthogonalisation threshold (Fig. 1 step 7); <= 0: 1/sqrt(2) */
    int32_t max_iters;         /* cap on Arnoldi steps; <= 0: 20000 */
    int32_t max_cycles;        /* cap on restart cycles; 0 = none.  When it is hit the
                                  solve returns after the x update without a final
                                  explicit residual (status CB_ERR_NOT_CONVERGED) */
    int32_t literal_breakdown; /* 1: step 12 compares h_{j+1,j} with eta * omega as
                                  printed; 0 (default): with eta times the norm before
                                  the re-orthogonalisation pass */
    int32_t fuse_updates;      /* first Gram-Schmidt update fused with the second
                                  projection (formed speculatively, dropped when step 7
                                  does not ask for it): 0 (default) per cycle, when the
                                  last cycle re-orthogonalised at least half its steps
                                  (never for a float64 basis); 1 never; 2 always.  The
                                  arithmetic is the same either way. */
} cb_options;

typedef struct cb_result {
    int32_t iterations;          /* Arnoldi steps (SpMVs inside cycles) */
    int32_t restarts;            /* cycles run */
    int32_t reorths;             /* steps that ran the second Gram-Schmidt pass */
    int32_t breakdowns;          /* cycles ended by the breakdown test */
    int32_t converged;           /* 1 iff the explicit residual met tol */
    int32_t status;              /* cb_status of the solve */
    double rel_residual;         /* last explicit ||b - A x|| / ||b||; -1 if not evaluated */
    double implicit_rel_residual;/* last |g_{j+1}| / ||b|| */
    double seconds;              /* wall time of the solve */
    double basis_bytes;          /* algorithmic bytes read+written in the basis kernels */
} cb_result;

/* Device workspace bytes cbgmres_solve needs for n rows, restart m, format. */
int64_t cbgmres_workspace_bytes(int32_t n, int32_t m, int format);

/* Solve A x = b.  x holds x0 on entry and the iterate on return (device,
 * float64[n]).  1 <= m <= 512 is the restart length, tol > 0 the relative residual
 * ||b - A x|| <= tol ||b|| that ends the solve (checked on the explicit
 * residual at a restart, Eq. 4; the implicit residual only ends a cycle
 * early).  workspace may be NULL (the library allocates and frees it) or a
 * device buffer of at least cbgmres_workspace_bytes.  history_host (nullable)
 * receives up to history_cap implicit relative residuals, one per step.
 * result_host receives the statistics.  Synchronous: returns when the solve
 * is done.  b = 0 gives x = 0 after 0 iterations.  A cap reached returns
 * CB_ERR_NOT_CONVERGED with x the last iterate; Inf/NaN returns
 * CB_ERR_NONFINITE. */
int cbgmres_solve(const cb_csr* A, const double* b, double* x, int32_t m, double tol, int format,
                  const cb_options* opt, void* workspace, size_t workspace_bytes,
                  double* history_host, int64_t history_cap, cb_result* result_host, void* stream);

/* ======================================================================
 * Preconditioned solve (Fig. 1 with M != I): right preconditioning, so the
 * Arnoldi steps build the Krylov space of A M^-1 (step 3: w = A (M^-1 v))
 * and the update is x = x0 + M^-1 (V y) (step 17); the stop test stays on
 * ||b - A x||.  The preconditioner offered is Jacobi, M = diag(A).
 * ====================================================================== */
typedef enum cb_precond_kind {
    CB_PRECOND_NONE = 0,
    CB_PRECOND_JACOBI = 1
} cb_precond_kind;

typedef struct cb_precond {
    int32_t kind;             /* cb_precond_kind */
    int32_t reserved;         /* 0 */
    const double* diag_inv;   /* JACOBI: device float64[n], M^-1 = diag(diag_inv) */
} cb_precond;

/* diag_inv[i] = 1 / a_ii by IEEE division (device float64[n], caller-owned);
 * 1 where row i has no diagonal entry or it is zero or not finite.
 * Asynchronous. */
int cb_jacobi_setup(const cb_csr* A, double* diag_inv, void* stream);

/* Device workspace bytes cbgmres_solve_precond needs: the solver workspace
 * plus nnz float64 values of A M^-1. */
int64_t cbgmres_precond_workspace_bytes(int32_t n, int32_t nnz, int32_t m, int format);

/* As cbgmres_solve, with the right preconditioner M (NULL or kind NONE: the
 * plain solve, workspace as for cbgmres_solve).  For JACOBI the values of
 * A M^-1 (a_ij * diag_inv[j], one rounding per entry) are formed in the
 * workspace once per call and the Arnoldi SpMV reads them, so a step costs
 * what an unpreconditioned step costs; the update x += M^-1 (V y) sums each
 * row's correction first, then scales it.  Synchronous.  CB_ERR_INVALID_ARG
 * for an unknown kind or a NULL diag_inv. */
int cbgmres_solve_precond(const cb_csr* A, const double* b, double* x, int32_t m, double tol, int format,
                          const cb_precond* M, const cb_options* opt, void* workspace,
                          size_t workspace_bytes, double* history_host, int64_t history_cap,
                          cb_result* result_host, void* stream);

/* Device workspace bytes cbgmres_ir_solve needs for (n, m, format): the
 * inner solver's workspace plus the FP64 residual r and correction d (n
 * values each) and a few scalars.  -1 for invalid arguments. */
int64_t cbgmres_ir_workspace_bytes(int32_t n, int32_t m, int format);

/* Mixed-precision form: FP64 iterative refinement around an inner
 * compressed-basis GMRES (restart read as refinement, Section V-C).  Each
 * outer step computes r = b - A x in FP64, runs one inner cycle of GMRES(m) on
 * A d = r from d = 0 with the given basis format and relative tolerance
 * inner_tol, and adds x += d in FP64; it stops when ||b - A x|| <= tol ||b||
 * or after max_outer steps.  Synchronous.
 * workspace: device memory of at least cbgmres_ir_workspace_bytes (256-byte
 * aligned; caller-owned), or NULL and 0 for a library allocation freed before
 * return; a smaller one gives CB_ERR_WORKSPACE.
 * result_host: iterations = inner steps in total, restarts = outer steps. */
int cbgmres_ir_solve(const cb_csr* A, const double* b, double* x, int32_t m, double inner_tol,
                     double tol, int format, int32_t max_outer, void* workspace,
                     size_t workspace_bytes, cb_result* result_host, void* stream);

/* ======================================================================
 * Basis format chosen before the first restart (the automatic choice that
 * Section VIII leaves open: try each candidate format briefly, score how fast
 * its residual falls per second, and finish the solve with the winner).
 *
 * Each candidate format runs a probe -- one GMRES(probe_steps) cycle from the
 * caller's x0, capped at probe_steps Arnoldi steps -- and is scored by its
 * rate: ln(rel_residual0 / rel_residual) / seconds, where rel_residual is the
 * explicit ||b - A x|| / ||b|| after the probe, rel_residual0 that of x0 and
 * seconds the probe's wall time.  A probe that did not lower the residual, or
 * met Inf/NaN, scores -inf; one that reached ||b - A x|| = 0 scores +inf.
 * The first candidate with the highest rate is chosen (cb_auto_pick), and
 * the solve continues with GMRES(m) in that format from that probe's
 * iterate.  A probe that meets tol ends the probing and is chosen.  One
 * untimed Arnoldi step with the first candidate runs before the probes so
 * that one-time costs (code loading, host buffers) fall outside them.
 * ====================================================================== */
#define CB_AUTO_MAX_CANDIDATES 8

typedef struct cb_auto_result {
    int32_t chosen;          /* index into candidates of the format continued with */
    int32_t chosen_format;   /* cb_basis_format of that candidate */
    int32_t probed;          /* probes run (fewer than candidates when one met tol) */
    int32_t status;          /* cb_status of the call */
    double rel_residual0;    /* ||b - A x0|| / ||b|| */
    int32_t probe_steps[CB_AUTO_MAX_CANDIDATES];        /* Arnoldi steps per probe */
    double probe_rel_residual[CB_AUTO_MAX_CANDIDATES];  /* explicit, after each probe */
    double probe_seconds[CB_AUTO_MAX_CANDIDATES];       /* wall time per probe */
    double probe_rate[CB_AUTO_MAX_CANDIDATES];          /* the score above */
    double seconds;          /* wall time of the whole call */
    cb_result solve;         /* the continuation in the chosen format */
} cb_auto_result;

/* The pick rule on its own (pure host code, no GPU): the index of the first
 * of count candidates with the highest rate ln(rel0 / rel[i]) / seconds[i],
 * scored as above; -1 if count < 1 or a pointer is NULL. */
int32_t cb_auto_pick(double rel0, const double* rel_host, const double* seconds_host, int32_t count);

/* Device workspace bytes cbgmres_solve_auto needs: the largest solver
 * workspace over the candidates at restart lengths m and probe_steps, plus
 * three float64[n] vectors (x0, the probe iterate, the best iterate).  -1 for
 * bad arguments. */
int64_t cbgmres_auto_workspace_bytes(int32_t n, int32_t m, int32_t probe_steps,
                                     const int32_t* candidates_host, int32_t count);

/* Solve A x = b with the basis format picked by probing.  x, b, m, tol, opt,
 * history_host/history_cap are as for cbgmres_solve; opt applies to the
 * probes (except max_iters and max_cycles) and to the continuation.
 * candidates_host holds 1..CB_AUTO_MAX_CANDIDATES basis formats;
 * 1 <= probe_steps <= 512.  workspace: NULL (allocated and freed here) or at
 * least cbgmres_auto_workspace_bytes.  Total Arnoldi steps = the sum of
 * probe_steps[] plus solve.iterations.  Synchronous.  Returns the
 * continuation's status; CB_ERR_INVALID_ARG / CB_ERR_WORKSPACE with nothing
 * launched for bad arguments. */
int cbgmres_solve_auto(const cb_csr* A, const double* b, double* x, int32_t m, double tol,
                       const int32_t* candidates_host, int32_t count, int32_t probe_steps,
                       const cb_options* opt, void* workspace, size_t workspace_bytes,
                       double* history_host, int64_t history_cap, cb_auto_result* result_host,
                       void* stream);

/* ======================================================================
 * Arithmetic-intensity sweep: the synthetic benchmark of Section IV-C
 * (Fig. 3).  Column col of V is read through its format's decoder (the same
 * tile loads and in-register decode as the Gram-Schmidt kernels) and every
 * value y goes through `ops` dependent FP64 steps y <- y * a + b; workgroup g
 * writes the sum of its results to partials[g] (device float64, at least
 * cb_intensity_groups(V->n) entries).  Per value: the format's stored bytes
 * read, 2 * ops FP64 operations.  Asynchronous.  CB_ERR_INVALID_ARG for a bad
 * basis, column or ops < 0.
 * ====================================================================== */
int32_t cb_intensity_groups(int64_t n);
int cb_intensity_run(const cb_basis* V, int32_t col, int32_t ops, double a, double b, double* partials,
                     void* stream);

/* ======================================================================
 * Batched solves of small systems (the serving path's packing of small
 * requests into one persistent launch).  Each system is solved by the method
 * of cbgmres_solve (Fig. 1 with restarts, Eq. 4 stop test, same options and
 * statistics) inside ONE workgroup that keeps all of its state -- basis,
 * vectors, H, Givens rotations -- on the GPU for the whole solve; the
 * workgroups of a launch take systems from the list until it is empty.  A
 * system's result does not depend on the rest of the batch (fixed reduction
 * order inside the workgroup); it may differ in the last bits from
 * cbgmres_solve on the same system, whose reductions are ordered across
 * workgroups.
 * ====================================================================== */
typedef struct cb_batch_item {
    cb_csr A;                /* device CSR, 1 <= n <= cbgmres_batch_max_n() */
    const double* b;         /* device float64[n] */
    double* x;               /* device float64[n]: x0 on entry, the iterate on return */
    void* workspace;         /* device, 256-byte aligned, owned by the caller, at least
                                cbgmres_batch_workspace_bytes(n, m, format) bytes; on
                                return it holds the last cycle's basis, column c at
                                byte c * cb_basis_column_bytes(format, n), followed (frsz2)
                                by the exponent words, column c at word
                                c * cb_basis_exponent_words(format, n) of a 256-byte
                                aligned array */
    size_t workspace_bytes;
    int32_t m;               /* restart length, 1 <= m <= cbgmres_batch_max_restart() */
    int32_t format;          /* cb_basis_format */
    double tol;              /* relative residual, > 0 */
} cb_batch_item;

/* Largest n and m a batch item may have. */
int32_t cbgmres_batch_max_n(void);
int32_t cbgmres_batch_max_restart(void);

/* Device workspace bytes of one batch item; -1 if the shape is out of range. */
int64_t cbgmres_batch_workspace_bytes(int32_t n, int32_t m, int format);

/* Solve `count` systems in one launch on `stream`.  items (host array) and the
 * options (nullable, as for cbgmres_solve) are read before return;
 * results_host[i] receives system i's statistics (seconds = the batch's wall
 * time).  Synchronous.  Returns CB_ERR_INVALID_ARG / CB_ERR_WORKSPACE (nothing
 * launched) for a bad item, else CB_OK if every system converged, else the
 * status of the first that did not.  Of the options, eta, max_iters and
 * literal_breakdown apply (max_cycles and fuse_updates do not). */
int cbgmres_solve_batch(const cb_batch_item* items, int32_t count, const cb_options* opt,
                        cb_result* results_host, void* stream);

/* ======================================================================
 * Serving: continuous batching of solve requests on one GPU (the serving
 * form of the method; not in the paper).
 * Requests are admitted while their device footprint fits in the HBM budget
 * (basis n*(m+1) stored bytes + CSR + work vectors); later arrivals wait in
 * FIFO order and are admitted as earlier solves finish and release memory.
 * Large requests run, in arrival order, on solve lanes (host threads, each
 * with its own HIP stream and cbgmres_solve on one request at a time).  Small
 * requests (n <= 16384, m <= cbgmres_batch_max_restart(), the paper's six
 * formats) go to a device-resident request loop: one persistent launch of
 * the one-workgroup solver whose workgroups take systems from a ring of
 * descriptors while it runs, so a small request that arrives while others are
 * being solved joins that launch as soon as a workgroup is free.  Its CSR, b,
 * x and Krylov basis stay in device memory for the whole solve, restarts
 * included.  Arrival order is kept within each kind; small requests do not
 * wait behind large ones.  The path depends on a request's shape only and
 * neither path's arithmetic depends on the other requests, so a result is the
 * same, bit for bit, alone and in any mix.
 * ====================================================================== */
typedef struct cb_server cb_server;

/* Create a server on `device` with an HBM budget in bytes and `lanes` solve
 * lanes for large requests (1..64), plus the device-resident loop for small
 * ones (its device arena is min(budget, 4 GiB), its host staging 256 MiB of
 * pinned memory).  NULL on failure (cb_last_error). */
cb_server* cb_server_create(size_t hbm_budget_bytes, int device, int lanes);

/* Bytes a request of this shape is charged against the budget. */
int64_t cb_server_request_bytes(int32_t n, int32_t nnz, int32_t m, int format);

/* Submit a solve.  Inputs are HOST arrays, copied before return.  Returns
 * CB_ERR_OVER_BUDGET if the request alone exceeds the budget.  Non-blocking;
 * *ticket identifies the request. */
int cb_server_submit(cb_server* s, int32_t n, int32_t nnz, const int32_t* row_ptr_host,
                     const int32_t* col_host, const double* val_host, const double* b_host,
                     const double* x0_host /* nullable: zeros */, int32_t m, double tol,
                     int format, uint64_t* ticket);

/* CB_PENDING until the ticket's solve has finished; then copies the solution
 * into x_host (nullable), the statistics into result_host (nullable), the
 * submit/start/finish times in seconds since server creation into
 * times_host[3] (nullable) and releases the ticket. */
int cb_server_poll(cb_server* s, uint64_t ticket, double* x_host, cb_result* result_host,
                   double* times_host);

/* Bytes currently charged against the budget, and requests waiting. */
int cb_server_stats(cb_server* s, int64_t* charged_bytes, int32_t* queued, int32_t* running);

/* The device-resident loop so far: small requests published to it, those
 * of them served by the launch that was already running when they were
 * published (continuous admission), and launches started.  Returns CB_OK, or
 * the error that disabled the loop (its requests then fail with it). */
int cb_server_ring_stats(cb_server* s, int64_t* published, int64_t* joined_running, int64_t* launches);

/* Wait for every submitted solve, then free the server. */
void cb_server_destroy(cb_server* s);

#ifdef __cplusplus
}
#endif

#endif /* CBGMRES_H */
