// Restarted GMRES with a compressed basis (the paper's Fig. 1) driven from
// the host with device-resident control.
//
// Every scalar decision of the method -- the re-orthogonalisation test (step
// 7), breakdown (step 12), the Givens rotations and the implicit residual
// (steps 16-17), the end of a cycle -- is taken on the GPU, by the last
// workgroup of the kernel whose reduction it needs (epilogue.hpp), and written
// to a control block in device memory.  A step is: the normalise-and-store of
// the step's basis vector fused with the SpMV on it (+ its norm), projection
// (+ h), update (+ norm and step 7 test), and the second projection and update
// when step 7 asks for them (+ breakdown test and Givens rotation); the SpMV's
// norm is summed by the first update's last workgroup.  In a cycle that
// follows one where most steps needed the second pass, the first update runs
// fused with the second projection (its rows are projected again while they
// are still in registers), saving a launch per step; the projection is then
// formed speculatively and dropped when step 7 does not ask for it.  w
// alternates between two buffers, since the fused store+SpMV kernel reads the
// previous w at other rows while it writes the new one.  The host
// enqueues a whole cycle of m steps without waiting; kernels of steps after
// the cycle has ended read the control block and return at once.  The host
// waits once per cycle, after the explicit residual of the restart (step 1 /
// 18, Eq. 4) has been evaluated, to learn whether to stop.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "cb_internal.hpp"
#include "epilogue.hpp"
#include "reduce.hpp"

namespace cb {

using namespace dev;

struct Layout {
    int64_t state, flag, counter, H, cs, sn, g, u, y, hist, w, w2, vals, exps, part, part_s, plan, total;
};

static int64_t al(int64_t x) { return (x + 255) & ~int64_t(255); }

static Layout layout_of(int32_t n, int32_t m, int fmt) {
    Layout L;
    int64_t off = 0;
    auto take = [&](int64_t bytes) { int64_t o = off; off += al(bytes); return o; };
    L.state = take(sizeof(State));
    L.flag = take(sizeof(int32_t));
    L.counter = take(kCounterBytes);
    L.H = take((int64_t)(m + 1) * m * 8);
    L.cs = take((int64_t)m * 8);
    L.sn = take((int64_t)m * 8);
    L.g = take((int64_t)(m + 1) * 8);
    L.u = take((int64_t)(m + 1) * 8);
    L.y = take((int64_t)m * 8);
    L.hist = take((int64_t)m * 8);
    L.w = take(padded_rows(n) * 8);
    L.w2 = take(padded_rows(n) * 8);
    L.vals = take(column_bytes(fmt, n) * (m + 1));
    L.exps = take(exponent_words(fmt, n) * 4 * (m + 1));
    // partial sums: the basis kernels' groups times columns, one per row group
    // of k_sumsq, or one per SpMV workgroup (the IR residual)
    int64_t np_ = (int64_t)project_groups(n) * (m + 2);
    if (np_ < row_groups(n)) np_ = row_groups(n);
    if (np_ < kSpmvGroups) np_ = kSpmvGroups;
    L.part = take(8 * np_);
    L.part_s = take(8 * (int64_t)kSpmvGroups);  // SpMV partials: one per SpMV workgroup
    L.plan = take(spmv_plan_bytes(n));           // SpMV column windows (rows of > 8 entries)
    L.total = off;
    return L;
}

// ----------------------------------------------------------------- scalar kernels
__global__ void k_sumsq(const double* __restrict__ x, int n, double* __restrict__ partials) {
    int row0 = blockIdx.x * kRowsPerWG + threadIdx.x * kSeg;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kSeg; ++q)
        if (row0 + q < n) s = fma(x[row0 + q], x[row0 + q], s);
    s = block_sum<kThreads>(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void k_init(State* st, int32_t* flag, unsigned* counter, double tol, double eta, int max_iters,
                       int literal) {
    for (int i = threadIdx.x; i < kCounterBytes / 4; i += blockDim.x) counter[i] = 0u;
    if (threadIdx.x != 0) return;
    State z = {};
    z.nb = sqrt(ld_ctl(&st->r2));
    z.tol_abs = tol * z.nb;
    z.eta = eta;
    z.max_iters = max_iters;
    z.literal = literal;
    z.rel = -1.0;
    z.gabs = -1.0;
    if (z.nb == 0.0) {
        z.stop = 1;
        z.converged = 1;
        z.rel = 0.0;
        z.gabs = 0.0;
    } else if (!isfinite(z.nb)) {
        z.stop = 1;
        z.status = CB_ERR_NONFINITE;
    }
    *st = z;
    *flag = 0;
}

// Step 1 / 18: beta = ||b - A x|| from the residual SpMV's partials and the
// stop test of Eq. 4.
__global__ __launch_bounds__(256) void k_cycle_begin(State* st, const int32_t* flag, double* g, int m,
                                                     const double* __restrict__ partials, int G) {
    const int t = threadIdx.x;
    __shared__ int go;
    double r2 = 0.0;
    for (int k = t; k < G; k += blockDim.x) r2 += partials[k];
    r2 = block_sum<256>(r2);
    if (t == 0) {
        volatile State& s = *st;
        s.prev_steps = s.steps;
        s.steps = 0;
        s.active = 0;
        s.reorth = 0;
        s.r2 = r2;
        s.beta = sqrt(s.r2);
        s.rel = s.beta / s.nb;
        go = 0;
        if (!isfinite(s.beta) || ld_ctl(flag)) {
            s.stop = 1;
            s.status = CB_ERR_NONFINITE;
        } else if (s.beta <= s.tol_abs) {
            s.stop = 1;
            s.converged = 1;
        } else if (s.iters >= s.max_iters) {
            s.stop = 1;
            s.status = CB_ERR_NOT_CONVERGED;
        } else {
            s.active = 1;
            s.cycles += 1;
            go = 1;
        }

    }
    __syncthreads();
    if (go)
        for (int i = t; i <= m; i += blockDim.x) g[i] = i == 0 ? ld_ctl(&st->beta) : 0.0;
}

// Step 17: back-substitution R y = g over the cycle's steps, by columns: y_i
// is fixed, then column i of R is removed from the right-hand side in parallel.
__global__ __launch_bounds__(256) void k_backsolve(State* st, const double* __restrict__ H,
                                                   const double* __restrict__ g, double* __restrict__ y,
                                                   int m, double col_bytes) {
    __shared__ double rhs[kMaxRestart];
    __shared__ double yi;
    const int k1 = ld_ctl(&st->steps);
    for (int i = threadIdx.x; i < k1; i += blockDim.x) rhs[i] = g[i];
    __syncthreads();
    for (int i = k1 - 1; i >= 0; --i) {
        const double* col = H + (int64_t)i * (m + 1);
        if (threadIdx.x == 0) {
            yi = rhs[i] / ld_ctl(&col[i]);
            y[i] = yi;
        }
        __syncthreads();
        for (int r = threadIdx.x; r < i; r += blockDim.x) rhs[r] -= col[r] * yi;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        volatile State& s = *st;
        s.basis_bytes = s.basis_bytes + (double)k1 * col_bytes;
    }
}

__global__ void k_axpy(double* __restrict__ x, const double* __restrict__ d, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = x[i] + d[i];
}

// x += M^-1 t for the Jacobi preconditioner, one product and one sum per entry
// (no contraction, as the step is written).
__global__ void k_precond_update(double* __restrict__ x, const double* __restrict__ dinv,
                                 const double* __restrict__ t, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = __dadd_rn(x[i], __dmul_rn(dinv[i], t[i]));
}

// dinv[i] = 1 / a_ii (IEEE division); 1 where the row has no diagonal entry or
// it is zero or not finite.  One thread per row.
__global__ void k_jacobi(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                         const double* __restrict__ val, int n, double* __restrict__ dinv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 1.0;
    for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        const double a = val[k];
        if (col[k] == i && a != 0.0 && isfinite(a)) d = 1.0 / a;
    }
    dinv[i] = d;
}

// The values of A M^-1: column j of A scaled by dinv[j], one product per entry.
__global__ void k_scale_cols(const int32_t* __restrict__ col, const double* __restrict__ val,
                             const double* __restrict__ dinv, int64_t nnz, double* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) out[k] = __dmul_rn(val[k], dinv[col[k]]);
}

// ----------------------------------------------------------------- host side
struct Pinned {
    void* p = nullptr;
    size_t cap = 0;
    void* get(size_t bytes) {
        if (bytes > cap) {
            if (p) (void)hipHostFree(p);
            p = nullptr;
            cap = 0;
            if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
            cap = bytes;
        }
        return p;
    }
};
static thread_local Pinned g_pinned;

static double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Two words of pinned, mapped, coherent host memory per host thread through
// which the solver's last workgroup reports a cycle's progress (steps finished,
// cycle ended) while the cycle runs.  NULL device pointer if unavailable.
struct Progress {
    int32_t* h = nullptr;
    int32_t* d = nullptr;
    bool tried = false;
    bool get() {
        if (!tried) {
            tried = true;
            void* p = nullptr;
            void* dp = nullptr;
            if (hipHostMalloc(&p, 64, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) return false;
            if (hipHostGetDevicePointer(&dp, p, 0) != hipSuccess) {
                (void)hipHostFree(p);
                return false;
            }
            h = static_cast<int32_t*>(p);
            d = static_cast<int32_t*>(dp);
        }
        return h != nullptr;
    }
};
static thread_local Progress g_progress;

// Launches are enqueued at most this many Arnoldi steps ahead of what the GPU
// has reported finished (reports come every kProgressEvery steps, so the host
// runs 4-8 steps ahead).  Steps after the cycle's last are launches that only
// read their guard and return (~2.4 us of GPU time each, four per step);
// enqueuing a cycle's m steps at once spent that on every step past
// convergence.
constexpr int kStepsAhead = 8;

// Wait until the GPU has finished `target` steps of the current cycle or ended
// it (spinning on the host-mapped words); returns true if the cycle has ended.
// The wait also ends when the stream has drained (no launch left that could
// report) or after 10 s, after which the caller simply enqueues the remaining
// steps: every step's launches check the cycle's guard on the GPU, so pacing
// affects only how many of them run, never the result.
static bool wait_progress(const volatile int32_t* p, int target, hipStream_t s) {
    const double t0 = now_s();
    for (unsigned it = 0;; ++it) {
        if (p[1]) return true;
        if (p[0] >= target) return false;
        if ((it & 1023u) == 1023u) {
            if (hipStreamQuery(s) != hipErrorNotReady) return p[1] != 0;
            if (now_s() - t0 > 10.0) return false;
        }
        std::this_thread::yield();  // steps take tens of microseconds; leave the core to other solves
    }
}

struct Ws {
    unsigned char* base;
    Layout L;
    template <class T>
    T* at(int64_t off) const { return reinterpret_cast<T*>(base + off); }
};


// ||x||^2 of a device vector into *dst (device), using the partial buffer.
static void enqueue_sumsq(const double* x, int n, double* part, double* dst, hipStream_t s) {
    const int G = row_groups(n);
    k_sumsq<<<G, kThreads, 0, s>>>(x, n, part);
    launch_reduce(part, G, 1, dst, 0, nullptr, s);
}

// The solve proper, on a prepared workspace.  Returns a cb_status.
// With a Jacobi right preconditioner (dinv non-NULL) the Arnoldi SpMV runs on
// A M^-1, whose values pval (A's values with column j scaled by dinv[j]) the
// caller has formed, and the x update adds M^-1 (V y); the explicit residual
// stays b - A x.
static int solve_impl(const cb_csr& A, const double* b, double* x, int m, double tol, int fmt,
                      const cb_options* opt, const Ws& W, double* history_host,
                      int64_t history_cap, cb_result* res, hipStream_t s,
                      const double* dinv = nullptr, const double* pval = nullptr, bool plan_ready = false) {
    const double t0 = now_s();
    const int n = A.n;
    const double eta = (opt && opt->eta > 0) ? opt->eta : 0.7071067811865476;
    const int max_iters = (opt && opt->max_iters > 0) ? opt->max_iters : 20000;
    const int max_cycles = opt ? opt->max_cycles : 0;
    const int literal = opt ? opt->literal_breakdown : 0;
    const int fuse_opt = opt ? opt->fuse_updates : 0;

    State* st = W.at<State>(W.L.state);
    int32_t* flag = W.at<int32_t>(W.L.flag);
    unsigned* counter = W.at<unsigned>(W.L.counter);
    double* H = W.at<double>(W.L.H);
    double* cs = W.at<double>(W.L.cs);
    double* sn = W.at<double>(W.L.sn);
    double* g = W.at<double>(W.L.g);
    double* u = W.at<double>(W.L.u);
    double* y = W.at<double>(W.L.y);
    double* hist = W.at<double>(W.L.hist);
    double* w = W.at<double>(W.L.w);
    double* w2 = W.at<double>(W.L.w2);
    double* part = W.at<double>(W.L.part);
    double* part_s = W.at<double>(W.L.part_s);
    const int Gs = spmv_groups(n, A.nnz);
    cb_csr AM = A;  // the operator of the Arnoldi steps: A, or A M^-1
    if (dinv) AM.val = pval;
    // column windows of the matrix's row blocks for the long-row SpMV (A and
    // A M^-1 share the pattern)
    void* plan = nullptr;
    if (spmv_uses_plan(n, A.nnz)) {
        plan = W.base + W.L.plan;
        if (!plan_ready) launch_spmv_plan(A, plan, s);  // else the caller formed it in this workspace
    }
    cb_basis V{fmt, n, m + 1, 0, W.base + W.L.vals,
               frsz2_bits_of(fmt) ? W.at<uint32_t>(W.L.exps) : nullptr};
    const double cbytes = (double)column_bytes(fmt, n);
    int* active = &st->active;
    int* reorth = &st->reorth;
    int* steps = &st->steps;

    // epilogue templates: a plain sum into the control block, and the solver
    // step logic (column j filled in per launch)
    Epi sum_e{};
    sum_e.mode = EPI_STORE;
    sum_e.counter = counter;
    Epi step_e{};
    step_e.counter = counter;
    step_e.st = st;
    step_e.H = H;
    step_e.cs = cs;
    step_e.sn = sn;
    step_e.g = g;
    step_e.hist = hist;
    step_e.m = m;
    step_e.col_bytes = cbytes;
    int32_t* prog_h = nullptr;
    if (g_progress.get()) {
        prog_h = g_progress.h;
        step_e.prog = g_progress.d;
    }

    State* hs = static_cast<State*>(g_pinned.get(sizeof(State) + (size_t)m * 8));
    if (!hs) return fail(CB_ERR_HIP, "hipHostMalloc failed");
    double* hh = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(hs) + sizeof(State));
    int64_t recorded = 0;

    // ||b||, tolerances, counters
    enqueue_sumsq(b, n, part, &st->r2, s);
    k_init<<<1, 256, 0, s>>>(st, flag, counter, tol, eta, max_iters, literal);
    CB_HIP(hipMemcpyAsync(hs, st, sizeof(State), hipMemcpyDeviceToHost, s));
    CB_HIP(hipStreamSynchronize(s));
    if (hs->stop) {
        if (hs->nb == 0.0) launch_fill(x, 0.0, n, s);
    } else {
        int cycles = 0;
        bool capped = false;
        bool fused = true;
        int prev_iters = 0, prev_reorths = 0;
        for (;;) {
            // restart: explicit residual into w, beta, stop test
            launch_spmv(A, x, b, w, part_s, 1, nullptr, s, plan);
            k_cycle_begin<<<1, 256, 0, s>>>(st, flag, g, m, part_s, Gs);
            CB_HIP(hipMemcpyAsync(hs, st, sizeof(State), hipMemcpyDeviceToHost, s));
            if (cycles > 0) CB_HIP(hipMemcpyAsync(hh, hist, (size_t)m * 8, hipMemcpyDeviceToHost, s));
            CB_HIP(hipStreamSynchronize(s));
            if (history_host && cycles > 0) {
                for (int k = 0; k < hs->prev_steps && recorded < history_cap; ++k)
                    history_host[recorded++] = hh[k] / hs->nb;
            }
            if (hs->stop) break;
            // Fuse the first update with the second projection in this cycle
            // when the last cycle re-orthogonalised at least half its steps
            // (the first cycle assumes so); the decision depends on the
            // solve's own history only.  A float64 basis keeps the separate
            // launches: with 16-byte-per-lane float64 tiles the fused kernel
            // holds half as many loads in flight and measured no faster.
            if (cycles > 0) {
                const int steps_done = hs->iters - prev_iters;
                fused = steps_done > 0 && 2 * (hs->reorths - prev_reorths) >= steps_done;
            }
            if (fmt == CB_F64) fused = false;
            if (fuse_opt == 1) fused = false;
            if (fuse_opt == 2) fused = true;
            prev_iters = hs->iters;
            prev_reorths = hs->reorths;
            step_e.fused = fused;
            double* wc = w;   // the current w (the residual r first)
            double* wn = w2;  // the buffer the next SpMV writes
            if (prog_h) {     // the stream is idle here (synchronised above)
                prog_h[0] = 0;
                prog_h[1] = 0;
                std::atomic_thread_fence(std::memory_order_seq_cst);
            }
            for (int j = 0; j < m; ++j) {
                double* hcol = H + (int64_t)j * (m + 1);
                // v_j = w / (beta or h_{j,j-1}), V_j = Q(v_j), w = A v_j; its
                // ||w||^2 partials go to the first update's epilogue
                launch_spmv_store(fmt, AM, V, j, wc, j == 0 ? &st->beta : &st->hn, wn, part_s, flag, active, s,
                                  plan);
                double* t = wc;
                wc = wn;
                wn = t;
                Epi eh = sum_e;          // h_{1:j+1,j}
                eh.out = hcol;
                launch_project(fmt, V, j + 1, wc, part, active, eh, s);
                // the first update; omega, ||w||, step 7 test, maybe Givens
                Epi ex = step_e;
                ex.out = u;
                ex.j = j;
                ex.extra = part_s;
                ex.extra_G = Gs;
                if (fused) {
                    // fused with the second projection: u is formed whether or
                    // not step 7 asks for it, and kept only if it does
                    ex.mode = EPI_FUSED_CHECK;
                    launch_subtract_project(fmt, V, j + 1, hcol, wc, part, active, ex, s);
                } else {
                    ex.mode = EPI_STEP_CHECK;
                    launch_subtract(fmt, V, j + 1, nullptr, hcol, wc, part, active, -1, ex, s);
                    Epi eu = step_e;     // u = V^T w, h += u
                    eu.mode = EPI_REORTH_PROJECT;
                    eu.out = u;
                    eu.j = j;
                    launch_project(fmt, V, j + 1, wc, part, reorth, eu, s);
                }
                Epi ef = step_e;         // ||w||, breakdown test, Givens
                ef.mode = EPI_REORTH_FINISH;
                ef.j = j;
                launch_subtract(fmt, V, j + 1, nullptr, u, wc, part, reorth, -1, ef, s);
                // stay kStepsAhead steps ahead of the GPU; stop once the cycle
                // has ended (later steps would only check their guards)
                if (prog_h && j + 1 < m && j >= kStepsAhead &&
                    wait_progress(prog_h, j + 1 - kStepsAhead, s))
                    break;
            }
            k_backsolve<<<1, 256, 0, s>>>(st, H, g, y, m, cbytes);
            if (dinv) {
                // t = V y into the free w2 (from zero, so t is the row sums
                // exactly), then x += M^-1 t
                launch_fill(w2, 0.0, n, s);
                launch_subtract(fmt, V, m, steps, y, w2, nullptr, steps, +1, Epi{}, s);
                k_precond_update<<<(n + 255) / 256, 256, 0, s>>>(x, dinv, w2, n);
            } else {
                launch_subtract(fmt, V, m, steps, y, x, nullptr, steps, +1, Epi{}, s);
            }
            CB_HIP(hipGetLastError());
            ++cycles;
            if (max_cycles > 0 && cycles >= max_cycles) {
                CB_HIP(hipMemcpyAsync(hs, st, sizeof(State), hipMemcpyDeviceToHost, s));
                CB_HIP(hipMemcpyAsync(hh, hist, (size_t)m * 8, hipMemcpyDeviceToHost, s));
                CB_HIP(hipStreamSynchronize(s));
                if (history_host) {
                    for (int k = 0; k < hs->steps && recorded < history_cap; ++k)
                        history_host[recorded++] = hh[k] / hs->nb;
                }
                capped = true;
                break;
            }
        }
        if (capped && hs->status == CB_OK) {
            // cycle cap: report without the explicit residual of the new x
            hs->status = CB_ERR_NOT_CONVERGED;
            hs->rel = -1.0;
        }
    }
    CB_HIP(hipStreamSynchronize(s));
    if (res) {
        res->iterations = hs->iters;
        res->restarts = hs->cycles;
        res->reorths = hs->reorths;
        res->breakdowns = hs->breakdowns;
        res->converged = hs->converged;
        res->status = hs->status;
        res->rel_residual = hs->rel;
        res->implicit_rel_residual = hs->gabs >= 0 ? hs->gabs / (hs->nb > 0 ? hs->nb : 1.0) : -1.0;
        res->seconds = now_s() - t0;
        res->basis_bytes = hs->basis_bytes;
    }
    return hs->status;
}

static int check_solve_args(const cb_csr* A, const double* b, const double* x, int32_t m,
                            double tol, int format) {
    if (!A || !b || !x) return fail(CB_ERR_INVALID_ARG, "NULL argument");
    if (A->n < 1 || A->n > kMaxRows || A->nnz < 0 || !A->row_ptr || (A->nnz && (!A->col || !A->val)))
        return fail(CB_ERR_INVALID_ARG, "bad matrix");
    if (m < 1 || m > kMaxRestart)
        return fail(CB_ERR_INVALID_ARG, "restart m=%d out of range [1, %d]", m, kMaxRestart);
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(CB_ERR_INVALID_ARG, "tol must be positive");
    if (!valid_format(format)) return fail(CB_ERR_INVALID_ARG, "unknown basis format %d", format);
    if (!aligned(x, 16) || !aligned(b, 8)) return fail(CB_ERR_INVALID_ARG, "x must be 16-byte and b 8-byte aligned");
    return CB_OK;
}

}  // namespace cb

using namespace cb;

extern "C" {

int64_t cbgmres_workspace_bytes(int32_t n, int32_t m, int format) {
    if (n < 1 || n > kMaxRows || m < 1 || !valid_format(format)) return -1;
    return layout_of(n, m, format).total;
}

int cbgmres_solve(const cb_csr* A, const double* b, double* x, int32_t m, double tol, int format,
                  const cb_options* opt, void* workspace, size_t workspace_bytes,
                  double* history_host, int64_t history_cap, cb_result* result_host, void* stream) {
    if (int e = check_solve_args(A, b, x, m, tol, format)) return e;
    hipStream_t s = (hipStream_t)stream;
    Ws W;
    W.L = layout_of(A->n, m, format);
    bool owned = false;
    if (workspace) {
        if ((int64_t)workspace_bytes < W.L.total)
            return fail(CB_ERR_WORKSPACE, "workspace %zu < %lld bytes", workspace_bytes,
                        (long long)W.L.total);
        W.base = static_cast<unsigned char*>(workspace);
    } else {
        void* p = nullptr;
        CB_HIP(hipMalloc(&p, (size_t)W.L.total));
        W.base = static_cast<unsigned char*>(p);
        owned = true;
    }
    int st = solve_impl(*A, b, x, m, tol, format, opt, W, history_host, history_cap, result_host, s);
    if (owned) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(W.base);
    }
    return st;
}

int cb_jacobi_setup(const cb_csr* A, double* diag_inv, void* stream) {
    if (!A || !diag_inv || A->n < 1 || A->n > kMaxRows || !A->row_ptr || A->nnz < 0 || (A->nnz && (!A->col || !A->val)))
        return fail(CB_ERR_INVALID_ARG, "bad matrix or output");
    k_jacobi<<<(A->n + 255) / 256, 256, 0, (hipStream_t)stream>>>(A->row_ptr, A->col, A->val, A->n, diag_inv);
    CB_HIP(hipGetLastError());
    return CB_OK;
}

int64_t cbgmres_precond_workspace_bytes(int32_t n, int32_t nnz, int32_t m, int format) {
    if (n < 1 || n > kMaxRows || nnz < 0 || m < 1 || !valid_format(format)) return -1;
    return layout_of(n, m, format).total + al((int64_t)nnz * 8);
}

int cbgmres_solve_precond(const cb_csr* A, const double* b, double* x, int32_t m, double tol, int format,
                          const cb_precond* M, const cb_options* opt, void* workspace,
                          size_t workspace_bytes, double* history_host, int64_t history_cap,
                          cb_result* result_host, void* stream) {
    if (!M || M->kind == CB_PRECOND_NONE)
        return cbgmres_solve(A, b, x, m, tol, format, opt, workspace, workspace_bytes, history_host,
                             history_cap, result_host, stream);
    if (M->kind != CB_PRECOND_JACOBI || !M->diag_inv)
        return fail(CB_ERR_INVALID_ARG, "unknown preconditioner kind %d or NULL diag_inv", M->kind);
    if (int e = check_solve_args(A, b, x, m, tol, format)) return e;
    const int64_t total = cbgmres_precond_workspace_bytes(A->n, A->nnz, m, format);
    if (workspace && (int64_t)workspace_bytes < total)
        return fail(CB_ERR_WORKSPACE, "workspace %zu < %lld bytes", workspace_bytes, (long long)total);
    hipStream_t s = (hipStream_t)stream;
    Ws W;
    W.L = layout_of(A->n, m, format);
    void* owned = nullptr;
    if (workspace) {
        W.base = static_cast<unsigned char*>(workspace);
    } else {
        CB_HIP(hipMalloc(&owned, (size_t)total));
        W.base = static_cast<unsigned char*>(owned);
    }
    double* pval = reinterpret_cast<double*>(W.base + W.L.total);
    if (A->nnz)
        k_scale_cols<<<(unsigned)((A->nnz + 255) / 256), 256, 0, s>>>(A->col, A->val, M->diag_inv, A->nnz, pval);
    int st = CB_OK;
    if (hipGetLastError() != hipSuccess)
        st = fail(CB_ERR_HIP, "launch failed");
    else
        st = solve_impl(*A, b, x, m, tol, format, opt, W, history_host, history_cap, result_host, s,
                        M->diag_inv, pval);
    if (owned) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(owned);
    }
    return st;
}

int64_t cbgmres_ir_workspace_bytes(int32_t n, int32_t m, int format) {
    if (n < 1 || n > kMaxRows || m < 1 || m > kMaxRestart || !valid_format(format)) return -1;
    return layout_of(n, m, format).total + 2 * al(padded_rows(n) * 8) + 256;
}

int cbgmres_ir_solve(const cb_csr* A, const double* b, double* x, int32_t m, double inner_tol,
                     double tol, int format, int32_t max_outer, void* workspace, size_t workspace_bytes,
                     cb_result* result_host, void* stream) {
    if (int e = check_solve_args(A, b, x, m, tol, format)) return e;
    if (!(inner_tol > 0.0)) return fail(CB_ERR_INVALID_ARG, "inner_tol must be positive");
    if (max_outer < 1) return fail(CB_ERR_INVALID_ARG, "max_outer must be >= 1");
    const int n = A->n;
    const int64_t total = cbgmres_ir_workspace_bytes(n, m, format);
    if (workspace && (int64_t)workspace_bytes < total)
        return fail(CB_ERR_WORKSPACE, "workspace %zu < %lld bytes", workspace_bytes, (long long)total);
    if (!aligned(workspace, 256)) return fail(CB_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    const double t0 = now_s();
    hipStream_t s = (hipStream_t)stream;
    Ws W;
    W.L = layout_of(n, m, format);
    const int64_t vec = al(padded_rows(n) * 8);
    void* owned = nullptr;
    if (workspace) {
        W.base = static_cast<unsigned char*>(workspace);
    } else {
        CB_HIP(hipMalloc(&owned, (size_t)total));
        W.base = static_cast<unsigned char*>(owned);
    }
    double* r = reinterpret_cast<double*>(W.base + W.L.total);
    double* d = reinterpret_cast<double*>(W.base + W.L.total + vec);
    double* scal = reinterpret_cast<double*>(W.base + W.L.total + 2 * vec);
    double* part = W.at<double>(W.L.part);
    double* hv = static_cast<double*>(g_pinned.get(sizeof(State) + (size_t)m * 8 + 64));
    int status = CB_ERR_NOT_CONVERGED;
    cb_result acc;
    memset(&acc, 0, sizeof acc);
    acc.rel_residual = -1.0;
    cb_options io{0.0, 0, 1, 0, 0};
    double nb = 0.0;
    if (!hv) { status = fail(CB_ERR_HIP, "hipHostMalloc failed"); goto done; }
    enqueue_sumsq(b, n, part, scal, s);
    if (hipMemcpyAsync(hv, scal, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { status = fail(CB_ERR_HIP, "copy failed"); goto done; }
    nb = std::sqrt(hv[0]);
    if (nb == 0.0) {
        launch_fill(x, 0.0, n, s);
        acc.converged = 1;
        acc.rel_residual = 0.0;
        status = CB_OK;
        goto done;
    }
    if (spmv_uses_plan(n, A->nnz)) launch_spmv_plan(*A, W.base + W.L.plan, s);
    for (;;) {
        launch_spmv(*A, x, b, r, part, 1, nullptr, s,
                    spmv_uses_plan(n, A->nnz) ? W.base + W.L.plan : nullptr);
        launch_reduce(part, spmv_groups(n, A->nnz), 1, scal, 0, nullptr, s);
        if (hipMemcpyAsync(hv, scal, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) { status = fail(CB_ERR_HIP, "copy failed"); goto done; }
        const double rn = std::sqrt(hv[0]);
        acc.rel_residual = rn / nb;
        if (!std::isfinite(rn)) { status = CB_ERR_NONFINITE; break; }
        if (rn <= tol * nb) { acc.converged = 1; status = CB_OK; break; }
        if (acc.restarts >= max_outer) { status = CB_ERR_NOT_CONVERGED; break; }
        launch_fill(d, 0.0, n, s);
        cb_result ir;
        int ist = solve_impl(*A, r, d, m, inner_tol, format, &io, W, nullptr, 0, &ir, s, nullptr, nullptr,
                             true);
        acc.iterations += ir.iterations;
        acc.reorths += ir.reorths;
        acc.breakdowns += ir.breakdowns;
        acc.basis_bytes += ir.basis_bytes;
        acc.restarts += 1;
        acc.implicit_rel_residual = ir.implicit_rel_residual;
        if (ist == CB_ERR_NONFINITE || ist == CB_ERR_HIP) { status = ist; break; }
        k_axpy<<<(n + 255) / 256, 256, 0, s>>>(x, d, n);
    }
done:
    (void)hipStreamSynchronize(s);
    if (owned) (void)hipFree(owned);
    acc.status = status;
    acc.seconds = now_s() - t0;
    if (result_host) *result_host = acc;
    return status;
}

// ---------------------------------------------------------------------------
// Basis format picked by probing before the first restart.

static double auto_rate(double rel0, double rel, double seconds) {
    if (!std::isfinite(rel) || rel < 0.0 || !(rel < rel0)) return -INFINITY;
    if (rel == 0.0 || !(seconds > 0.0)) return INFINITY;
    return std::log(rel0 / rel) / seconds;
}

int32_t cb_auto_pick(double rel0, const double* rel_host, const double* seconds_host, int32_t count) {
    if (count < 1 || !rel_host || !seconds_host) return -1;
    int32_t best = 0;
    double best_rate = auto_rate(rel0, rel_host[0], seconds_host[0]);
    for (int32_t i = 1; i < count; ++i) {
        const double r = auto_rate(rel0, rel_host[i], seconds_host[i]);
        if (r > best_rate) {
            best = i;
            best_rate = r;
        }
    }
    return best;
}

static int64_t auto_solver_bytes(int32_t n, int32_t m, int32_t p, const int32_t* cand, int32_t count) {
    int64_t bytes = 0;
    for (int32_t i = 0; i < count; ++i)
        bytes = std::max({bytes, layout_of(n, m, cand[i]).total, layout_of(n, p, cand[i]).total});
    return al(bytes);
}

int64_t cbgmres_auto_workspace_bytes(int32_t n, int32_t m, int32_t probe_steps,
                                     const int32_t* candidates_host, int32_t count) {
    if (n < 1 || n > kMaxRows || m < 1 || m > kMaxRestart || probe_steps < 1 || probe_steps > kMaxRestart ||
        !candidates_host || count < 1 || count > CB_AUTO_MAX_CANDIDATES)
        return -1;
    for (int32_t i = 0; i < count; ++i)
        if (!valid_format(candidates_host[i])) return -1;
    return auto_solver_bytes(n, m, probe_steps, candidates_host, count) + 3 * al(padded_rows(n) * 8) + 256;
}

int cbgmres_solve_auto(const cb_csr* A, const double* b, double* x, int32_t m, double tol,
                       const int32_t* candidates_host, int32_t count, int32_t probe_steps,
                       const cb_options* opt, void* workspace, size_t workspace_bytes,
                       double* history_host, int64_t history_cap, cb_auto_result* result_host,
                       void* stream) {
    if (!candidates_host || count < 1 || count > CB_AUTO_MAX_CANDIDATES)
        return fail(CB_ERR_INVALID_ARG, "candidate count must be in [1, %d]", CB_AUTO_MAX_CANDIDATES);
    if (int e = check_solve_args(A, b, x, m, tol, candidates_host[0])) return e;
    for (int32_t i = 0; i < count; ++i)
        if (!valid_format(candidates_host[i]))
            return fail(CB_ERR_INVALID_ARG, "unknown basis format %d", candidates_host[i]);
    if (probe_steps < 1 || probe_steps > kMaxRestart)
        return fail(CB_ERR_INVALID_ARG, "probe_steps=%d out of range [1, %d]", probe_steps, kMaxRestart);
    const int n = A->n;
    const int64_t total = cbgmres_auto_workspace_bytes(n, m, probe_steps, candidates_host, count);
    if (workspace && (int64_t)workspace_bytes < total)
        return fail(CB_ERR_WORKSPACE, "workspace %zu < %lld bytes", workspace_bytes, (long long)total);
    const double t0 = now_s();
    hipStream_t s = (hipStream_t)stream;
    struct Owned {
        void* p = nullptr;
        hipStream_t s;
        ~Owned() {
            if (p) {
                (void)hipStreamSynchronize(s);
                (void)hipFree(p);
            }
        }
    } owned{nullptr, s};
    Ws W;
    if (workspace) {
        W.base = static_cast<unsigned char*>(workspace);
    } else {
        CB_HIP(hipMalloc(&owned.p, (size_t)total));
        W.base = static_cast<unsigned char*>(owned.p);
    }
    const int64_t solver_bytes = auto_solver_bytes(n, m, probe_steps, candidates_host, count);
    const int64_t vec = al(padded_rows(n) * 8);
    double* x0 = reinterpret_cast<double*>(W.base + solver_bytes);
    double* xp = reinterpret_cast<double*>(W.base + solver_bytes + vec);      // the probe's iterate
    double* xb = reinterpret_cast<double*>(W.base + solver_bytes + 2 * vec);  // the best probe's
    double* scal = reinterpret_cast<double*>(W.base + solver_bytes + 3 * vec);

    cb_auto_result out;
    memset(&out, 0, sizeof out);
    out.chosen_format = candidates_host[0];
    out.rel_residual0 = -1.0;
    out.solve.rel_residual = -1.0;
    out.solve.implicit_rel_residual = -1.0;
    auto finish = [&](int status) {
        out.status = status;
        out.solve.status = status;
        out.seconds = now_s() - t0;
        if (result_host) *result_host = out;
        return status;
    };

    // ||b|| and ||b - A x0||
    W.L = layout_of(n, m, candidates_host[0]);
    double* part = W.at<double>(W.L.part);
    double* hv = static_cast<double*>(g_pinned.get(sizeof(State) + (size_t)std::max(m, probe_steps) * 8 + 64));
    if (!hv) return fail(CB_ERR_HIP, "hipHostMalloc failed");
    enqueue_sumsq(b, n, part, scal, s);
    launch_spmv(*A, x, b, xp, part, 1, nullptr, s);
    launch_reduce(part, spmv_groups(n, A->nnz), 1, scal + 1, 0, nullptr, s);
    CB_HIP(hipMemcpyAsync(hv, scal, 16, hipMemcpyDeviceToHost, s));
    CB_HIP(hipStreamSynchronize(s));
    const double nb = std::sqrt(hv[0]);
    if (nb == 0.0) {  // b = 0: x = 0 solves it exactly
        launch_fill(x, 0.0, n, s);
        CB_HIP(hipStreamSynchronize(s));
        out.rel_residual0 = 0.0;
        out.solve.converged = 1;
        out.solve.rel_residual = 0.0;
        return finish(CB_OK);
    }
    const double rel0 = std::sqrt(hv[1]) / nb;
    out.rel_residual0 = rel0;
    out.solve.rel_residual = rel0;
    if (!std::isfinite(rel0)) return finish(CB_ERR_NONFINITE);
    if (rel0 <= tol) {
        out.solve.converged = 1;
        return finish(CB_OK);
    }
    CB_HIP(hipMemcpyAsync(x0, x, (size_t)n * 8, hipMemcpyDeviceToDevice, s));

    // untimed warm-up step, then one probe per candidate
    cb_options po{0.0, 1, 0, 0, 0};
    if (opt) {
        po.eta = opt->eta;
        po.literal_breakdown = opt->literal_breakdown;
        po.fuse_updates = opt->fuse_updates;
    }
    CB_HIP(hipMemcpyAsync(xp, x0, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
    W.L = layout_of(n, 1, candidates_host[0]);
    if (solve_impl(*A, b, xp, 1, tol, candidates_host[0], &po, W, nullptr, 0, nullptr, s) == CB_ERR_HIP)
        return finish(CB_ERR_HIP);
    po.max_iters = probe_steps;
    double rel[CB_AUTO_MAX_CANDIDATES], secs[CB_AUTO_MAX_CANDIDATES];
    for (int32_t i = 0; i < count; ++i) {
        const int c = candidates_host[i];
        CB_HIP(hipMemcpyAsync(xp, x0, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
        CB_HIP(hipStreamSynchronize(s));
        W.L = layout_of(n, probe_steps, c);
        cb_result pr;
        const int st = solve_impl(*A, b, xp, probe_steps, tol, c, &po, W, nullptr, 0, &pr, s);
        if (st == CB_ERR_HIP) return finish(CB_ERR_HIP);
        rel[i] = st == CB_ERR_NONFINITE ? NAN : pr.rel_residual;
        secs[i] = pr.seconds;
        out.probe_steps[i] = pr.iterations;
        out.probe_rel_residual[i] = rel[i];
        out.probe_seconds[i] = secs[i];
        out.probe_rate[i] = auto_rate(rel0, rel[i], secs[i]);
        out.probed = i + 1;
        // keep the best probe's iterate: swap the buffers when this one leads
        if (pr.converged || cb_auto_pick(rel0, rel, secs, i + 1) == i) {
            std::swap(xp, xb);
            out.chosen = i;
        }
        if (pr.converged) break;
    }
    out.chosen_format = candidates_host[out.chosen];

    // continue from the chosen probe's iterate in its format
    CB_HIP(hipMemcpyAsync(x, xb, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
    W.L = layout_of(n, m, out.chosen_format);
    const int st = solve_impl(*A, b, x, m, tol, out.chosen_format, opt, W, history_host, history_cap,
                              &out.solve, s);
    return finish(st);
}

}  // extern "C"
