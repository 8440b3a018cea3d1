// Second reduction stage and the solver's per-step decisions, run at the end
// of the kernel that produced the per-workgroup partial sums.
//
// Every workgroup writes its partials (one per column it owns), then takes a
// ticket from the counter of its group of 32 workgroups.  The workgroup that
// draws its group's last ticket sums the group's partials per column in
// workgroup-index order, writes each sum over the partial of the group's first
// workgroup, and takes a ticket from the top counter; the workgroup that draws
// the last top ticket sums the group sums in group order (so the result does
// not depend on which workgroup finished last), stores or applies the sums,
// and the counters are left at zero for the next launch on the stream.  The
// reduction is spread over the groups' last workgroups, which run while other
// groups still stream, so the final workgroup adds only a few values per
// column.  Partials are written with device-scope (agent) relaxed atomic
// stores, which are coherent across the XCDs' L2 caches, and each thread waits
// for its stores to complete before a ticket is drawn; the workgroups that go
// on to read other workgroups' partials read them with device-scope atomic
// loads, so no cache-wide invalidation is needed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cb_internal.hpp"
#include "reduce.hpp"

namespace cb {

// Device-resident control block of a solve (one per workspace).
struct State {
    double nb, tol_abs, eta;
    double beta;       // ||r|| at the start of the cycle
    double r2;         // ||r||^2 (or ||b||^2 at init)
    double om2;        // ||A v||^2
    double hn2;        // ||w||^2 after a Gram-Schmidt pass
    double hn;         // h_{j+1,j}: the divisor of the next basis vector
    double omega;      // ||A v||
    double omega_pre;  // ||w|| before the re-orthogonalisation pass
    double gabs;       // |g_{j+1}|
    double rel;        // last explicit relative residual
    double basis_bytes;
    int32_t active;    // 1 while the current cycle continues
    int32_t reorth;    // 1 while the current step needs the second pass
    int32_t steps;     // steps taken in the current cycle
    int32_t prev_steps;
    int32_t iters, reorths, breakdowns, converged;
    int32_t stop, status, cycles, max_iters;
    int32_t literal, pad0, pad1, pad2;
};

enum EpiMode : int {
    EPI_STORE = 0,          // out[c] = sum
    EPI_STEP_CHECK = 1,     // first Gram-Schmidt pass done: norm -> step 7 test
    EPI_REORTH_PROJECT = 2, // u = sum; h += u
    EPI_REORTH_FINISH = 3,  // second pass done: norm -> breakdown test, Givens
    EPI_FUSED_CHECK = 4,    // first update fused with the second projection:
                            // sums u_0..u_{ncols-2} and ||w||^2 (last column) ->
                            // step 7 test; u kept (h += u) only if it asks for it
};

// Arnoldi steps between the progress reports of a cycle (Epi::prog).
constexpr int kProgressEvery = 4;

struct Epi {
    int mode;
    int ncols;             // sums to form
    int G;                 // partials per column (column stride of `partials`)
    double* out;           // EPI_STORE / EPI_REORTH_PROJECT (u)
    unsigned* counter;     // ticket counters (kCounterBytes, zero between launches)
    int cw;                // columns per workgroup chunk (blockIdx.y), multi-column sums
    const double* extra;   // EPI_STEP_CHECK: the SpMV's ||A v||^2 partials
    int extra_G;
    // solver context (modes 1-3)
    State* st;
    double* H;             // column-major (m+1) x m
    double* cs;
    double* sn;
    double* g;
    double* hist;
    int j;                 // Arnoldi step (0-based): column j of H
    int m;
    double col_bytes;
    int fused;             // this cycle runs the first update fused with the second projection
    int* prog;             // NULL, or host-mapped words: [0] steps finished in the cycle, [1] 1 once it ended
};

namespace dev {

__device__ __forceinline__ void store_partial(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// For the nc columns c0 .. c0+nc-1 (nc <= 256): lds[i] = sum over k < M of
// partials[(c0 + i) * G + m0 + k * stride].  tpc threads share a column (the
// fewest, up to 256 / nc, that leave each at most 8 loads per batch): thread s
// of the column issues the loads of k = s, s + tpc, ..., s + 7 tpc together
// and adds them in order, batch after batch; then the tpc sums are added in
// index order.  The order depends on (M, nc) only.
__device__ __forceinline__ void reduce_range(const double* __restrict__ partials, int G, int m0, int M,
                                             int stride, int c0, int nc, double* lds) {
    int tpc = 1;
    while (tpc * 2 <= 256 / nc && tpc * 8 < M) tpc *= 2;
    const int t = threadIdx.x;
    double s = 0.0;
    if (t < tpc * nc) {
        const double* p = partials + (int64_t)(c0 + t / tpc) * G + m0;
        for (int k = t % tpc; k < M; k += 8 * tpc) {
            double q[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int kk = k + u * tpc;
                q[u] = kk < M ? ld_ctl(p + (int64_t)kk * stride) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) s += q[u];
        }
    }
    lds[t] = s;
    __syncthreads();
    if (t < nc) {
        double u = lds[t * tpc];
        for (int k = 1; k < tpc; ++k) u += lds[t * tpc + k];
        lds[256 + t] = u;
    }
    __syncthreads();
    if (t < nc) lds[t] = lds[256 + t];
    __syncthreads();
}

// The control-block fields the last workgroup's thread 0 needs, read once
// with control loads issued together (one memory round trip instead of one
// per field), and g_j.
struct Snap {
    double eta, omega, omega_pre, basis_bytes, tol_abs, gj;
    int literal, reorths, iters, max_iters, breakdowns;
};
__device__ __forceinline__ Snap snapshot(const Epi& e) {
    const State* st = e.st;
    Snap z;
    z.eta = ld_ctl(&st->eta);
    z.omega = ld_ctl(&st->omega);
    z.omega_pre = ld_ctl(&st->omega_pre);
    z.basis_bytes = ld_ctl(&st->basis_bytes);
    z.tol_abs = ld_ctl(&st->tol_abs);
    z.literal = ld_ctl(&st->literal);
    z.reorths = ld_ctl(&st->reorths);
    z.iters = ld_ctl(&st->iters);
    z.max_iters = ld_ctl(&st->max_iters);
    z.breakdowns = ld_ctl(&st->breakdowns);
    z.gj = ld_ctl(&e.g[e.j]);
    return z;
}

// What the last workgroup's step logic reads that no workgroup of the launch
// writes: the SpMV's ||A v||^2 partials (the first batch of sum_partials: each
// thread's loads at t, t + 256, ...), H column j, the earlier rotations and the
// control block.  The last workgroup issues all of these loads together with
// those of its final column sums, so they cost one memory round trip instead
// of one each.  Loads use clamped indices (no branches); values past the end
// are masked where they are used.
constexpr int kPreOm = 8;
constexpr int kPreRows = (kMaxRestart + 255) / 256;  // rows of H column j per thread
struct Pre {
    double om[kPreOm];
    double h[kPreRows], c[kPreRows], s[kPreRows], u[kPreRows];
    Snap z;
};
__device__ __forceinline__ void prefetch(const Epi& e, Pre& p) {
    if (e.mode == EPI_STORE) return;
    const int t = threadIdx.x, j = e.j;
    if (e.mode == EPI_STEP_CHECK || e.mode == EPI_FUSED_CHECK) {
#pragma unroll
        for (int u = 0; u < kPreOm; ++u) p.om[u] = ld_ctl(e.extra + min(t + 256 * u, e.extra_G - 1));
    }
    const double* h = e.H + (int64_t)j * (e.m + 1);
    const int jc = max(j - 1, 0);
#pragma unroll
    for (int k = 0; k < kPreRows; ++k) {
        const int i = t + 256 * k;
        p.h[k] = h[min(i, j)];
        p.c[k] = e.cs[min(i, jc)];
        p.s[k] = e.sn[min(i, jc)];
        p.u[k] = 0.0;
    }
    p.z = snapshot(e);
}

// Fig. 1 steps 12-17 for column j once h_{1:j+1,j} is final: breakdown test,
// Givens rotations, implicit residual, end-of-cycle decision.  Called by all
// threads of one workgroup; H column j, cs and sn are staged in LDS; z is
// valid in thread 0.  Results go to memory with plain stores (read by later
// kernels on the stream and by the host after it synchronises).
__device__ __forceinline__ void finish_step(const Epi& e, int breakdown, double hn, const Snap& z, double* lds,
                                            const Pre& p) {
    State& s = *e.st;
    const int j = e.j;
    double* h = e.H + (int64_t)j * (e.m + 1);
    double* lh = lds;                // j + 2 entries
    double* lc = lds + (j + 2);      // j entries
    double* ls = lc + j;             // j entries
#pragma unroll
    for (int k = 0; k < kPreRows; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i <= j) lh[i] = p.h[k];
        if (i < j) {
            lc[i] = p.c[k];
            ls[i] = p.s[k];
        }
    }
    __syncthreads();
    if (!isfinite(hn)) {
        if (threadIdx.x == 0) {
            s.active = 0;
            s.stop = 1;
            s.status = CB_ERR_NONFINITE;
            if (e.prog) __hip_atomic_store(&e.prog[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        return;
    }
    if (threadIdx.x == 0) {
        if (hn == 0.0) breakdown = 1;
        lh[j + 1] = hn;
        // the earlier rotations in order; the entry carried from rotation i to
        // i+1 stays in a register, and the LDS reads of each chunk of 8
        // rotations are issued together ahead of the arithmetic (chunks of 8
        // keep this thread's registers below the kernels' main loops)
        double carry = lh[0];
        for (int i0 = 0; i0 < j; i0 += 8) {
            double b[8], c[8], sn[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int i = min(i0 + k, j - 1);
                b[k] = lh[i + 1];
                c[k] = lc[i];
                sn[k] = ls[i];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (i0 + k < j) {
                    lh[i0 + k] = c[k] * carry + sn[k] * b[k];
                    carry = -sn[k] * carry + c[k] * b[k];
                }
            }
        }
        lh[j] = carry;
        const double rho = sqrt(lh[j] * lh[j] + hn * hn);
        const double c = lh[j] / rho, sn = hn / rho;
        e.cs[j] = c;
        e.sn[j] = sn;
        lh[j] = rho;
        lh[j + 1] = 0.0;
        const double g1 = -sn * z.gj;
        e.g[j + 1] = g1;
        e.g[j] = c * z.gj;
        const int iters = z.iters + 1;
        const double gabs = fabs(g1);
        s.iters = iters;
        s.steps = j + 1;
        s.gabs = gabs;
        e.hist[j] = gabs;
        const bool ended = gabs <= z.tol_abs || breakdown || iters >= z.max_iters || j + 1 == e.m;
        if (ended) {
            s.active = 0;
            s.breakdowns = z.breakdowns + breakdown;
        }
        // the host paces its launches by these (they order nothing on the
        // GPU); every kProgressEvery steps and at the end only, since the
        // launch cannot complete before its write to host memory has
        if (e.prog) {
            if (ended) __hip_atomic_store(&e.prog[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            if (ended || (j + 1) % kProgressEvery == 0)
                __hip_atomic_store(&e.prog[0], j + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) h[i] = lh[i];
}

// LDS (doubles) the epilogue needs: the column sums, or H column j with the
// rotations for the Givens update of the solver modes.
constexpr int kEpiLds = 3 * (kMaxRestart + 2) > 512 ? 3 * (kMaxRestart + 2) : 512;

// Ticket counters: a top counter and one counter per group of 32 workgroups,
// each in its own 128-byte line (same-address device-scope atomics serialise,
// so a single counter for ~1000 workgroups costs tens of microseconds).  A
// launch may use at most kCounterBytes / 128 - 1 group lines.
constexpr int kTicketGroup = 32;
constexpr int kCounterLine = 32;  // unsigned words per 128-byte line
constexpr int kMaxTicketGroups = kCounterBytes / 128 - 1;

__device__ __forceinline__ bool draw_last(unsigned* c, unsigned count) {
    const bool last = __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == count - 1;
    if (last) __hip_atomic_store(c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // ready for the next launch
    return last;
}

// The two-level reduction of the partials partials[c * G + g] (g = blockIdx.x
// < G; the columns of workgroup (g, y) are [y cw, min(ncols, (y+1) cw))).
// Returns true in the one workgroup that finishes last; there lds[c] (c <
// min(ncols, 256), columns in chunks of 256 handled by reduce_final) is not yet
// formed -- reduce_final does that.
__device__ __forceinline__ bool reduce_tickets(const Epi& e, double* partials, double* lds) {
    __shared__ int flag;
    const int G = e.G, ng = (G + kTicketGroup - 1) / kTicketGroup;
    const int q = blockIdx.x / kTicketGroup;
    const int m0 = q * kTicketGroup, gsize = min(kTicketGroup, G - m0);
    const int c0 = blockIdx.y * e.cw, c1 = min(e.ncols, c0 + e.cw);
    __builtin_amdgcn_s_waitcnt(0);  // this thread's partial stores have completed
    __syncthreads();
    if (threadIdx.x == 0)
        flag = draw_last(e.counter + kCounterLine * (1 + blockIdx.y * ng + q), (unsigned)gsize);
    __syncthreads();
    if (!flag) return false;
    // the group's sums, over the partial of its first workgroup
    for (int a = c0; a < c1; a += 256) {
        const int nc = min(256, c1 - a);
        reduce_range(partials, G, m0, gsize, 1, a, nc, lds);
        for (int i = threadIdx.x; i < nc; i += blockDim.x) store_partial(partials + (int64_t)(a + i) * G + m0, lds[i]);
        __syncthreads();
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // a launch with a single group has no second round: its last workgroup
    // reads its own group sums back
    if (gridDim.y * ng == 1) return true;
    if (threadIdx.x == 0) flag = draw_last(e.counter, gridDim.y * (unsigned)ng);
    __syncthreads();
    return flag != 0;
}

// In the last workgroup: lds[i] = the full sum of column a + i, i < nc.
__device__ __forceinline__ void reduce_final(const Epi& e, const double* partials, int a, int nc, double* lds) {
    const int ng = (e.G + kTicketGroup - 1) / kTicketGroup;
    reduce_range(partials, e.G, 0, ng, kTicketGroup, a, nc, lds);
}

// sum of p[0 .. G) in a fixed order, valid in thread 0 (blockDim.x == 256):
// thread t adds p[t], p[t + 256], ... in order, eight loads in flight at a
// time, then the threads are summed with block_sum.
__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int G) {
    double t = 0.0;
    for (int k = threadIdx.x; k < G; k += 8 * 256) {
        double q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] = k + u * 256 < G ? ld_ctl(p + k + u * 256) : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) t += q[u];
    }
    return block_sum<256>(t);
}

// Fig. 1 steps 6-12 once ||w||^2 = t after a Gram-Schmidt pass is known
// (the STEP_CHECK / FUSED_CHECK / REORTH_FINISH modes; last workgroup, all
// threads, p from prefetch): h_{j+1,j}, the step 7 test, the breakdown test,
// then the Givens update of finish_step when the step is complete.  In
// FUSED_CHECK mode u (p.u, also in e.out) is added to H column j when the
// second pass is needed, else dropped.
__device__ __forceinline__ void step_logic(const Epi& e, double t, double* lds, const Pre& p) {
    // the SpMV's ||A v||^2 partials, when this step needs omega: the sums of
    // sum_partials, from the prefetched first batch when that is all of them
    double om2 = 0.0;
    if (e.mode != EPI_REORTH_FINISH) {
        if (e.extra_G <= kPreOm * 256) {
            double a = 0.0;
#pragma unroll
            for (int u = 0; u < kPreOm; ++u) a += (int)threadIdx.x + 256 * u < e.extra_G ? p.om[u] : 0.0;
            om2 = block_sum<256>(a);
        } else {
            om2 = sum_partials(e.extra, e.extra_G);
        }
    }
    __shared__ int do_finish, bd, keep_u;
    __shared__ double hn_s;
    const Snap& z = p.z;
    if (threadIdx.x == 0) {
        State& s = *e.st;
        do_finish = 0;
        bd = 0;
        keep_u = 0;
        const double hn = sqrt(t);
        s.hn2 = t;
        s.hn = hn;
        hn_s = hn;
        if (e.mode == EPI_STEP_CHECK || e.mode == EPI_FUSED_CHECK) {
            const double omega = sqrt(om2);
            const bool fused = e.mode == EPI_FUSED_CHECK;
            s.om2 = om2;
            s.omega = omega;
            // the first projection and update (and the fused second projection)
            s.basis_bytes = z.basis_bytes + (fused ? 3.0 : 2.0) * (e.j + 1) * e.col_bytes;
            if (hn < z.eta * omega) {
                s.reorth = 1;  // steps 7-11 follow
                s.omega_pre = hn;
                keep_u = fused;  // a fused launch has computed u already
            } else {
                s.reorth = 0;
                do_finish = 1;
            }
        } else {  // EPI_REORTH_FINISH
            s.reorths = z.reorths + 1;
            // the second update, and the second projection if it ran apart
            s.basis_bytes = z.basis_bytes + (e.fused ? 1.0 : 2.0) * (e.j + 1) * e.col_bytes;
            bd = z.literal ? (hn < z.eta * z.omega) : (hn < z.eta * z.omega_pre);
            s.reorth = 0;
            do_finish = 1;
        }
    }
    __syncthreads();
    if (keep_u) {  // h_{1:j+1,j} += u
        double* h = e.H + (int64_t)e.j * (e.m + 1);
#pragma unroll
        for (int k = 0; k < kPreRows; ++k) {
            const int i = threadIdx.x + 256 * k;
            if (i < e.ncols - 1) h[i] = p.h[k] + p.u[k];
        }
    }
    if (do_finish) finish_step(e, bd, hn_s, z, lds, p);
}

// Run by every workgroup of the launch after its partials are written
// (all threads; blockDim.x == 256).
__device__ __forceinline__ void epilogue(const Epi& e, double* partials, double* lds) {
    if (!reduce_tickets(e, partials, lds)) return;
    Pre p;
    prefetch(e, p);  // in flight with the final sums' loads
    if (e.mode == EPI_FUSED_CHECK) {
        // u_c (c < ncols - 1) into e.out and p.u, ||w||^2 from the last column
        __shared__ double nn;
#pragma unroll
        for (int k = 0; k <= kPreRows; ++k) {
            const int c0 = 256 * k;
            if (c0 >= e.ncols) break;
            const int nc = min(256, e.ncols - c0);
            reduce_final(e, partials, c0, nc, lds);
            const int i = threadIdx.x;
            if (i < nc) {
                if (c0 + i < e.ncols - 1) {
                    e.out[c0 + i] = lds[i];
                    if (k < kPreRows) p.u[k] = lds[i];
                } else {
                    nn = lds[i];
                }
            }
            __syncthreads();
        }
        step_logic(e, nn, lds, p);
        return;
    }
    if ((e.mode == EPI_STORE && e.ncols > 1) || e.mode == EPI_REORTH_PROJECT) {
        double* h = e.H + (int64_t)e.j * (e.m + 1);
#pragma unroll
        for (int k = 0; k <= kPreRows; ++k) {
            const int c0 = 256 * k;
            if (c0 >= e.ncols) break;
            const int nc = min(256, e.ncols - c0);
            reduce_final(e, partials, c0, nc, lds);
            const int i = threadIdx.x;
            if (i < nc) {
                const double u = lds[i];
                e.out[c0 + i] = u;
                if (e.mode == EPI_REORTH_PROJECT && k < kPreRows) h[c0 + i] = p.h[k] + u;
            }
            __syncthreads();
        }
        return;
    }
    // one sum (a squared norm)
    reduce_final(e, partials, 0, 1, lds);
    const double t = lds[0];
    if (e.mode == EPI_STORE) {
        if (threadIdx.x == 0) e.out[0] = t;
        return;
    }
    step_logic(e, t, lds, p);
}

}  // namespace dev
}  // namespace cb
