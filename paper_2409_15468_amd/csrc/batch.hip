// Restarted GMRES with a compressed basis (Fig. 1) for small systems, one
// workgroup per system and many systems per launch.
//
// A system of up to a few ten thousand rows cannot fill the GPU: the
// multi-workgroup path spends most of its time in launch latency.  Here one
// workgroup of 512 threads runs a whole solve -- every cycle, step and
// restart -- with its scalars (H column, Givens rotations, g, R, y) in LDS and
// its vectors and basis in its own device workspace, which stays in the
// caches.  Workgroups take systems from the launch's list with an atomic
// ticket until the list is empty, so a launch is persistent over the batch and
// slots free up as systems finish.
//
// Wave w of the workgroup owns the 512-row tiles w, w + 8, w + 16, ... of
// every vector, with the same lane-to-row map and the same tile codecs as the
// multi-workgroup kernels, so stored columns have the same layout and bits.
// Each thread reads and writes only its own rows of w and x; only the SpMV
// reads other rows (of v), after a barrier.  All reductions run in a fixed
// order (lane tree, then the 8 waves in index order), so a system's result
// does not depend on the workgroup that solves it or on the rest of the batch.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "cb_internal.hpp"
#include "codec.hpp"
#include "reduce.hpp"
#include "tiles.hpp"

namespace cb {

using namespace dev;

namespace {

constexpr int kBT = kBatchThreads;
constexpr int kBW = kBT / 64;  // waves per workgroup
constexpr int kMR = kBatchMaxRestart;

// a system as the kernel sees it; the workspace is already carved up
struct BatchItem {
    const int32_t* row_ptr;
    const int32_t* col;
    const double* val;
    const double* b;
    double* x;
    unsigned char* vals;  // basis columns, col_bytes apart
    uint32_t* exps;       // FRSZ2 block exponents, exp_stride words apart (NULL otherwise)
    double* v;            // the FP64 basis vector the next SpMV reads
    double* w;
    int64_t col_bytes, exp_stride;
    int32_t n, nnz, m, format;
    double tol;
};

struct BatchOpts {
    double eta;
    int32_t max_iters;
    int32_t literal;
};

// A serving-ring descriptor: the system's device buffers (in `it`) and the
// host-memory copies of its inputs and output.
struct RingDesc {
    BatchItem it;
    const int32_t* h_row_ptr;
    const int32_t* h_col;
    const double* h_val;
    const double* h_b;
    const double* h_x0;
    double* h_x;
};

// The ring's control words (host memory, pinned, mapped, coherent): tail and
// stop in cache lines of their own, then per slot the done word (sequence
// number + 1 once the slot's result is final) and the launch that served it.
struct RingCtl {
    unsigned tail;
    unsigned pad0[31];
    unsigned stop;
    unsigned pad1[31];
    unsigned done[kRingSlots];
    unsigned served_by[kRingSlots];
};

struct BatchLayout {
    int64_t vals, exps, v, w, total;
};

int64_t al256(int64_t x) { return (x + 255) & ~int64_t(255); }

BatchLayout batch_layout(int32_t n, int32_t m, int fmt) {
    BatchLayout L;
    int64_t off = 0;
    auto take = [&](int64_t bytes) { int64_t o = off; off += al256(bytes); return o; };
    L.vals = take(column_bytes(fmt, n) * (m + 1));
    L.exps = take(exponent_words(fmt, n) * 4 * (m + 1));
    L.v = take(padded_rows(n) * 8);
    L.w = take(padded_rows(n) * 8);
    L.total = off;
    return L;
}

struct Shared {
    double red[kBW][kMR + 2];  // per-wave column sums
    double h[kMR + 2];         // column j of H, rotated into column j of R
    double u[kMR + 1];         // second-pass projections
    double cs[kMR], sn[kMR];   // Givens rotations
    double g[kMR + 1];         // rotated right-hand side
    double R[kMR * (kMR + 1) / 2];  // R packed by columns: column i at i(i+1)/2
    double y[kMR];
    double part[kBW];
    double gabs;
    int item;
};
static_assert(sizeof(Shared) <= 65536, "batch solver LDS");

// Sum over the workgroup of one value per thread; every thread gets the same
// result (lane tree, then the waves in index order).
__device__ __forceinline__ double wg_sum(double v, Shared& S) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) S.part[wave] = v;
    __syncthreads();
    double t = S.part[0];
#pragma unroll
    for (int k = 1; k < kBW; ++k) t += S.part[k];
    __syncthreads();
    return t;
}

// first tile of this wave and the stride between its tiles
__device__ __forceinline__ int tile_first() { return (threadIdx.x >> 6) * kTile; }
constexpr int kTileStride = kBW * kTile;

// ||x||^2 over the system's rows
template <int FMT>
__device__ double wg_sumsq(const double* x, int n, int np, Shared& S) {
    const int lane = threadIdx.x & 63;
    double t = 0.0;
    for (int tile0 = tile_first(); tile0 < np; tile0 += kTileStride) {
        double xv[8];
        load_rows<FMT>(x, tile0, lane, n, xv);
#pragma unroll
        for (int q = 0; q < 8; ++q) t = fma(xv[q], xv[q], t);
    }
    return wg_sum(t, S);
}

// y = A x (b == NULL) or y = b - A x, one thread per row, nonzeros in CSR
// order; returns ||y||^2.
template <int FMT>
__device__ double wg_spmv(const BatchItem& it, const double* x, const double* b, double* y, int np,
                          Shared& S) {
    using M = Map<FMT>;
    const int lane = threadIdx.x & 63;
    double t = 0.0;
    for (int tile0 = tile_first(); tile0 < np; tile0 += kTileStride) {
        double out[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int r = tile0 + M::row(lane, q);
            double s = 0.0;
            if (r < it.n) {
                const int k1 = it.row_ptr[r + 1];
                for (int k = it.row_ptr[r]; k < k1; ++k) s = fma(it.val[k], x[it.col[k]], s);
                if (b) s = b[r] - s;
            }
            out[q] = s;
            t = fma(s, s, t);
        }
        store_rows<FMT>(y, tile0, lane, it.n, out);
    }
    return wg_sum(t, S);
}

// out[c] = <D(v_c), w> for c < jc (Fig. 1 step 5: all against the same w)
template <int FMT>
__device__ void wg_project(const BasisView& V, int jc, const double* w, double* out, Shared& S) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c = lane; c < jc; c += 64) S.red[wave][c] = 0.0;
    for (int tile0 = tile_first(); tile0 < V.np; tile0 += kTileStride) {
        double wv[8];
        load_rows<FMT>(w, tile0, lane, V.n, wv);
        if (tile0 + kTile <= V.np) project_tile_narrow<FMT, kFull>(V, 0, jc, tile0, lane, wv, S.red[wave]);
        else project_tile_narrow<FMT, 0>(V, 0, jc, tile0, lane, wv, S.red[wave]);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < jc; c += kBT) {
        double s = S.red[0][c];
#pragma unroll
        for (int k = 1; k < kBW; ++k) s += S.red[k][c];
        out[c] = s;
    }
    __syncthreads();
}

// w[k] += sign * sum_{c<jc} coef[c] D(v_c)[k] (the sum first, then the add);
// returns ||w||^2 after the update.
template <int FMT>
__device__ double wg_update(const BasisView& V, int jc, const double* coef, double* w, int sign, Shared& S) {
    const int lane = threadIdx.x & 63;
    double t = 0.0;
    for (int tile0 = tile_first(); tile0 < V.np; tile0 += kTileStride) {
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        // single-buffered: the one-workgroup solver has no registers to spare
        if (tile0 + kTile <= V.np) subtract_tile<FMT, 4, kFull, false>(V, jc, coef, tile0, lane, acc);
        else subtract_tile<FMT, 4, 0, false>(V, jc, coef, tile0, lane, acc);
        double wv[8];
        load_rows<FMT>(w, tile0, lane, V.n, wv);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            wv[q] = sign > 0 ? wv[q] + acc[q] : wv[q] - acc[q];
            t = fma(wv[q], wv[q], t);
        }
        store_rows<FMT>(w, tile0, lane, V.n, wv);
    }
    return wg_sum(t, S);
}

// v = w / d (IEEE division per entry, Fig. 1 steps 1 and 13) and column col of
// the basis := Q(v) (step 14).  Returns true, in every thread, if a stored
// value is not finite.
template <int FMT>
__device__ bool wg_store(const BasisView& V, int col, const double* w, double d, double* v) {
    const int lane = threadIdx.x & 63;
    unsigned char* vals = const_cast<unsigned char*>(V.values) + (int64_t)col * V.col_bytes;
    uint32_t* ex = V.exps ? const_cast<uint32_t*>(V.exps) + (int64_t)col * V.exp_stride : nullptr;
    bool bad = false;
    for (int tile0 = tile_first(); tile0 < V.np; tile0 += kTileStride) {
        double vv[8];
        load_rows<FMT>(w, tile0, lane, V.n, vv);
#pragma unroll
        for (int q = 0; q < 8; ++q) vv[q] = vv[q] / d;
        store_rows<FMT>(v, tile0, lane, V.n, vv);
        bad |= encode_tile<FMT>(vals, ex, V.np, tile0, lane, vv);
    }
    return __syncthreads_or(bad) != 0;
}

// One solve, all threads of the workgroup.  Scalars are computed redundantly
// by every thread from LDS values, so every branch is uniform.
template <int FMT>
__device__ void batch_solve(const BatchItem& it, const BatchOpts& o, cb_result* res, Shared& S) {
    const int n = it.n, m = it.m, tid = threadIdx.x;
    const int np = 32 * ((n + 31) / 32);
    BasisView V;
    V.values = it.vals;
    V.exps = it.exps;
    V.col_bytes = it.col_bytes;
    V.exp_stride = it.exp_stride;
    V.n = n;
    V.np = np;
    double* v = it.v;
    double* w = it.w;
    const double cbytes = (double)V.col_bytes;

    int iters = 0, cycles = 0, reorths = 0, breakdowns = 0, converged = 0, status = CB_OK;
    double rel = -1.0, gabs = -1.0, basis_bytes = 0.0;
    bool bad = false;
    const double nb = sqrt(wg_sumsq<FMT>(it.b, n, np, S));
    const double tol_abs = it.tol * nb;
    if (nb == 0.0) {
        for (int i = tid; i < n; i += kBT) it.x[i] = 0.0;
        converged = 1;
        rel = 0.0;
        gabs = 0.0;
    } else if (!isfinite(nb)) {
        status = CB_ERR_NONFINITE;
    } else {
        for (;;) {
            // restart (steps 1 and 18): r = b - A x, beta, the stop test of Eq. 4
            const double beta = sqrt(wg_spmv<FMT>(it, it.x, it.b, w, np, S));
            rel = beta / nb;
            if (!isfinite(beta) || bad) { status = CB_ERR_NONFINITE; break; }
            if (beta <= tol_abs) { converged = 1; break; }
            if (iters >= o.max_iters) { status = CB_ERR_NOT_CONVERGED; break; }
            cycles += 1;
            for (int i = tid; i <= m; i += kBT) S.g[i] = i == 0 ? beta : 0.0;
            bad |= wg_store<FMT>(V, 0, w, beta, v);
            int steps = 0;
            bool nonfinite = false;
            for (int j = 0; j < m; ++j) {
                // v (and g) visible to the whole workgroup
                __syncthreads();
                const double omega = sqrt(wg_spmv<FMT>(it, v, nullptr, w, np, S));
                wg_project<FMT>(V, j + 1, w, S.h, S);
                double hn = sqrt(wg_update<FMT>(V, j + 1, S.h, w, -1, S));
                basis_bytes += 2.0 * (j + 1) * cbytes;
                int bd = 0;
                if (hn < o.eta * omega) {  // step 7: re-orthogonalise
                    const double omega_pre = hn;
                    wg_project<FMT>(V, j + 1, w, S.u, S);
                    for (int c = tid; c <= j; c += kBT) S.h[c] += S.u[c];
                    hn = sqrt(wg_update<FMT>(V, j + 1, S.u, w, -1, S));
                    reorths += 1;
                    basis_bytes += 2.0 * (j + 1) * cbytes;
                    bd = o.literal ? (hn < o.eta * omega) : (hn < o.eta * omega_pre);
                }
                if (!isfinite(hn)) { nonfinite = true; break; }
                if (hn == 0.0) bd = 1;
                if (tid == 0) {
                    // steps 15-16: old rotations on column j, the new rotation, g
                    double* h = S.h;
                    h[j + 1] = hn;
                    double carry = h[0];
                    for (int i0 = 0; i0 < j; i0 += 16) {  // LDS reads of 16 rotations ahead
                        double b1[16], c[16], s[16];
#pragma unroll
                        for (int k = 0; k < 16; ++k) {
                            const int i = min(i0 + k, j - 1);
                            b1[k] = h[i + 1];
                            c[k] = S.cs[i];
                            s[k] = S.sn[i];
                        }
#pragma unroll
                        for (int k = 0; k < 16; ++k) {
                            if (i0 + k < j) {
                                h[i0 + k] = c[k] * carry + s[k] * b1[k];
                                carry = -s[k] * carry + c[k] * b1[k];
                            }
                        }
                    }
                    h[j] = carry;
                    const double rho = sqrt(h[j] * h[j] + hn * hn);
                    const double c = h[j] / rho, s = hn / rho;
                    S.cs[j] = c;
                    S.sn[j] = s;
                    h[j] = rho;
                    S.g[j + 1] = -s * S.g[j];
                    S.g[j] = c * S.g[j];
                    double* Rc = S.R + j * (j + 1) / 2;
                    for (int i = 0; i <= j; ++i) Rc[i] = h[i];
                    S.gabs = fabs(S.g[j + 1]);
                }
                __syncthreads();
                gabs = S.gabs;
                iters += 1;
                steps = j + 1;
                if (gabs <= tol_abs || bd || iters >= o.max_iters || j + 1 == m) {
                    breakdowns += bd;
                    break;
                }
                bad |= wg_store<FMT>(V, j + 1, w, hn, v);
            }
            if (nonfinite) { status = CB_ERR_NONFINITE; break; }
            // step 17: R y = g by columns (wave 0; rows r = lane, lane + 64),
            // then x += V y
            if (tid < 64) {
                double r0 = tid < steps ? S.g[tid] : 0.0;
                double r1 = tid + 64 < steps ? S.g[tid + 64] : 0.0;
                for (int i = steps - 1; i >= 0; --i) {
                    const double* Rc = S.R + i * (i + 1) / 2;
                    const double gi = i < 64 ? readlane_f64(r0, i) : readlane_f64(r1, i - 64);
                    const double yi = gi / Rc[i];
                    if (tid == 0) S.y[i] = yi;
                    if (tid < i) r0 -= Rc[tid] * yi;
                    if (tid + 64 < i) r1 -= Rc[tid + 64] * yi;
                }
            }
            __syncthreads();
            wg_update<FMT>(V, steps, S.y, it.x, +1, S);
            basis_bytes += (double)steps * cbytes;
        }
    }
    if (tid == 0) {
        res->iterations = iters;
        res->restarts = cycles;
        res->reorths = reorths;
        res->breakdowns = breakdowns;
        res->converged = converged;
        res->status = status;
        res->rel_residual = rel;
        res->implicit_rel_residual = gabs >= 0 ? gabs / (nb > 0 ? nb : 1.0) : -1.0;
        res->seconds = 0.0;
        res->basis_bytes = basis_bytes;
    }
    __syncthreads();
}

// A descriptor, read with control loads (the same device addresses may have
// held an earlier launch's descriptors).
__device__ __forceinline__ BatchItem load_item(const BatchItem* p) {
    static_assert(sizeof(BatchItem) % 8 == 0, "descriptor size");
    uint64_t raw[sizeof(BatchItem) / 8];
    const uint64_t* src = reinterpret_cast<const uint64_t*>(p);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(BatchItem) / 8); ++k) raw[k] = ld_ctl(src + k);
    BatchItem it;
    __builtin_memcpy(&it, raw, sizeof(BatchItem));
    return it;
}

// Persistent over the batch: each workgroup takes the next system until the
// list is exhausted.  *next must read 0 at launch.
__global__ __launch_bounds__(kBT) void k_batch(const BatchItem* __restrict__ items, int count,
                                               unsigned* next, BatchOpts o, cb_result* results) {
    __shared__ Shared S;
    for (;;) {
        if (threadIdx.x == 0) S.item = (int)atomicAdd(next, 1u);
        __syncthreads();
        const int i = S.item;
        __syncthreads();
        if (i >= count) return;
        const BatchItem it = load_item(items + i);
        switch (it.format) {
        case CB_F64: batch_solve<CB_F64>(it, o, results + i, S); break;
        case CB_F32: batch_solve<CB_F32>(it, o, results + i, S); break;
        case CB_F16: batch_solve<CB_F16>(it, o, results + i, S); break;
        case CB_FRSZ2_16: batch_solve<CB_FRSZ2_16>(it, o, results + i, S); break;
        case CB_FRSZ2_21: batch_solve<CB_FRSZ2_21>(it, o, results + i, S); break;
        default: batch_solve<CB_FRSZ2_32>(it, o, results + i, S); break;
        }
    }
}

// ----------------------------------------------------------------- serving ring
// A persistent launch that takes small solves from a ring of descriptors the
// host publishes while it runs (continuous batching).  The descriptors, the
// inputs they point to (CSR, b, x0), the output x, the results and the
// control words live in host memory that is pinned, mapped and coherent (the
// GPU reads it uncached over the bus); the solve itself runs out of device
// memory.  A workgroup claims the next published descriptor with a
// compare-and-swap on a device counter (so nothing is claimed before it is
// published), copies the inputs into the system's device buffers, solves, writes
// x and the result back, and raises the slot's done word (system-scope release).
// Every wait is bounded: a workgroup leaves when the host sets `stop` and
// nothing is left to claim, when it has found nothing to claim for
// `idle_polls` polls in a row, or -- so that streams sharing its hardware
// queue are not held up for long -- once the launch is older than `slice`
// ticks of the 100 MHz real-time counter; the host relaunches while work is
// pending.
// Loads and stores of the ring's host memory are system-scope atomics, so
// they bypass the GPU caches: a staging area that held an earlier system's
// inputs is never read from a stale cache line.  Polls are relaxed (an
// acquire at system scope would invalidate the caches on every poll); the
// descriptor loads that follow a successful claim are issued only after the
// claim's result has been seen.
template <class T>
__device__ __forceinline__ T ld_sys(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ RingDesc load_desc(const RingDesc* p) {
    static_assert(sizeof(RingDesc) % 8 == 0, "descriptor size");
    uint64_t raw[sizeof(RingDesc) / 8];
    const uint64_t* src = reinterpret_cast<const uint64_t*>(p);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(RingDesc) / 8); ++k)
        raw[k] = __hip_atomic_load(src + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    RingDesc d;
    __builtin_memcpy(&d, raw, sizeof(RingDesc));
    return d;
}

// host memory -> device memory, and back
template <class T>
__device__ __forceinline__ void wg_copy_in(T* __restrict__ dst, const T* __restrict__ src, int64_t count) {
    for (int64_t i = threadIdx.x; i < count; i += kBT) dst[i] = ld_sys(src + i);
}
__device__ __forceinline__ void wg_copy_out(double* __restrict__ dst, const double* __restrict__ src,
                                            int64_t count) {
    for (int64_t i = threadIdx.x; i < count; i += kBT)
        __hip_atomic_store(dst + i, src[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ __launch_bounds__(kBT) void k_batch_ring(const RingDesc* __restrict__ descs, cb_result* results,
                                                    RingCtl* ctl, unsigned* head, BatchOpts o, int idle_polls,
                                                    uint64_t slice, uint32_t launch_id) {
    __shared__ Shared S;
    const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
    for (;;) {
        if (threadIdx.x == 0) {
            int got = -1;
            int idle = 0;
            while (idle < idle_polls && __builtin_amdgcn_s_memrealtime() - t_start < slice) {
                const unsigned t = ld_sys(&ctl->tail);
                const unsigned h = ld_ctl(head);
                if (h < t) {
                    if (atomicCAS(head, h, h + 1) == h) {
                        got = (int)h;
                        break;
                    }
                    continue;  // another workgroup took it: look again at once
                }
                if (ld_sys(&ctl->stop)) break;
                __builtin_amdgcn_s_sleep(127);  // ~8k cycles between polls of the bus
                ++idle;
            }
            S.item = got;
        }
        __syncthreads();
        const int seq = S.item;
        __syncthreads();
        if (seq < 0) return;
        const int slot = seq & (kRingSlots - 1);
        // this CU's first-level cache may still hold lines of an earlier system
        // that used the same device memory: drop them
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const RingDesc d = load_desc(descs + slot);
        const BatchItem& it = d.it;
        // inputs into the device buffers (x0 into x)
        wg_copy_in(const_cast<int32_t*>(it.row_ptr), d.h_row_ptr, (int64_t)it.n + 1);
        wg_copy_in(const_cast<int32_t*>(it.col), d.h_col, (int64_t)it.nnz);
        wg_copy_in(const_cast<double*>(it.val), d.h_val, (int64_t)it.nnz);
        wg_copy_in(const_cast<double*>(it.b), d.h_b, (int64_t)it.n);
        wg_copy_in(it.x, d.h_x0, (int64_t)it.n);
        __syncthreads();
        cb_result* res = results + slot;
        switch (it.format) {
        case CB_F64: batch_solve<CB_F64>(it, o, res, S); break;
        case CB_F32: batch_solve<CB_F32>(it, o, res, S); break;
        case CB_F16: batch_solve<CB_F16>(it, o, res, S); break;
        case CB_FRSZ2_16: batch_solve<CB_FRSZ2_16>(it, o, res, S); break;
        case CB_FRSZ2_21: batch_solve<CB_FRSZ2_21>(it, o, res, S); break;
        default: batch_solve<CB_FRSZ2_32>(it, o, res, S); break;
        }
        wg_copy_out(d.h_x, it.x, (int64_t)it.n);
        if (threadIdx.x == 0)
            __hip_atomic_store(&ctl->served_by[slot], launch_id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");  // this thread's writes, system scope
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(&ctl->done[slot], (unsigned)seq + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

int64_t batch_workspace_bytes(int32_t n, int32_t m, int format) { return batch_layout(n, m, format).total; }

// ----------------------------------------------------------------- serving ring, host side
struct BatchRing {
    unsigned char* host = nullptr;  // pinned, mapped, coherent: RingCtl, descriptors, results
    RingCtl* ctl = nullptr;
    RingDesc* descs = nullptr;
    cb_result* results = nullptr;
    RingCtl* ctl_dev = nullptr;
    RingDesc* descs_dev = nullptr;
    cb_result* results_dev = nullptr;
    unsigned* head = nullptr;       // device: claim counter
    hipEvent_t ended = nullptr;     // recorded after each launch
    bool launched = false;
    uint32_t published = 0;         // next sequence number
    uint32_t launches = 0;
    std::vector<uint8_t> busy;      // slot held by an unfinished system
    int grid = 64, idle_polls = 4096;
    uint64_t slice = 0;             // real-time counter ticks (100 MHz)
    BatchOpts opts{0.7071067811865476, 20000, 0};
};

BatchRing* ring_create(int grid, int idle_polls, double slice_s) {
    BatchRing* r = new BatchRing();
    r->grid = grid;
    r->idle_polls = idle_polls;
    r->slice = (uint64_t)(slice_s * 1e8);
    r->busy.assign(kRingSlots, 0);
    const size_t o_desc = (sizeof(RingCtl) + 255) & ~size_t(255);
    const size_t o_res = o_desc + ((kRingSlots * sizeof(RingDesc) + 255) & ~size_t(255));
    const size_t total = o_res + kRingSlots * sizeof(cb_result);
    void* h = nullptr;
    if (hipHostMalloc(&h, total, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
        delete r;
        return nullptr;
    }
    std::memset(h, 0, total);
    r->host = static_cast<unsigned char*>(h);
    void* dptr = nullptr;
    if (hipHostGetDevicePointer(&dptr, h, 0) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&r->head), 256) != hipSuccess ||
        hipMemset(r->head, 0, 256) != hipSuccess ||
        hipEventCreateWithFlags(&r->ended, hipEventDisableTiming) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        ring_destroy(r);
        return nullptr;
    }
    unsigned char* d = static_cast<unsigned char*>(dptr);
    r->ctl = reinterpret_cast<RingCtl*>(r->host);
    r->descs = reinterpret_cast<RingDesc*>(r->host + o_desc);
    r->results = reinterpret_cast<cb_result*>(r->host + o_res);
    r->ctl_dev = reinterpret_cast<RingCtl*>(d);
    r->descs_dev = reinterpret_cast<RingDesc*>(d + o_desc);
    r->results_dev = reinterpret_cast<cb_result*>(d + o_res);
    return r;
}

int ring_publish(BatchRing* r, const cb_batch_item& q, const int32_t* h_row_ptr, const int32_t* h_col,
                 const double* h_val, const double* h_b, const double* h_x0, double* h_x, uint32_t* seq) {
    if (q.A.n < 1 || q.A.n > kBatchMaxN || q.A.nnz < 0 || q.m < 1 || q.m > kBatchMaxRestart ||
        !(q.tol > 0.0) || !batch_format(q.format) || !q.b || !q.x || !q.workspace || !q.A.row_ptr ||
        (q.A.nnz > 0 && (!q.A.col || !q.A.val)) || !h_row_ptr || !h_b || !h_x0 || !h_x ||
        (q.A.nnz > 0 && (!h_col || !h_val)) || !aligned(q.x, 16) || !aligned(q.b, 16) ||
        !aligned(q.workspace, 256) || (int64_t)q.workspace_bytes < batch_workspace_bytes(q.A.n, q.m, q.format))
        return fail(CB_ERR_INVALID_ARG, "ring: bad system");
    const uint32_t s = r->published;
    const int slot = (int)(s & (kRingSlots - 1));
    if (r->busy[slot]) return fail(CB_ERR_WORKSPACE, "ring: all %d slots busy", kRingSlots);
    unsigned char* ws = static_cast<unsigned char*>(q.workspace);
    const BatchLayout lay = batch_layout(q.A.n, q.m, q.format);
    RingDesc d;
    d.it = BatchItem{q.A.row_ptr, q.A.col, q.A.val, q.b, q.x, ws + lay.vals,
                     frsz2_bits_of(q.format) ? reinterpret_cast<uint32_t*>(ws + lay.exps) : nullptr,
                     reinterpret_cast<double*>(ws + lay.v), reinterpret_cast<double*>(ws + lay.w),
                     column_bytes(q.format, q.A.n), exponent_words(q.format, q.A.n),
                     q.A.n, q.A.nnz, q.m, q.format, q.tol};
    d.h_row_ptr = h_row_ptr;
    d.h_col = h_col;
    d.h_val = h_val;
    d.h_b = h_b;
    d.h_x0 = h_x0;
    d.h_x = h_x;
    r->descs[slot] = d;
    std::memset(&r->results[slot], 0, sizeof(cb_result));
    __atomic_store_n(&r->ctl->done[slot], 0u, __ATOMIC_RELAXED);
    r->busy[slot] = 1;
    r->published = s + 1;
    __atomic_store_n(&r->ctl->tail, s + 1, __ATOMIC_RELEASE);  // the descriptor before the count
    *seq = s;
    return CB_OK;
}

bool ring_poll(BatchRing* r, uint32_t seq, cb_result* res, uint32_t* launch) {
    const int slot = (int)(seq & (kRingSlots - 1));
    if (__atomic_load_n(&r->ctl->done[slot], __ATOMIC_ACQUIRE) != seq + 1u) return false;
    if (res) *res = r->results[slot];
    if (launch) *launch = r->ctl->served_by[slot];
    r->busy[slot] = 0;
    return true;
}

bool ring_running(BatchRing* r) {
    return r->launched && hipEventQuery(r->ended) == hipErrorNotReady;
}

uint32_t ring_kick(BatchRing* r, hipStream_t s, int* status) {
    *status = CB_OK;
    if (ring_running(r)) return 0;
    const uint32_t id = ++r->launches;
    k_batch_ring<<<r->grid, kBT, 0, s>>>(r->descs_dev, r->results_dev, r->ctl_dev, r->head, r->opts,
                                         r->idle_polls, r->slice, id);
    if (hipGetLastError() != hipSuccess || hipEventRecord(r->ended, s) != hipSuccess) {
        *status = fail(CB_ERR_HIP, "ring launch failed");
        return 0;
    }
    r->launched = true;
    return id;
}

void ring_stop(BatchRing* r) {
    __atomic_store_n(&r->ctl->stop, 1u, __ATOMIC_RELEASE);
    if (r->launched) (void)hipEventSynchronize(r->ended);
    r->launched = false;
    __atomic_store_n(&r->ctl->stop, 0u, __ATOMIC_RELEASE);
}

void ring_destroy(BatchRing* r) {
    if (!r) return;
    if (r->ctl) ring_stop(r);
    if (r->ended) (void)hipEventDestroy(r->ended);
    if (r->head) (void)hipFree(r->head);
    if (r->host) (void)hipHostFree(r->host);
    delete r;
}

}  // namespace cb

using namespace cb;

extern "C" {

int32_t cbgmres_batch_max_n(void) { return kBatchMaxN; }
int32_t cbgmres_batch_max_restart(void) { return kBatchMaxRestart; }

int64_t cbgmres_batch_workspace_bytes(int32_t n, int32_t m, int format) {
    if (n < 1 || n > kBatchMaxN || m < 1 || m > kBatchMaxRestart || !batch_format(format)) return -1;
    return batch_workspace_bytes(n, m, format);
}

int cbgmres_solve_batch(const cb_batch_item* items, int32_t count, const cb_options* opt,
                        cb_result* results_host, void* stream) {
    if (count < 0 || (count > 0 && (!items || !results_host)))
        return fail(CB_ERR_INVALID_ARG, "bad batch arguments");
    if (count == 0) return CB_OK;
    hipStream_t s = (hipStream_t)stream;
    const double t0 = now_s();
    std::vector<BatchItem> d(count);
    for (int i = 0; i < count; ++i) {
        const cb_batch_item& q = items[i];
        if (!q.b || !q.x || !q.workspace || !q.A.row_ptr || (q.A.nnz > 0 && (!q.A.col || !q.A.val)))
            return fail(CB_ERR_INVALID_ARG, "batch item %d: NULL pointer", i);
        if (q.A.n < 1 || q.A.n > kBatchMaxN || q.A.nnz < 0)
            return fail(CB_ERR_INVALID_ARG, "batch item %d: n=%d out of range [1, %d]", i, q.A.n, kBatchMaxN);
        if (q.m < 1 || q.m > kBatchMaxRestart)
            return fail(CB_ERR_INVALID_ARG, "batch item %d: m=%d out of range [1, %d]", i, q.m,
                        kBatchMaxRestart);
        if (!(q.tol > 0.0) || !std::isfinite(q.tol) || !batch_format(q.format))
            return fail(CB_ERR_INVALID_ARG, "batch item %d: bad tol or format (the generic-l and block-64 "
                        "FRSZ2 formats run through cbgmres_solve)", i);
        if ((reinterpret_cast<uintptr_t>(q.workspace) & 255) != 0)
            return fail(CB_ERR_WORKSPACE, "batch item %d: workspace not 256-byte aligned", i);
        if (!aligned(q.x, 16) || !aligned(q.b, 16))  // both are read in 16-byte pieces
            return fail(CB_ERR_INVALID_ARG, "batch item %d: x and b must be 16-byte aligned", i);
        if ((int64_t)q.workspace_bytes < batch_workspace_bytes(q.A.n, q.m, q.format))
            return fail(CB_ERR_WORKSPACE, "batch item %d: workspace %zu < %lld bytes", i, q.workspace_bytes,
                        (long long)batch_workspace_bytes(q.A.n, q.m, q.format));
        unsigned char* ws = static_cast<unsigned char*>(q.workspace);
        const BatchLayout lay = batch_layout(q.A.n, q.m, q.format);
        d[i] = BatchItem{q.A.row_ptr, q.A.col, q.A.val, q.b, q.x, ws + lay.vals,
                         frsz2_bits_of(q.format) ? reinterpret_cast<uint32_t*>(ws + lay.exps) : nullptr,
                         reinterpret_cast<double*>(ws + lay.v), reinterpret_cast<double*>(ws + lay.w),
                         column_bytes(q.format, q.A.n), exponent_words(q.format, q.A.n),
                         q.A.n, q.A.nnz, q.m, q.format, q.tol};
    }
    BatchOpts o;
    o.eta = (opt && opt->eta > 0) ? opt->eta : 0.7071067811865476;
    o.max_iters = (opt && opt->max_iters > 0) ? opt->max_iters : 20000;
    o.literal = opt ? opt->literal_breakdown : 0;
    // device block: ticket counter, descriptors, results
    const size_t o_items = 256, o_res = o_items + al256((int64_t)count * sizeof(BatchItem));
    const size_t total = o_res + (size_t)count * sizeof(cb_result);
    std::vector<unsigned char> host(o_res, 0);
    std::memcpy(host.data() + o_items, d.data(), (size_t)count * sizeof(BatchItem));
    unsigned char* mem = nullptr;
    CB_HIP(hipMallocAsync(reinterpret_cast<void**>(&mem), total, s));
    int st = CB_OK;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int grid = count < cus ? count : cus;
    if (hipMemcpyAsync(mem, host.data(), o_res, hipMemcpyHostToDevice, s) != hipSuccess) {
        st = fail(CB_ERR_HIP, "descriptor copy failed");
    } else {
        k_batch<<<grid, kBT, 0, s>>>(reinterpret_cast<const BatchItem*>(mem + o_items), count,
                                     reinterpret_cast<unsigned*>(mem), o,
                                     reinterpret_cast<cb_result*>(mem + o_res));
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(results_host, mem + o_res, (size_t)count * sizeof(cb_result), hipMemcpyDeviceToHost,
                           s) != hipSuccess)
            st = fail(CB_ERR_HIP, "batch launch failed");
    }
    (void)hipFreeAsync(mem, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == CB_OK) st = fail(CB_ERR_HIP, "batch solve failed");
    if (st != CB_OK) return st;
    const double dt = now_s() - t0;
    int worst = CB_OK;
    for (int i = 0; i < count; ++i) {
        results_host[i].seconds = dt;
        if (results_host[i].status != CB_OK && worst == CB_OK) worst = results_host[i].status;
    }
    return worst;
}

}  // extern "C"
