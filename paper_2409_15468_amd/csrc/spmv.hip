// CSR sparse matrix-vector product in FP64 (Fig. 1 steps 1 and 3) with the
// squared norm of the result fused in (step 4).
//
// Short rows (the 5- and 7-point stencils): a wave stages the products of 64
// rows' nonzeros in LDS from coalesced loads and each lane adds its row's
// products in CSR order (spmv_rows_staged).  Longer rows: a group of LPR lanes
// works on one row: lane i of the group accumulates the row's entries i,
// i+LPR, ... with FMA in CSR order, then the group sums with a fixed tree of
// cross-lane moves (group_sum: DPP inside 16-lane rows); LPR is the power of
// two nearest to half the average row length, so most lanes own one or two
// nonzeros and a row's column indices are read as one coalesced run.  At most
// kSpmvGroups workgroups loop over the row blocks; the row-to-workgroup map
// depends on the matrix only, keeping the norm's reduction order fixed.
#include <climits>

#include "cb_internal.hpp"
#include "epilogue.hpp"
#include "reduce.hpp"
#include "tiles.hpp"

namespace cb {

using namespace dev;

// The row blocks of this workgroup, XCD-aware.  Workgroups are dispatched to
// the XCDs round-robin (w -> XCD w % kXcds) and each XCD has its own L2, so
// when the grid is a multiple of kXcds the nblk blocks are cut into kXcds
// contiguous ranges, one per XCD, whose workgroups take the blocks of the
// range in turn: workgroups of one XCD then work on neighbouring rows at the
// same time and share in its L2 the parts of x those rows read.  Otherwise
// workgroup w takes the blocks w, w + G, ....  Blocks first, first + stride,
// ... below end; the map depends on (nblk, G) only.
struct BlockSeq {
    int first, stride, end;
};
__device__ __forceinline__ BlockSeq xcd_blocks(int nblk) {
    const int G = gridDim.x, w = blockIdx.x;
    if (G % kXcds != 0) return {w, G, nblk};
    const int x = w % kXcds;
    const int lo = (int)((int64_t)nblk * x / kXcds), hi = (int)((int64_t)nblk * (x + 1) / kXcds);
    return {lo + w / kXcds, G / kXcds, hi};
}

// y = A x over the row blocks of 256/LPR rows given by xcd_blocks
// (x[c] read as xs[c] / d when DIV: the normalised vector formed on the fly);
// with b != NULL the result is b - A x.  Returns this thread's share of
// ||y||^2.  Lane li of a row's group of LPR lanes accumulates the row's
// entries li, li + LPR, ... with FMA in CSR order, then the group sums with
// group_sum.  The loads are what limits a row: row pointer, then
// column index and value, then the x gather, each waiting on the one before.
// So each group works on U row blocks at once and issues the loads of every
// level for all U rows (the first two entries per lane, unconditionally, with
// clamped indices) before it waits; entries past 2 LPR in a row, if any, follow
// in a loop.  The sums are the same, in the same order, as one row at a time.
template <int LPR, bool DIV, int U = 4>
__device__ __forceinline__ double spmv_rows(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                            const double* __restrict__ val, const double* __restrict__ xs,
                                            double d, const double* __restrict__ b, double* __restrict__ y) {
    constexpr int RPW = 256 / LPR;
    const int sub = threadIdx.x / LPR;
    const int li = threadIdx.x % LPR;
    const int nblk = (n + RPW - 1) / RPW;
    const BlockSeq bs = xcd_blocks(nblk);
    double nrm = 0.0;
    if (__builtin_amdgcn_readfirstlane(rp[n]) == 0) {  // no entries at all: y = b or 0
        for (int blk = bs.first; blk < bs.end; blk += bs.stride) {
            const int row = blk * RPW + sub;
            if (row < n && li == 0) {
                const double t = b ? b[row] : 0.0;
                y[row] = t;
                nrm = fma(t, t, nrm);
            }
        }
        return nrm;
    }
    for (int blk0 = bs.first; blk0 < bs.end; blk0 += U * bs.stride) {
        int row[U], k0[U], k1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // rows >= n (and blocks past this workgroup's share) have no entries
            const int blk = blk0 + u * bs.stride;
            row[u] = blk < bs.end ? blk * RPW + sub : n;
            const int r = min(row[u], n);
            k0[u] = rp[r];
            k1[u] = rp[min(row[u] + 1, n)];
        }
        int c[U][2];
        double v[U][2];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int k = k0[u] + li + e * LPR;
                // a real entry, or (dropped below) the entry before the row's
                // end: an address the row's own loads bring in anyway, not one
                // that every lane of the launch would hit
                const int kk = k < k1[u] ? k : max(k1[u] - 1, 0);
                c[u][e] = ci[kk];
                v[u][e] = val[kk];
            }
        }
        double xv[U][2];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int e = 0; e < 2; ++e) xv[u][e] = xs[c[u][e]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                if (k0[u] + li + e * LPR < k1[u]) s = fma(v[u][e], DIV ? xv[u][e] / d : xv[u][e], s);
            }
            for (int k = k0[u] + li + 2 * LPR; k < k1[u]; k += LPR) {
                const double xk = DIV ? xs[ci[k]] / d : xs[ci[k]];
                s = fma(val[k], xk, s);
            }
            s = group_sum<LPR>(s);
            if (row[u] < n && li == 0) {
                if (b) s = b[row[u]] - s;
                y[row[u]] = s;
                nrm = fma(s, s, nrm);
            }
        }
    }
    return nrm;
}

// Windowed form of spmv_rows for matrices whose rows reach only nearby
// columns (a band): rows go in blocks of kWinRows; a plan (k_spmv_plan) holds
// each block's smallest and largest column.  A block first stages its row
// pointers and, when the block's window of x fits kWinMax doubles, that window
// (x / d formed there once per element when DIV) in LDS with coalesced loads;
// then each lane loads its entries for 4 rounds of rows at a time into one of
// two register sets, the next set's loads in flight while the current set's
// rows gather x from LDS and are summed (blocks whose window does not fit
// gather from memory).  Scattered gathers of random columns otherwise touch a different
// cache line per lane, and row pointer, entries and x each wait on the one
// before, which bounds the SpMV far below the memory bandwidth.  Each row's
// sum is formed exactly as in spmv_rows (same lanes, same order); the blocks
// go to workgroups by xcd_blocks, a map fixed by the block count and the grid,
// so the norm's partial sums do not depend on timing.
constexpr int kWinRows = 512;  // rows per block (256 measured 3% slower per banded solve)
constexpr int kWinMax = 3072;  // doubles of x staged per block (24 KB: four workgroups per CU)
// The rows of one block of spmv_rows_win once its row pointers (and, STAGED,
// its window of x) sit in LDS.  STAGED is a template argument so that the
// gathers from LDS and those from memory are separate code: mixed in one loop
// the compiler's merged control flow lets a global load and an LDS read share
// a destination register, and every LDS read then waits for all entry loads.
template <int LPR, bool DIV, bool STAGED>
__device__ __forceinline__ void spmv_win_block(int n, int r0, const int* __restrict__ ci,
                                               const double* __restrict__ val, const double* __restrict__ xs,
                                               double d, const double* __restrict__ b, double* __restrict__ y,
                                               const double* xw, const int* rpl, int lo, int span, double& nrm) {
    constexpr int RPW = 256 / LPR;                       // rows per round
    constexpr int U = 4;                                 // rounds per register set
    constexpr int NS = LPR * (kWinRows / 256) / U;       // sets per block
    static_assert(NS >= 2 && NS % 2 == 0, "two register sets in turn");
    const int sub = threadIdx.x / LPR;
    const int li = threadIdx.x % LPR;
    auto gather = [&](int col) -> double {
        if (STAGED) return xw[min(max(col - lo, 0), span - 1)];  // inside the window for every real entry
        return DIV ? xs[col] / d : xs[col];
    };
    struct Set {
        int k0[U], k1[U], c[U][2];
        double v[U][2], bq[U];
    };
    auto issue = [&](Set& t, int set) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int lr = (set * U + u) * RPW + sub;  // row within the block
            t.k0[u] = rpl[lr];
            t.k1[u] = rpl[lr + 1];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int k = t.k0[u] + li + e * LPR;
                const int kk = k < t.k1[u] ? k : max(t.k1[u] - 1, 0);  // as in spmv_rows
                t.c[u][e] = ci[kk];
                t.v[u][e] = val[kk];
            }
            // b at the row, issued with the entries (a row past n reads row n - 1, unused)
            t.bq[u] = b ? b[min(r0 + (set * U + u) * RPW + sub, n - 1)] : 0.0;
        }
    };
    auto consume = [&](const Set& t, int set) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double xv[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) xv[e] = gather(t.c[u][e]);
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                if (t.k0[u] + li + e * LPR < t.k1[u]) s = fma(t.v[u][e], xv[e], s);
            }
            for (int k = t.k0[u] + li + 2 * LPR; k < t.k1[u]; k += LPR) s = fma(val[k], gather(ci[k]), s);
            s = group_sum<LPR>(s);
            const int row = r0 + (set * U + u) * RPW + sub;
            if (row < n && li == 0) {
                if (b) s = t.bq[u] - s;
                y[row] = s;
                nrm = fma(s, s, nrm);
            }
        }
    };
    // two register sets in turn: while one set's rows are summed, the next
    // set's entries are in flight.  No copy from one set into the other and no
    // exit inside the loop, either of which would wait for every load in
    // flight.  (8 rounds per set take 256 registers; 2 per set, or holding the
    // residual kernel to 128, measured 1% slower per banded solve.)
    Set A, B;
    issue(A, 0);
    for (int p = 0; p < NS / 2 - 1; ++p) {
        issue(B, 2 * p + 1);
        consume(A, 2 * p);
        issue(A, 2 * p + 2);
        consume(B, 2 * p + 1);
    }
    issue(B, NS - 1);
    consume(A, NS - 2);
    consume(B, NS - 1);
}

template <int LPR, bool DIV>
__device__ __forceinline__ double spmv_rows_win(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                const double* __restrict__ val, const double* __restrict__ xs,
                                                double d, const double* __restrict__ b, double* __restrict__ y,
                                                const int2* __restrict__ win, double* xw, int* rpl) {
    const int nwin = (n + kWinRows - 1) / kWinRows;
    const BlockSeq bs = xcd_blocks(nwin);
    double nrm = 0.0;
    for (int blk = bs.first; blk < bs.end; blk += bs.stride) {
        const int2 wr = win[blk];
        const int lo = wr.x, span = wr.y - wr.x + 1;  // span <= 0: no entries
        const bool staged = span > 0 && span <= kWinMax;
        const int r0 = blk * kWinRows;
        __syncthreads();  // the previous block's reads of the stage are done
        // row pointers of the block's rows (rows past n: no entries) and the
        // window of x, 12 elements per thread at most (kWinMax / 256), all
        // loads issued before any is used
        constexpr int P = kWinRows / 256;  // row pointers per thread
        int rpa[P];
#pragma unroll
        for (int q = 0; q < P; ++q) rpa[q] = rp[min(r0 + 256 * q + (int)threadIdx.x, n)];
        const int rpb = rp[min(r0 + kWinRows, n)];
        if (staged) {
            constexpr int E = kWinMax / 256;
            double t[E];
#pragma unroll
            for (int u = 0; u < E; ++u) t[u] = xs[lo + min((int)threadIdx.x + 256 * u, span - 1)];
#pragma unroll
            for (int u = 0; u < E; ++u) {
                const int i = (int)threadIdx.x + 256 * u;
                if (i < span) xw[i] = DIV ? t[u] / d : t[u];
            }
        }
#pragma unroll
        for (int q = 0; q < P; ++q) rpl[threadIdx.x + 256 * q] = rpa[q];
        if (threadIdx.x == 0) rpl[kWinRows] = rpb;
        __syncthreads();
        if (staged)
            spmv_win_block<LPR, DIV, true>(n, r0, ci, val, xs, d, b, y, xw, rpl, lo, span, nrm);
        else
            spmv_win_block<LPR, DIV, false>(n, r0, ci, val, xs, d, b, y, xw, rpl, lo, span, nrm);
    }
    return nrm;
}

// The plan of spmv_rows_win: win[blk] = (smallest, largest) column over the
// entries of rows [kWinRows blk, kWinRows (blk + 1)) ∩ [0, n), or (0, -1) when
// they have none.  One workgroup per block.
__global__ __launch_bounds__(256) void k_spmv_plan(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                   int2* __restrict__ win) {
    const int blk = blockIdx.x;
    const int r0 = blk * kWinRows, r1 = min(n, r0 + kWinRows);
    const int k0 = rp[r0], k1 = rp[r1];
    int lo = INT_MAX, hi = -1;
    // the block's entries: a head up to a 16-byte boundary, then 4 at a time
    const int ka = min(k1, (k0 + 3) & ~3);
    for (int k = k0 + (int)threadIdx.x; k < ka; k += 256) {
        lo = min(lo, ci[k]);
        hi = max(hi, ci[k]);
    }
    for (int k = ka + 4 * (int)threadIdx.x; k < k1; k += 4 * 256) {
        if (k + 4 <= k1) {
            const int4 q = *reinterpret_cast<const int4*>(ci + k);
            lo = min(min(lo, q.x), min(min(q.y, q.z), q.w));
            hi = max(max(hi, q.x), max(max(q.y, q.z), q.w));
        } else {
            for (int t = k; t < k1; ++t) {
                lo = min(lo, ci[t]);
                hi = max(hi, ci[t]);
            }
        }
    }
    __shared__ int slo[256], shi[256];
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            slo[threadIdx.x] = min(slo[threadIdx.x], slo[threadIdx.x + h]);
            shi[threadIdx.x] = max(shi[threadIdx.x], shi[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) win[blk] = shi[0] < 0 ? make_int2(0, -1) : make_int2(slo[0], shi[0]);
}

// Short rows (at most 8 nonzeros per row on average): a wave takes 64
// consecutive rows; their nonzeros, a contiguous run of at most 512 entries,
// are read as 8 coalesced loads per lane, multiplied by the gathered x (x[c] /
// d when DIV) into LDS, and each lane then adds its row's products in CSR
// order.  A run longer than 512 entries falls back to one lane per row.
// With b != NULL the result is b - A x.  Returns this thread's share of
// ||y||^2.  The latency chain of a block is row pointers -> column indices
// and values -> x: the 8 loads of each level are issued together
// (unconditionally, entries past the run read its last entry again and are
// dropped), and the next block's row pointers are loaded while this block
// runs, so a block waits on two memory round trips, not sixteen.
constexpr int kStagedMax = 512;
template <bool DIV>
__device__ __forceinline__ double spmv_rows_staged(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                   const double* __restrict__ val, const double* __restrict__ xs,
                                                   double d, const double* __restrict__ b, double* __restrict__ y,
                                                   double* prod) {
    constexpr int C = kStagedMax / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwb = (n + 63) / 64;  // blocks of 64 rows, 4 per workgroup block
    const BlockSeq bs = xcd_blocks((nwb + 3) / 4);
    // the lane's row pointers in workgroup block gb (rows past n: no entries)
    auto ptrs = [&](int gb, int& a, int& e) {
        const int r = min(gb * 4 + wave, nwb - 1) * 64 + lane;
        a = rp[min(r, n)];
        e = rp[min(r + 1, n)];
    };
    double nrm = 0.0;
    int my0 = 0, my1 = 0;
    if (bs.first < bs.end) ptrs(bs.first, my0, my1);
    for (int gb = bs.first; gb < bs.end; gb += bs.stride) {
        const int wb = gb * 4 + wave;
        if (wb >= nwb) break;  // the last workgroup block's missing waves
        const int r = wb * 64 + lane;
        const int c0 = my0, c1 = my1;
        if (gb + bs.stride < bs.end) ptrs(gb + bs.stride, my0, my1);  // the next block's, in flight
        const int k0 = __builtin_amdgcn_readfirstlane(c0);
        const int k1 = __builtin_amdgcn_readlane(c1, 63);
        const double bv = b ? b[min(r, n - 1)] : 0.0;
        double s = 0.0;
        if (k1 - k0 <= kStagedMax) {
            if (k1 > k0) {
                int cc[C];
                double vv[C], xv[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int k = min(k0 + c * 64 + lane, k1 - 1);
                    cc[c] = ci[k];
                    vv[c] = val[k];
                }
#pragma unroll
                for (int c = 0; c < C; ++c) xv[c] = xs[cc[c]];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const bool live = k0 + c * 64 + lane < k1;
                    prod[c * 64 + lane] = live ? vv[c] * (DIV ? xv[c] / d : xv[c]) : 0.0;
                }
            }
            __builtin_amdgcn_wave_barrier();
            for (int k = c0; k < c1; ++k) s += prod[k - k0];
            __builtin_amdgcn_wave_barrier();
        } else {
            for (int k = c0; k < c1; ++k) {
                const double xk = DIV ? xs[ci[k]] / d : xs[ci[k]];
                s = fma(val[k], xk, s);
            }
        }
        if (r < n) {
            if (b) s = bv - s;
            y[r] = s;
            nrm = fma(s, s, nrm);
        }
    }
    return nrm;
}

// Fig. 1 steps 13-14 of the previous step fused with steps 3-4 of this one:
// column col of the basis := Q(w / d) (IEEE division per entry, as k_store),
// and y = A (w / d) with the quotients formed again where the SpMV reads them
// (the same division, so the same values), ||y||^2 per workgroup.  The encode
// runs over the 2048-row groups g = blockIdx.x, +gridDim.x, ...; the SpMV over
// the row blocks.  w is only read, y is another buffer.
// WIN = 0: the staged short-row scheme (lpr 0); WIN = -1: lanes per row
// picked at run time by lpr, no plan; WIN = LPR (8, 16, 32 or 64 lanes per
// row): the windowed rows with the plan `win`.  Each instance holds only its
// scheme, so the short-row kernel keeps its small register count (and its
// occupancy: its loads wait on each other).
template <int FMT, int WIN>
__global__ __launch_bounds__(256) void k_spmv_store(int n, int np, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, const double* __restrict__ val,
                                                    int lpr, const double* __restrict__ w,
                                                    const double* __restrict__ divisor, double* __restrict__ y,
                                                    double* __restrict__ partials, unsigned char* __restrict__ values,
                                                    uint32_t* __restrict__ exps, int32_t* __restrict__ flag,
                                                    const int* __restrict__ guard, int bits, int bs_log,
                                                    const int2* __restrict__ win) {
    if (guard && ld_ctl(guard) == 0) return;
    const double d = ld_ctl(divisor);
    const int lane = threadIdx.x & 63;
    bool bad = false;
    for (int g = blockIdx.x; g * kRowsPerWG < np; g += gridDim.x) {
        const int tile0 = g * kRowsPerWG + (threadIdx.x >> 6) * kTile;
        double v[8];
        load_rows<FMT>(w, tile0, lane, n, v);
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = v[q] / d;
        bad |= encode_tile<FMT>(values, exps, np, tile0, lane, v, bits, bs_log);
    }
    if (bad) atomicOr(flag, 1);
    double nrm;
    if constexpr (WIN > 0) {
        __shared__ double xw[kWinMax];
        __shared__ int rpl[kWinRows + 1];
        nrm = spmv_rows_win<WIN, true>(n, rp, ci, val, w, d, nullptr, y, win, xw, rpl);
    } else if constexpr (WIN == 0) {
        __shared__ double prod[4][kStagedMax];
        nrm = spmv_rows_staged<true>(n, rp, ci, val, w, d, nullptr, y, prod[threadIdx.x >> 6]);
    } else {
        switch (lpr) {
        case 1: nrm = spmv_rows<1, true>(n, rp, ci, val, w, d, nullptr, y); break;
        case 2: nrm = spmv_rows<2, true>(n, rp, ci, val, w, d, nullptr, y); break;
        case 4: nrm = spmv_rows<4, true>(n, rp, ci, val, w, d, nullptr, y); break;
        case 8: nrm = spmv_rows<8, true>(n, rp, ci, val, w, d, nullptr, y); break;
        case 16: nrm = spmv_rows<16, true>(n, rp, ci, val, w, d, nullptr, y); break;
        case 32: nrm = spmv_rows<32, true>(n, rp, ci, val, w, d, nullptr, y); break;
        default: nrm = spmv_rows<64, true>(n, rp, ci, val, w, d, nullptr, y); break;
        }
    }
    const double t = block_sum<256>(nrm);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_spmv_staged(int n, const int* __restrict__ rp,
                                                     const int* __restrict__ ci,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ b, double* __restrict__ y,
                                                     double* __restrict__ partials, int mode,
                                                     const int* __restrict__ guard) {
    if (guard && ld_ctl(guard) == 0) return;
    __shared__ double prod[4][kStagedMax];
    const double nrm = spmv_rows_staged<false>(n, rp, ci, val, x, 1.0, mode ? b : nullptr, y,
                                               prod[threadIdx.x >> 6]);
    if (partials) {
        const double t = block_sum<256>(nrm);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

template <int LPR>
__global__ __launch_bounds__(256) void k_spmv(int n, const int* __restrict__ rp,
                                              const int* __restrict__ ci,
                                              const double* __restrict__ val,
                                              const double* __restrict__ x,
                                              const double* __restrict__ b, double* __restrict__ y,
                                              double* __restrict__ partials, int mode,
                                              const int* __restrict__ guard) {
    if (guard && ld_ctl(guard) == 0) return;
    // row blocks by xcd_blocks (the grid depends on the matrix only)
    const double nrm = spmv_rows<LPR, false>(n, rp, ci, val, x, 1.0, mode ? b : nullptr, y);
    if (partials) {
        const double t = block_sum<256>(nrm);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

// The same with the column-window plan (LPR 8, 16, 32 or 64).
template <int LPR>
__global__ __launch_bounds__(256) void k_spmv_win(int n, const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const double* __restrict__ val,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ b, double* __restrict__ y,
                                                  double* __restrict__ partials, int mode,
                                                  const int* __restrict__ guard, const int2* __restrict__ win) {
    if (guard && ld_ctl(guard) == 0) return;
    __shared__ double xw[kWinMax];
    __shared__ int rpl[kWinRows + 1];
    const double nrm = spmv_rows_win<LPR, false>(n, rp, ci, val, x, 1.0, mode ? b : nullptr, y, win, xw, rpl);
    if (partials) {
        const double t = block_sum<256>(nrm);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

// 0 selects the staged short-row scheme (at most 8 nonzeros per row on
// average), else the lanes per row: the power of two nearest to half the
// average row length.
int spmv_lanes_per_row(int32_t n, int32_t nnz) {
    if ((int64_t)nnz <= 8 * (int64_t)n) return 0;
    double avg = n > 0 ? (double)nnz / (double)n : 1.0;
    int lpr = 1;
    while (lpr < 64 && 2.0 * lpr <= avg) lpr *= 2;
    return lpr;
}

// Workgroups of the SpMV: one per block of rows up to kSpmvGroups, which then
// loop over blocks; few partial sums keep their consumer's reduction short.
int spmv_groups(int32_t n, int32_t nnz) {
    const int lpr = spmv_lanes_per_row(n, nnz);
    const int rpw = lpr ? 256 / lpr : 256;
    const int64_t blocks = ((int64_t)n + rpw - 1) / rpw;
    return (int)(blocks < kSpmvGroups ? blocks : kSpmvGroups);
}

int64_t spmv_plan_bytes(int32_t n) { return 8 * (((int64_t)n + kWinRows - 1) / kWinRows); }

bool spmv_uses_plan(int32_t n, int32_t nnz) { return spmv_lanes_per_row(n, nnz) >= 8; }

void launch_spmv_plan(const cb_csr& A, void* plan, hipStream_t s) {
    const int nwin = (A.n + kWinRows - 1) / kWinRows;
    k_spmv_plan<<<nwin, 256, 0, s>>>(A.n, A.row_ptr, A.col, static_cast<int2*>(plan));
}

void launch_spmv(const cb_csr& A, const double* x, const double* b, double* y, double* partials,
                 int mode, const int* guard, hipStream_t s, const void* plan) {
    const int2* win = static_cast<const int2*>(plan);
    const int lpr = spmv_lanes_per_row(A.n, A.nnz);
    const int G = spmv_groups(A.n, A.nnz);
    if (win && lpr >= 8) {
        switch (lpr) {
        case 8: k_spmv_win<8><<<G, 256, 0, s>>>(A.n, A.row_ptr, A.col, A.val, x, b, y, partials, mode, guard, win); break;
        case 16: k_spmv_win<16><<<G, 256, 0, s>>>(A.n, A.row_ptr, A.col, A.val, x, b, y, partials, mode, guard, win); break;
        case 32: k_spmv_win<32><<<G, 256, 0, s>>>(A.n, A.row_ptr, A.col, A.val, x, b, y, partials, mode, guard, win); break;
        default: k_spmv_win<64><<<G, 256, 0, s>>>(A.n, A.row_ptr, A.col, A.val, x, b, y, partials, mode, guard, win); break;
        }
        return;
    }
#define CB_SPMV_CASE(L)                                                                         \
    case L:                                                                                     \
        k_spmv<L><<<G, 256, 0, s>>>(A.n, A.row_ptr, A.col, A.val, x, b, y, partials, mode, guard); \
        break;
    switch (lpr) {
    case 0:
        k_spmv_staged<<<G, 256, 0, s>>>(A.n, A.row_ptr, A.col, A.val, x, b, y, partials, mode, guard);
        break;
        CB_SPMV_CASE(1)
        CB_SPMV_CASE(2)
        CB_SPMV_CASE(4)
        CB_SPMV_CASE(8)
        CB_SPMV_CASE(16)
        CB_SPMV_CASE(32)
        default:
        CB_SPMV_CASE(64)
    }
#undef CB_SPMV_CASE
}

void launch_spmv_store(int fmt, const cb_csr& A, const cb_basis& V, int col, const double* w,
                       const double* divisor, double* y, double* partials, int32_t* flag, const int* guard,
                       hipStream_t s, const void* plan) {
    const int2* win = static_cast<const int2*>(plan);
    const BasisView b = view_of(V);
    unsigned char* vals = static_cast<unsigned char*>(V.values) + (int64_t)col * b.col_bytes;
    uint32_t* ex = V.exps ? V.exps + (int64_t)col * b.exp_stride : nullptr;
    const int lpr = spmv_lanes_per_row(A.n, A.nnz);
    const int G = spmv_groups(A.n, A.nnz);
#define CB_SS_LAUNCH(F, W)                                                                             \
    k_spmv_store<F, W><<<G, 256, 0, s>>>(A.n, b.np, A.row_ptr, A.col, A.val, lpr, w, divisor, y, partials, \
                                         vals, ex, flag, guard, b.bits, b.bs_log, win)
#define CB_SS_CASE(F)                                                                                  \
    case F:                                                                                            \
        if (lpr == 0) CB_SS_LAUNCH(F, 0);                                                              \
        else if (!win || lpr < 8) CB_SS_LAUNCH(F, -1);                                                 \
        else if (lpr == 8) CB_SS_LAUNCH(F, 8);                                                         \
        else if (lpr == 16) CB_SS_LAUNCH(F, 16);                                                       \
        else if (lpr == 32) CB_SS_LAUNCH(F, 32);                                                       \
        else CB_SS_LAUNCH(F, 64);                                                                      \
        break;
    switch (kernel_format(fmt)) {
        CB_SS_CASE(CB_F64)
        CB_SS_CASE(CB_F32)
        CB_SS_CASE(CB_F16)
        CB_SS_CASE(CB_FRSZ2_16)
        CB_SS_CASE(CB_FRSZ2_21)
        CB_SS_CASE(CB_FRSZ2_GEN)
        CB_SS_CASE(CB_FRSZ2_GENW)
        CB_SS_CASE(CB_FRSZ2_16_B64)
        CB_SS_CASE(CB_FRSZ2_32_B64)
        default:
        CB_SS_CASE(CB_FRSZ2_32)
    }
#undef CB_SS_CASE
#undef CB_SS_LAUNCH
}

}  // namespace cb
