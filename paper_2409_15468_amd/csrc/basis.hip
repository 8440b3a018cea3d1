// Basis kernels: normalise+encode (store), decode (load), the fused
// decode + classical Gram-Schmidt projection and update, the fused decode +
// solution update, and the fixed-order second reduction stage.
//
// Row partition: workgroup g of the row kernels owns rows
// [2048 g, 2048 (g+1)) -- 64 FRSZ2 blocks -- and thread t of it the 8 rows
// from 2048 g + 8 t.  The partition depends on n only (and, for the fused
// update + projection, on the device's resident capacity), so every reduction
// (per-thread chain, then a fixed shuffle tree, then the 4 waves in order,
// then the workgroups in order) is the same on every run and for every caller.
#include <atomic>

#include "cb_internal.hpp"
#include "codec.hpp"
#include "epilogue.hpp"
#include "reduce.hpp"
#include "tiles.hpp"

namespace cb {

using namespace dev;

// ----------------------------------------------------------------- store (encode)
// Workgroup g, wave w encodes the 512-row tile starting at 2048 g + 512 w.
// The codes go out with non-temporal stores: over launches that encode
// different columns they sustain 2-3% more.  (Of the solver's columns only
// each cycle's first is stored here; the steps' columns are encoded by the
// store + SpMV kernel with ordinary stores, as the next kernel reads them.)
template <int FMT>
__global__ __launch_bounds__(kThreads) void k_store(unsigned char* __restrict__ values,
                                                    uint32_t* __restrict__ exps, int n, int np,
                                                    const double* w, const double* __restrict__ divisor,
                                                    double* v_out, int32_t* __restrict__ flag,
                                                    const int* __restrict__ guard, int bits, int bs_log) {
    if (guard && ld_ctl(guard) == 0) return;
    const int lane = threadIdx.x & 63;
    const int tile0 = blockIdx.x * kRowsPerWG + (threadIdx.x >> 6) * kTile;
    double v[8];
    load_rows<FMT>(w, tile0, lane, n, v);
    if (divisor) {
        const double d = ld_ctl(divisor);
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = v[q] / d;  // IEEE division per entry
    }
    __shared__ double stage[kThreads / 64][kTile];
    if (v_out) store_rows_lds<FMT>(v_out, tile0, lane, n, v, stage[threadIdx.x >> 6]);
    const bool bad = encode_tile<FMT, true>(values, exps, np, tile0, lane, v, bits, bs_log);
    if (flag && bad) atomicOr(flag, 1);
}

// ----------------------------------------------------------------- load (decode)
// Workgroup g, wave w decodes the 512-row tile starting at 2048 g + 512 w:
// one tile per wave and many waves (a loop over several tiles per wave with
// the next tile's loads in flight measured 6% slower: the wave then waits for
// its own stores, where fresh waves do not).  The output goes out with
// non-temporal stores: ordinary stores leave it in the Infinity Cache as dirty
// lines that later launches (or the next kernel's traffic) must write back,
// and measured over launches that decode different columns into different
// vectors they sustain 6% less.
template <int FMT>
__global__ __launch_bounds__(kThreads) void k_load(BasisView V, int col, double* __restrict__ x) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tile0 = blockIdx.x * kRowsPerWG + wave * kTile;
    Tile<FMT> t[1];
    const int cols[1] = {col};
    if (tile0 + kTile <= V.np) load_tiles<FMT, 1, kFull | kStream>(t, V, cols, tile0, lane);
    else load_tiles<FMT, 1, kStream>(t, V, cols, tile0, lane);
    double out[8];
    t[0].decode(out);
    __shared__ double stage[kThreads / 64][kTile];
    store_rows_lds<FMT, true>(x, tile0, lane, V.n, out, stage[wave]);
}

// ----------------------------------------------------------------- CGS projection
// Workgroup (g, y) takes the row groups g, g + G, g + 2G, ... (2048 rows each;
// G <= kProjectGroups keeps the partials few) and the columns
// [y cw, (y+1) cw), and writes partials[c * G + g], its sum of D(v_c) * w:
// per column the waves accumulate over their row groups in order and the waves
// are then added in order.  The last workgroup forms the sums over g
// (epilogue.hpp).  Small n gets several column chunks so that the launch still
// has enough waves to keep HBM busy.
template <int FMT>
__global__ __launch_bounds__(kThreads) void k_project(BasisView V, int j,
                                                      const double* __restrict__ w,
                                                      double* __restrict__ partials, int G, int cw,
                                                      int stream, const int* __restrict__ guard, Epi e) {
    if (guard && ld_ctl(guard) == 0) return;
    __shared__ double red[kThreads / 64][kMaxRestart + 1];
    __shared__ double elds[kEpiLds];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = blockIdx.x;
    const int ngroups = row_groups_dev(V.np);
    const int c0 = blockIdx.y * cw;  // this workgroup's columns [c0, c1)
    const int c1 = min(j, c0 + cw);
    for (int i = lane; i < c1 - c0; i += 64) red[wave][i] = 0.0;
    for (int rg = g; rg < ngroups; rg += G) {
        const int tile0 = rg * kRowsPerWG + wave * kTile;
        double wv[8];
        load_rows<FMT>(w, tile0, lane, V.n, wv);
        const bool full = tile0 + kTile <= V.np;
        if constexpr (FMT == CB_FRSZ2_GENW) {  // 4 column tiles at a time: no spills, same sums
            if (stream) {
                if (full) project_tile_narrow<FMT, kFull | kStream>(V, c0, c1, tile0, lane, wv, red[wave]);
                else project_tile_narrow<FMT, kStream>(V, c0, c1, tile0, lane, wv, red[wave]);
            } else {
                if (full) project_tile_narrow<FMT, kFull>(V, c0, c1, tile0, lane, wv, red[wave]);
                else project_tile_narrow<FMT, 0>(V, c0, c1, tile0, lane, wv, red[wave]);
            }
        } else {
            if (stream) {
                if (full) project_tile<FMT, kFull | kStream>(V, c0, c1, tile0, lane, wv, red[wave]);
                else project_tile<FMT, kStream>(V, c0, c1, tile0, lane, wv, red[wave]);
            } else {
                if (full) project_tile<FMT, kFull>(V, c0, c1, tile0, lane, wv, red[wave]);
                else project_tile<FMT, 0>(V, c0, c1, tile0, lane, wv, red[wave]);
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < c1 - c0; i += kThreads) {
        double s = red[0][i];
#pragma unroll
        for (int k = 1; k < kThreads / 64; ++k) s += red[k][i];
        store_partial(partials + (int64_t)(c0 + i) * G + g, s);
    }
    epilogue(e, partials, elds);
}

// ----------------------------------------------------------------- CGS update / x update
// Start of the update kernels: the guard, the device-side count jdev (if any;
// the host's j then bounds it) and the coefficients h[0 .. j) are loaded
// together -- one memory round trip, not three -- and the coefficients go to
// hc in LDS (the caller synchronises before reading them).  Returns 0 if the
// guard says the launch has nothing to do; j becomes the count to use.
__device__ __forceinline__ int load_coefficients(const int* __restrict__ guard, const int* __restrict__ jdev,
                                                 const double* __restrict__ h, int& j, double* hc) {
    constexpr int HR = (kMaxRestart + 1 + kThreads - 1) / kThreads;
    const int go = guard ? ld_ctl(guard) : 1;
    const int jd = jdev ? ld_ctl(jdev) : j;
    double hv[HR];
#pragma unroll
    for (int k = 0; k < HR; ++k) hv[k] = j > 0 ? ld_ctl(&h[min((int)threadIdx.x + kThreads * k, j - 1)]) : 0.0;
    if (go == 0) return 0;
    j = jd;
#pragma unroll
    for (int k = 0; k < HR; ++k) {
        const int i = (int)threadIdx.x + kThreads * k;
        if (i < j) hc[i] = hv[k];
    }
    return 1;
}

// w[k] += sign * sum_{c<j} h[c] * D(v_c)[k] over the row groups g, g + G, ...
// of workgroup g; partials[g] = sum of w[k]^2 over those rows after the update
// (row groups in order, then the waves in order), if partials != NULL, and
// then the epilogue.
template <int FMT, int U>
__global__ __launch_bounds__(kThreads) void k_subtract(BasisView V, int j, const int* __restrict__ jdev,
                                                       const double* __restrict__ h,
                                                       double* __restrict__ w,
                                                       double* __restrict__ partials, int sign, int stream,
                                                       const int* __restrict__ guard, Epi e) {
    __shared__ double elds[kEpiLds];
    // the coefficients (written by an earlier kernel), read once into LDS
    __shared__ double hc[kMaxRestart + 1];
    __shared__ double stage[kThreads / 64][kTile];
    const int go = load_coefficients(guard, jdev, h, j, hc);
    if (!go) return;
    __syncthreads();
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ngroups = row_groups_dev(V.np);
    double nrm = 0.0;
    for (int rg = blockIdx.x; rg < ngroups; rg += gridDim.x) {
        const int tile0 = rg * kRowsPerWG + wave * kTile;
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        const bool full = tile0 + kTile <= V.np;
        if (stream) {
            if (full) subtract_tile<FMT, U, kFull | kStream>(V, j, hc, tile0, lane, acc);
            else subtract_tile<FMT, U, kStream>(V, j, hc, tile0, lane, acc);
        } else {
            if (full) subtract_tile<FMT, U, kFull>(V, j, hc, tile0, lane, acc);
            else subtract_tile<FMT, U, 0>(V, j, hc, tile0, lane, acc);
        }
        double wv[8];
        load_rows<FMT>(w, tile0, lane, V.n, wv);
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            wv[q] = sign > 0 ? wv[q] + acc[q] : wv[q] - acc[q];
            t = fma(wv[q], wv[q], t);  // rows >= n hold 0
        }
        nrm += t;
        store_rows_lds<FMT>(w, tile0, lane, V.n, wv, stage[wave]);
    }
    if (partials) {
        const double t = block_sum<kThreads>(nrm);
        if (tid == 0) store_partial(partials + blockIdx.x, t);
        epilogue(e, partials, elds);
    }
}

// The first Gram-Schmidt update fused with the second projection (Fig. 1 steps
// 5b-6 and 8): w -= sum_{c<j} h[c] D(v_c) over the workgroup's row groups,
// then u_c = <D(v_c), w> for c < j on the updated rows, which are still in
// registers.  partials[c * G + g] holds the workgroup's u_c for c < j and its
// ||w||^2 at c = j; the epilogue (FUSED_CHECK) keeps u only if step 7 asks for
// the second pass.  Sums are formed in the same orders as k_subtract (norm)
// and k_project with one column chunk (u).
// At most 256 registers (two waves per SIMD): with one, a launch of more
// workgroups than CUs runs in two rounds and pays its start-up twice.
template <int FMT, int U>
__global__ __launch_bounds__(kThreads, 2) void k_subtract_project(BasisView V, int j,
                                                               const double* __restrict__ h,
                                                               double* __restrict__ w,
                                                               double* __restrict__ partials, int stream,
                                                               const int* __restrict__ guard, Epi e) {
    __shared__ double elds[kEpiLds];
    __shared__ double hc[kMaxRestart + 1];
    __shared__ double red[kThreads / 64][kMaxRestart + 2];
    __shared__ double stage[kThreads / 64][kTile];
    const int go = load_coefficients(guard, nullptr, h, j, hc);
    if (!go) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int G = gridDim.x;
    const int ngroups = row_groups_dev(V.np);
    for (int i = lane; i < j; i += 64) red[wave][i] = 0.0;
    __syncthreads();
    double nrm = 0.0;
    for (int rg = blockIdx.x; rg < ngroups; rg += G) {
        const int tile0 = rg * kRowsPerWG + wave * kTile;
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        const bool full = tile0 + kTile <= V.np;
        // ordinary (cache-allocating) loads even for a streaming basis: the
        // projection below re-reads these columns, last first, right away
        if (full) subtract_tile<FMT, U, kFull>(V, j, hc, tile0, lane, acc);
        else subtract_tile<FMT, U, 0>(V, j, hc, tile0, lane, acc);
        double wv[8];
        load_rows<FMT>(w, tile0, lane, V.n, wv);
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            wv[q] = wv[q] - acc[q];
            t = fma(wv[q], wv[q], t);  // rows >= n hold 0
        }
        nrm += t;
        store_rows_lds<FMT>(w, tile0, lane, V.n, wv, stage[wave]);
        if constexpr (FMT == CB_F64) {  // 4 column tiles at a time: fewer registers, same sums
            if (stream) {
                if (full) project_tile_narrow<FMT, kFull | kStream>(V, 0, j, tile0, lane, wv, red[wave]);
                else project_tile_narrow<FMT, kStream>(V, 0, j, tile0, lane, wv, red[wave]);
            } else {
                if (full) project_tile_narrow<FMT, kFull>(V, 0, j, tile0, lane, wv, red[wave]);
                else project_tile_narrow<FMT, 0>(V, 0, j, tile0, lane, wv, red[wave]);
            }
        } else {
            if (stream) {
                if (full) project_tile<FMT, kFull | kStream>(V, 0, j, tile0, lane, wv, red[wave]);
                else project_tile<FMT, kStream>(V, 0, j, tile0, lane, wv, red[wave]);
            } else {
                if (full) project_tile<FMT, kFull>(V, 0, j, tile0, lane, wv, red[wave]);
                else project_tile<FMT, 0>(V, 0, j, tile0, lane, wv, red[wave]);
            }
        }
    }
    const double wn = wave_sum(nrm);
    if (lane == 0) red[wave][j] = wn;
    __syncthreads();
    for (int i = tid; i <= j; i += kThreads) {
        double s = red[0][i];
#pragma unroll
        for (int k = 1; k < kThreads / 64; ++k) s += red[k][i];
        store_partial(partials + (int64_t)i * G + blockIdx.x, s);
    }
    epilogue(e, partials, elds);
}

// ----------------------------------------------------------------- stage 2
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ partials, int G,
                                                double* __restrict__ out, int op,
                                                const int* __restrict__ guard) {
    if (guard && ld_ctl(guard) == 0) return;
    const int c = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < G; i += 256) s += partials[(int64_t)c * G + i];
    s = block_sum<256>(s);
    if (threadIdx.x == 0) out[c] = op ? ld_ctl(&out[c]) + s : s;
}

__global__ void k_fill(double* __restrict__ x, double v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// ----------------------------------------------------------------- launchers
#define CB_DISPATCH(fmt, KERNEL_CALL)                      \
    switch (kernel_format(fmt)) {                          \
    case CB_F64: { constexpr int F = CB_F64; KERNEL_CALL; break; }           \
    case CB_F32: { constexpr int F = CB_F32; KERNEL_CALL; break; }           \
    case CB_F16: { constexpr int F = CB_F16; KERNEL_CALL; break; }           \
    case CB_FRSZ2_16: { constexpr int F = CB_FRSZ2_16; KERNEL_CALL; break; } \
    case CB_FRSZ2_21: { constexpr int F = CB_FRSZ2_21; KERNEL_CALL; break; } \
    case CB_FRSZ2_GEN: { constexpr int F = CB_FRSZ2_GEN; KERNEL_CALL; break; } \
    case CB_FRSZ2_GENW: { constexpr int F = CB_FRSZ2_GENW; KERNEL_CALL; break; } \
    case CB_FRSZ2_16_B64: { constexpr int F = CB_FRSZ2_16_B64; KERNEL_CALL; break; } \
    case CB_FRSZ2_32_B64: { constexpr int F = CB_FRSZ2_32_B64; KERNEL_CALL; break; } \
    default: { constexpr int F = CB_FRSZ2_32; KERNEL_CALL; break; }          \
    }

__global__ void k_zero(unsigned* __restrict__ c, int words) {
    for (int i = threadIdx.x; i < words; i += blockDim.x) c[i] = 0u;
}

// Non-temporal basis loads pay off once the columns one pass reads no longer
// fit in the 256 MB Infinity Cache next to the rest of the working set; below
// that, the solver's four passes per step over the same columns hit in it.
constexpr int kResidentWaves = 2048;

static int streams_basis(const BasisView& b, int j) {
    constexpr int64_t kCacheResident = (int64_t)192 << 20;
    return (int64_t)j * (b.col_bytes + 4 * b.exp_stride) > kCacheResident;
}

void launch_zero_counter(unsigned* counter, hipStream_t s) {
    k_zero<<<1, 256, 0, s>>>(counter, kCounterBytes / 4);
}

void launch_store(int fmt, const cb_basis& V, int col, const double* w, const double* divisor,
                  double* v_out, int32_t* flag, const int* guard, hipStream_t s) {
    BasisView b = view_of(V);
    unsigned char* vals = static_cast<unsigned char*>(V.values) + (int64_t)col * b.col_bytes;
    uint32_t* ex = V.exps ? V.exps + (int64_t)col * b.exp_stride : nullptr;
    dim3 grid((unsigned)row_groups(V.n));
    CB_DISPATCH(fmt, (k_store<F><<<grid, kThreads, 0, s>>>(vals, ex, b.n, b.np, w, divisor, v_out,
                                                           flag, guard, b.bits, b.bs_log)));
}

void launch_load(int fmt, const cb_basis& V, int col, double* x, hipStream_t s) {
    BasisView b = view_of(V);
    dim3 grid((unsigned)row_groups(V.n));
    CB_DISPATCH(fmt, (k_load<F><<<grid, kThreads, 0, s>>>(b, col, x)));
}

void launch_project(int fmt, const cb_basis& V, int j, const double* w, double* partials,
                    const int* guard, const Epi& e, hipStream_t s) {
    BasisView b = view_of(V);
    const int G = dot_groups(V.n);
    // Column chunks (multiples of 8 columns) only while the launch has fewer
    // waves than the GPU keeps resident (~2048 at this kernel's register
    // use): every workgroup pays a fixed tail (its partial stores and ticket),
    // so workgroups are made as long as the resident waves allow.
    int chunks = kResidentWaves / (4 * G);
    chunks = chunks < 1 ? 1 : chunks;
    int max_chunks = (j + 15) / 16;
    const int ngroups = (G + kTicketGroup - 1) / kTicketGroup;  // ticket groups per chunk
    if (max_chunks > kMaxTicketGroups / ngroups) max_chunks = kMaxTicketGroups / ngroups;
    chunks = chunks > max_chunks ? max_chunks : chunks;
    chunks = chunks < 1 ? 1 : chunks;
    int cw = (j + chunks - 1) / chunks;
    cw = (cw + 7) / 8 * 8;
    chunks = (j + cw - 1) / cw;
    dim3 grid((unsigned)G, (unsigned)chunks);
    Epi ee = e;
    ee.G = G;
    ee.ncols = j;
    ee.cw = cw;
    const int stream = streams_basis(b, j);
    CB_DISPATCH(fmt, (k_project<F><<<grid, kThreads, 0, s>>>(b, j, w, partials, G, cw, stream, guard, ee)));
}

void launch_subtract(int fmt, const cb_basis& V, int j, const int* jdev, const double* h,
                     double* w, double* partials, const int* guard, int sign, const Epi& e,
                     hipStream_t s) {
    BasisView b = view_of(V);
    const int G = project_groups(V.n);
    dim3 grid((unsigned)G);
    Epi ee = e;
    ee.G = G;
    ee.ncols = 1;
    ee.cw = 1;
    // with the count on the device, size the policy for the largest count j
    const int stream = streams_basis(b, j);
    CB_DISPATCH(fmt, (k_subtract<F, 4><<<grid, kThreads, 0, s>>>(b, j, jdev, h, w, partials, sign, stream,
                                                                guard, ee)));
}

// Workgroups of `kernel` the current device holds at once (its occupancy per
// CU times the CU count), cached per device and kernel format; 0 if the
// runtime cannot say.
static int resident_groups(const void* kernel, int fmt) {
    constexpr int kDevs = 16, kFmts = 16;
    static std::atomic<int> cache[kDevs][kFmts];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevs || fmt < 0 || fmt >= kFmts) return 0;
    int r = cache[dev][fmt].load(std::memory_order_relaxed);
    if (r > 0) return r;
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess)
        return 0;
    r = cus * per_cu;
    if (r > 0) cache[dev][fmt].store(r, std::memory_order_relaxed);
    return r;
}

void launch_subtract_project(int fmt, const cb_basis& V, int j, const double* h, double* w, double* partials,
                             const int* guard, const Epi& e, hipStream_t s) {
    BasisView b = view_of(V);
    int G = project_groups(V.n);
    // Whole waves of resident workgroups: at three per CU (the 16-bit
    // formats), 1024 workgroups would run as 768 and then a lone 256 (measured
    // 0.8% of an n = 2^22 inner solve); 768 that loop over the row groups do not.
    CB_DISPATCH(fmt, ({
        const int R = resident_groups(reinterpret_cast<const void*>(&k_subtract_project<F, 4>), F);
        if (R > 0 && G > R) G = G / R * R;
    }));
    dim3 grid((unsigned)G);
    Epi ee = e;
    ee.G = G;
    ee.ncols = j + 1;  // u_0 .. u_{j-1} and the norm
    ee.cw = j + 1;
    const int stream = streams_basis(b, j);
    CB_DISPATCH(fmt, (k_subtract_project<F, 4><<<grid, kThreads, 0, s>>>(b, j, h, w, partials, stream, guard, ee)));
}

void launch_reduce(const double* partials, int G, int ncols, double* out, int op, const int* guard,
                   hipStream_t s) {
    if (ncols <= 0) return;
    k_reduce<<<ncols, 256, 0, s>>>(partials, G, out, op, guard);
}

void launch_fill(double* x, double v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, v, n);
}

}  // namespace cb
