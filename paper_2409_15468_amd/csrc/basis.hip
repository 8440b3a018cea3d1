// Basis kernels: normalise+encode (store), decode (load), the fused
// decode + classical Gram-Schmidt projection and update, the fused decode +
// solution update, and the fixed-order second reduction stage.
//
// Row partition: workgroup g of the row kernels owns rows
// [2048 g, 2048 (g+1)) -- 64 FRSZ2 blocks -- and thread t of it the 8 rows
// from 2048 g + 8 t.  The partition depends on n only, so every reduction
// (per-thread chain, then a fixed shuffle tree, then the 4 waves in order,
// then the workgroups in order) is the same on every run and for every caller.
#include "cb_internal.hpp"
#include "codec.hpp"
#include "reduce.hpp"

namespace cb {

using namespace dev;

// ----------------------------------------------------------------- store (encode)
template <int FMT>
__global__ __launch_bounds__(kThreads) void k_store(unsigned char* __restrict__ values,
                                                    uint32_t* __restrict__ exps, int n, int np,
                                                    const double* w, const double* __restrict__ divisor,
                                                    double* v_out, int32_t* __restrict__ flag,
                                                    const int* __restrict__ guard) {
    if (guard && *guard == 0) return;
    const int row = blockIdx.x * kThreads + threadIdx.x;
    if (row >= np) return;  // whole 32-lane groups leave together (np % 32 == 0)
    double v = 0.0;
    if (row < n) {
        v = w[row];
        if (divisor) v = v / *divisor;  // IEEE division per entry
        if (v_out) v_out[row] = v;
    }
    if constexpr (FMT == CB_F64) {
        reinterpret_cast<double*>(values)[row] = v;
        if (flag && !isfinite(v)) atomicOr(flag, 1);
    } else if constexpr (FMT == CB_F32) {
        float f = (float)v;
        reinterpret_cast<float*>(values)[row] = f;
        if (flag && !isfinite(f)) atomicOr(flag, 1);
    } else if constexpr (FMT == CB_F16) {
        uint32_t h = double_to_half_rne(v);
        reinterpret_cast<uint16_t*>(values)[row] = (uint16_t)h;
        if (flag && (h & 0x7C00u) == 0x7C00u) atomicOr(flag, 1);
    } else {
        constexpr int L = FMT == CB_FRSZ2_16 ? 16 : FMT == CB_FRSZ2_21 ? 21 : 32;
        const int lane = threadIdx.x & 31;
        const int blk = row >> 5;
        uint32_t E;
        const uint32_t c = frsz2_encode_lane<L>(v, &E);
        if (lane == 0) {
            exps[blk] = E;
            if (flag && E == 0x7FFu) atomicOr(flag, 1);
        }
        if constexpr (L == 32) {
            reinterpret_cast<uint32_t*>(values)[row] = c;
        } else if constexpr (L == 16) {
            reinterpret_cast<uint16_t*>(values)[row] = (uint16_t)c;
        } else {
            // word k of the block holds stream bits [32k, 32k+32): pieces of the
            // codes q0 = floor(32k/21), q0+1 and q0+2
            const int q0 = (32 * lane) / 21;
            const uint32_t c0 = (uint32_t)__shfl((int)c, q0, 32);
            const uint32_t c1 = (uint32_t)__shfl((int)c, min(q0 + 1, 31), 32);
            const uint32_t c2 = (uint32_t)__shfl((int)c, min(q0 + 2, 31), 32);
            const uint64_t stream = (uint64_t)c0 | ((uint64_t)(q0 + 1 < 32 ? c1 : 0u) << 21) |
                                    ((uint64_t)(q0 + 2 < 32 ? c2 : 0u) << 42);
            if (lane < 21)
                reinterpret_cast<uint32_t*>(values)[blk * 21 + lane] =
                    (uint32_t)(stream >> (32 * lane - 21 * q0));
        }
    }
}

// ----------------------------------------------------------------- load (decode)
template <int FMT>
__global__ __launch_bounds__(kThreads) void k_load(BasisView V, int col, double* __restrict__ x) {
    const int row0 = blockIdx.x * kRowsPerWG + threadIdx.x * kSeg;
    if (row0 >= V.np) return;
    Seg<FMT> s;
    seg_load(s, V, col, row0);
    double out[kSeg];
    s.decode(out);
    if (row0 + kSeg <= V.n) {
        double2* p = reinterpret_cast<double2*>(x + row0);
#pragma unroll
        for (int k = 0; k < 4; ++k) p[k] = make_double2(out[2 * k], out[2 * k + 1]);
    } else {
#pragma unroll
        for (int q = 0; q < kSeg; ++q)
            if (row0 + q < V.n) x[row0 + q] = out[q];
    }
}

__device__ __forceinline__ void load_w(const double* __restrict__ w, int row0, int n, double* wv) {
    if (row0 + kSeg <= n) {
        const double2* p = reinterpret_cast<const double2*>(w + row0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double2 t = p[k];
            wv[2 * k] = t.x;
            wv[2 * k + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < kSeg; ++q) wv[q] = (row0 + q < n) ? w[row0 + q] : 0.0;
    }
}

// ----------------------------------------------------------------- CGS projection
// partials[c * G + g] = sum over the workgroup's rows of D(v_c) * w, c < j.
template <int FMT, int U>
__global__ __launch_bounds__(kThreads) void k_project(BasisView V, int j,
                                                      const double* __restrict__ w,
                                                      double* __restrict__ partials, int G,
                                                      const int* __restrict__ guard) {
    if (guard && *guard == 0) return;
    __shared__ double red[kThreads / 64][kColChunk];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = blockIdx.x;
    const int c0 = blockIdx.y * kColChunk;
    const int c1 = min(j, c0 + kColChunk);
    int row0 = g * kRowsPerWG + tid * kSeg;
    const bool live = row0 < V.np;
    if (!live) row0 = 0;  // keep loads in bounds; the lane contributes 0
    double wv[kSeg];
    load_w(w, live ? row0 : V.n, V.n, wv);
    for (int c = c0; c < c1; c += U) {
        Seg<FMT> s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) seg_load(s[u], V, min(c + u, c1 - 1), row0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double p = (live && c + u < c1) ? s[u].dot(wv) : 0.0;
            p = wave_sum(p);
            if (lane == 0 && c + u < c1) red[wave][c + u - c0] = p;
        }
    }
    __syncthreads();
    for (int i = tid; i < c1 - c0; i += kThreads) {
        double t = red[0][i];
#pragma unroll
        for (int k = 1; k < kThreads / 64; ++k) t += red[k][i];
        partials[(int64_t)(c0 + i) * G + g] = t;
    }
}

// ----------------------------------------------------------------- CGS update / x update
// w[k] += sign * sum_{c<j} h[c] * D(v_c)[k]; partials[g] = sum of w[k]^2 over
// the workgroup's rows after the update (if partials != NULL).
template <int FMT, int U>
__global__ __launch_bounds__(kThreads) void k_subtract(BasisView V, int j, const int* __restrict__ jdev,
                                                       const double* __restrict__ h,
                                                       double* __restrict__ w,
                                                       double* __restrict__ partials, int sign,
                                                       const int* __restrict__ guard) {
    if (guard && *guard == 0) return;
    if (jdev) j = *jdev;
    const int tid = threadIdx.x;
    int row0 = blockIdx.x * kRowsPerWG + tid * kSeg;
    const bool live = row0 < V.np;
    if (!live) row0 = 0;
    double acc[kSeg];
#pragma unroll
    for (int q = 0; q < kSeg; ++q) acc[q] = 0.0;
    for (int c = 0; c < j; c += U) {
        Seg<FMT> s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) seg_load(s[u], V, min(c + u, j - 1), row0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double hc = (c + u < j) ? h[c + u] : 0.0;
            if (c + u < j) s[u].axpy(hc, acc);
        }
    }
    double nrm = 0.0;
    if (live) {
        double wv[kSeg];
        load_w(w, row0, V.n, wv);
#pragma unroll
        for (int q = 0; q < kSeg; ++q) {
            wv[q] = sign > 0 ? wv[q] + acc[q] : wv[q] - acc[q];
            if (row0 + q < V.n) nrm = fma(wv[q], wv[q], nrm);
        }
        if (row0 + kSeg <= V.n) {
            double2* p = reinterpret_cast<double2*>(w + row0);
#pragma unroll
            for (int k = 0; k < 4; ++k) p[k] = make_double2(wv[2 * k], wv[2 * k + 1]);
        } else {
#pragma unroll
            for (int q = 0; q < kSeg; ++q)
                if (row0 + q < V.n) w[row0 + q] = wv[q];
        }
    }
    if (partials) {
        double t = block_sum<kThreads>(nrm);
        if (tid == 0) partials[blockIdx.x] = t;
    }
}

// ----------------------------------------------------------------- stage 2
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ partials, int G,
                                                double* __restrict__ out, int op,
                                                const int* __restrict__ guard) {
    if (guard && *guard == 0) return;
    const int c = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < G; i += 256) s += partials[(int64_t)c * G + i];
    s = block_sum<256>(s);
    if (threadIdx.x == 0) out[c] = op ? out[c] + s : s;
}

__global__ void k_fill(double* __restrict__ x, double v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// ----------------------------------------------------------------- launchers
#define CB_DISPATCH(fmt, KERNEL_CALL)                      \
    switch (fmt) {                                         \
    case CB_F64: { constexpr int F = CB_F64; KERNEL_CALL; break; }           \
    case CB_F32: { constexpr int F = CB_F32; KERNEL_CALL; break; }           \
    case CB_F16: { constexpr int F = CB_F16; KERNEL_CALL; break; }           \
    case CB_FRSZ2_16: { constexpr int F = CB_FRSZ2_16; KERNEL_CALL; break; } \
    case CB_FRSZ2_21: { constexpr int F = CB_FRSZ2_21; KERNEL_CALL; break; } \
    default: { constexpr int F = CB_FRSZ2_32; KERNEL_CALL; break; }          \
    }

template <int F>
constexpr int unroll_of() {
    return F == CB_F64 ? 4 : 8;
}

void launch_store(int fmt, const cb_basis& V, int col, const double* w, const double* divisor,
                  double* v_out, int32_t* flag, const int* guard, hipStream_t s) {
    BasisView b = view_of(V);
    unsigned char* vals = static_cast<unsigned char*>(V.values) + (int64_t)col * b.col_bytes;
    uint32_t* ex = V.exps ? V.exps + (int64_t)col * b.exp_stride : nullptr;
    dim3 grid((unsigned)((b.np + kThreads - 1) / kThreads));
    CB_DISPATCH(fmt, (k_store<F><<<grid, kThreads, 0, s>>>(vals, ex, b.n, b.np, w, divisor, v_out,
                                                           flag, guard)));
}

void launch_load(int fmt, const cb_basis& V, int col, double* x, hipStream_t s) {
    BasisView b = view_of(V);
    dim3 grid((unsigned)row_groups(V.n));
    CB_DISPATCH(fmt, (k_load<F><<<grid, kThreads, 0, s>>>(b, col, x)));
}

void launch_project(int fmt, const cb_basis& V, int j, const double* w, double* partials,
                    const int* guard, hipStream_t s) {
    BasisView b = view_of(V);
    const int G = row_groups(V.n);
    dim3 grid((unsigned)G, (unsigned)((j + kColChunk - 1) / kColChunk));
    CB_DISPATCH(fmt, (k_project<F, unroll_of<F>()><<<grid, kThreads, 0, s>>>(b, j, w, partials, G,
                                                                              guard)));
}

void launch_subtract(int fmt, const cb_basis& V, int j, const int* jdev, const double* h,
                     double* w, double* partials, const int* guard, int sign, hipStream_t s) {
    BasisView b = view_of(V);
    dim3 grid((unsigned)row_groups(V.n));
    CB_DISPATCH(fmt, (k_subtract<F, unroll_of<F>()><<<grid, kThreads, 0, s>>>(b, j, jdev, h, w, partials,
                                                                               sign, guard)));
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
