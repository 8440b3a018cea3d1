// Arithmetic-intensity sweep kernel (the synthetic benchmark of Section IV-C,
// Fig. 3): read one basis column through its format's decoder -- the same
// tile loads and in-register decode as the Gram-Schmidt kernels -- and apply a
// chosen number of dependent FP64 multiply-adds to each value, so that the
// arithmetic per byte read can be swept from memory-bound to compute-bound.
//
// Workgroup g owns the 2048-row groups g, g + G, ...; wave w the 512-row tile
// w of each; every lane decodes its 8 values and runs 8 independent chains
// y <- y * a + b of `ops` steps, then adds the results of its rows below n.
// One partial sum per workgroup keeps the work observable.
#include "cb_internal.hpp"
#include "codec.hpp"
#include "reduce.hpp"
#include "tiles.hpp"

namespace cb {

using namespace dev;

template <int FMT>
__global__ __launch_bounds__(kThreads) void k_intensity(BasisView V, int col, int ops, double a, double b,
                                                        double* __restrict__ partials) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ngroups = row_groups_dev(V.np);
    double acc = 0.0;
    for (int rg = blockIdx.x; rg < ngroups; rg += gridDim.x) {
        const int tile0 = rg * kRowsPerWG + wave * kTile;
        Tile<FMT> t[1];
        const int cols[1] = {col};
        if (tile0 + kTile <= V.np) load_tiles<FMT, 1, kFull | kStream>(t, V, cols, tile0, lane);
        else load_tiles<FMT, 1, kStream>(t, V, cols, tile0, lane);
        double y[8];
        t[0].decode(y);
        for (int i = 0; i < ops; ++i) {
#pragma unroll
            for (int q = 0; q < 8; ++q) y[q] = fma(y[q], a, b);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (tile0 + Map<FMT>::row(lane, q) < V.n) acc += y[q];  // rows past n are padding
    }
    const double s = block_sum<kThreads>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

}  // namespace cb

using namespace cb;

extern "C" {

int32_t cb_intensity_groups(int64_t n) {
    if (n < 1 || n > kMaxRows) return -1;
    return project_groups(n);
}

int cb_intensity_run(const cb_basis* V, int32_t col, int32_t ops, double a, double b, double* partials,
                     void* stream) {
    if (!V || !V->values || !partials || !valid_format(V->format) || V->n < 1 || V->n > kMaxRows || col < 0 || col >= V->ncols ||
        ops < 0 || (frsz2_bits_of(V->format) && !V->exps) || !aligned(V->values, 16) || !aligned(V->exps, 4) ||
        !aligned(partials, 8))
        return fail(CB_ERR_INVALID_ARG, "bad intensity-sweep arguments");
    hipStream_t s = (hipStream_t)stream;
    const BasisView bv = view_of(*V);
    const int G = project_groups(V->n);
    switch (kernel_format(V->format)) {
    case CB_F64: k_intensity<CB_F64><<<G, kThreads, 0, s>>>(bv, col, ops, a, b, partials); break;
    case CB_F32: k_intensity<CB_F32><<<G, kThreads, 0, s>>>(bv, col, ops, a, b, partials); break;
    case CB_F16: k_intensity<CB_F16><<<G, kThreads, 0, s>>>(bv, col, ops, a, b, partials); break;
    case CB_FRSZ2_16: k_intensity<CB_FRSZ2_16><<<G, kThreads, 0, s>>>(bv, col, ops, a, b, partials); break;
    case CB_FRSZ2_21: k_intensity<CB_FRSZ2_21><<<G, kThreads, 0, s>>>(bv, col, ops, a, b, partials); break;
    case CB_FRSZ2_GEN: k_intensity<CB_FRSZ2_GEN><<<G, kThreads, 0, s>>>(bv, col, ops, a, b, partials); break;
    case CB_FRSZ2_GENW: k_intensity<CB_FRSZ2_GENW><<<G, kThreads, 0, s>>>(bv, col, ops, a, b, partials); break;
    case CB_FRSZ2_16_B64: k_intensity<CB_FRSZ2_16_B64><<<G, kThreads, 0, s>>>(bv, col, ops, a, b, partials); break;
    case CB_FRSZ2_32_B64: k_intensity<CB_FRSZ2_32_B64><<<G, kThreads, 0, s>>>(bv, col, ops, a, b, partials); break;
    default: k_intensity<CB_FRSZ2_32><<<G, kThreads, 0, s>>>(bv, col, ops, a, b, partials); break;
    }
    CB_HIP(hipGetLastError());
    return CB_OK;
}

}  // extern "C"
