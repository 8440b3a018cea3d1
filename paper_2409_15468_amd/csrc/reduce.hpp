// Fixed-order reductions inside a wavefront (64 lanes) and a workgroup.
#pragma once

#include <hip/hip_runtime.h>

namespace cb {
namespace dev {

// Butterfly sum over the 64 lanes; every lane ends with the same total and the
// order of the additions is fixed.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over a workgroup of NT threads (NT a multiple of 64); the result is
// valid in thread 0.  Waves are combined in index order.
template <int NT>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double part[NT / 64];
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) part[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        t = part[0];
#pragma unroll
        for (int k = 1; k < NT / 64; ++k) t += part[k];
    }
    return t;
}

}  // namespace dev
}  // namespace cb
