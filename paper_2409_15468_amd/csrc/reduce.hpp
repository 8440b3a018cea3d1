// Fixed-order reductions inside a wavefront (64 lanes) and a workgroup.
#pragma once

#include <hip/hip_runtime.h>

namespace cb {
namespace dev {

// Load of a control word -- a guard flag, a step count, a divisor, a solver
// scalar -- that an earlier kernel on the stream or another workgroup wrote:
// a device-scope atomic load.  Such words sit at addresses every workgroup
// reads, which the compiler would otherwise load through the scalar cache;
// that cache is not kept coherent with writes of other kernels when kernels
// of other streams run beside this one.
template <class T>
__device__ __forceinline__ T ld_ctl(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, returned in every lane.  Inside each row of 16 lanes
// the butterfly uses DPP moves (swap neighbours, swap pairs, mirror halves of
// 8, mirror the row); the four row sums are then read from lanes 0, 16, 32, 48
// and added as (r0 + r1) + (r2 + r3).  The order is fixed.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// (a, b) -> (a', b') with a' = [a lanes 0-31, b lanes 0-31] and
// b' = [a lanes 32-63, b lanes 32-63] (v_permlane32_swap), per 32-bit half.
__device__ __forceinline__ void swap32(double& a, double& b) {
    auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
    auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
    a = __hiloint2double(hi[0], lo[0]);
    b = __hiloint2double(hi[1], lo[1]);
}
// Odd 16-lane rows of a swapped with even rows of b (v_permlane16_swap).
__device__ __forceinline__ void swap16(double& a, double& b) {
    auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
    auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
    a = __hiloint2double(hi[0], lo[0]);
    b = __hiloint2double(hi[1], lo[1]);
}

// Sum over each aligned group of L lanes (L = 1, 2, 4, ..., 64), returned in
// every lane of the group: the neighbour / pair / half-row-mirror / row-mirror
// DPP butterfly of wave_sum inside 16-lane rows, then 16- and 32-lane swaps
// (a + b after swapping a copy of v with itself leaves the pair's sum in both
// lanes).  All VALU moves; the order is fixed.
template <int L>
__device__ __forceinline__ double group_sum(double v) {
    if constexpr (L >= 2) v += dpp_f64<0xB1>(v);
    if constexpr (L >= 4) v += dpp_f64<0x4E>(v);
    if constexpr (L >= 8) v += dpp_f64<0x141>(v);
    if constexpr (L >= 16) v += dpp_f64<0x140>(v);
    if constexpr (L >= 32) {
        double a = v, b = v;
        swap16(a, b);
        v = a + b;
    }
    if constexpr (L >= 64) {
        double a = v, b = v;
        swap32(a, b);
        v = a + b;
    }
    return v;
}

// Eight wave sums at once (a transposed reduce-scatter): on return lane 8c
// (c = 0..7) holds sum over the 64 lanes of p[c].  Halves of the wave trade
// half their columns (32-lane swap), then rows (16-lane swap), then half-rows
// (DPP rotate by 8 inside a row), and each group of 8 lanes finishes with the
// neighbour / pair / half-row-mirror butterfly.  The order is fixed.
__device__ __forceinline__ double wave_sum8(double* p) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        swap32(p[c], p[c + 4]);
        p[c] += p[c + 4];  // lanes 0-31: column c, lanes 32-63: column c+4
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        swap16(p[c], p[c + 2]);
        p[c] += p[c + 2];  // p[0]: columns 0,2,4,6 by row; p[1]: 1,3,5,7
    }
    const bool upper = (threadIdx.x & 8) != 0;
    const double send = upper ? p[0] : p[1];
    const double keep = upper ? p[1] : p[0];
    double s = keep + dpp_f64<0x128>(send);  // row_ror:8
    s += dpp_f64<0xB1>(s);
    s += dpp_f64<0x4E>(s);
    s += dpp_f64<0x141>(s);
    return s;
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
    __syncthreads();  // part[] may be reused by the next call
    return t;
}

}  // namespace dev
}  // namespace cb
