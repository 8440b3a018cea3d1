// Device-side storage codecs for one basis column: FRSZ2 (l = 16, 21, 32) and
// the float64/float32/float16 baselines.
//
// Reading side: a thread owns a segment of 8 consecutive rows (row0 % 8 == 0),
// issues the loads for a column in `load`, and consumes them in `dot` (sum of
// decoded value times w), `axpy` (acc += h * decoded value) or `decode`.
// FRSZ2 values are never materialised with their scale: each code becomes the
// exact signed integer +-M (a 32-bit convert plus a sign-bit insert), the
// segment's products are accumulated, and the block scale 2^(E_eff-1023-(l-2))
// is applied once per segment with ldexp.  Scaling by a power of two is exact,
// so this equals decoding first (Eq. 2) up to the order of the sums.
//
// Writing side: a 32-lane group holds one FRSZ2 block (Section III-A): the
// block's largest exponent is found with lane shuffles across the group, then
// each lane aligns its significand to it, truncates to l-1 bits, prepends the
// sign and the group packs the codes LSB-first into l words.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cb_internal.hpp"

namespace cb {
namespace dev {

__device__ __forceinline__ uint32_t lo32(double x) { return (uint32_t)__double2loint(x); }
__device__ __forceinline__ uint32_t hi32(double x) { return (uint32_t)__double2hiint(x); }
__device__ __forceinline__ double make_double(uint32_t hi, uint32_t lo) {
    return __hiloint2double((int)hi, (int)lo);
}

// (-1)^s * M as a double, exact for M < 2^32; the sign is bit 31 of `sbits`.
__device__ __forceinline__ double signed_mag(uint32_t M, uint32_t sbits) {
    double d = (double)M;
    return make_double(hi32(d) | (sbits & 0x80000000u), lo32(d));
}

__device__ __forceinline__ double half_to_double(uint32_t h16) {
    _Float16 hv = __builtin_bit_cast(_Float16, (unsigned short)h16);
    return (double)(float)hv;
}

// float64 -> binary16, one rounding to nearest-even, by integer operations on
// the IEEE fields.  Overflow gives +-Inf, NaN stays NaN.
__device__ __forceinline__ uint32_t double_to_half_rne(double x) {
    uint32_t hi = hi32(x), lo = lo32(x);
    uint32_t sign = (hi >> 16) & 0x8000u;
    int e = (int)((hi >> 20) & 0x7FF);
    uint64_t f = ((uint64_t)(hi & 0xFFFFFu) << 32) | lo;
    if (e == 0x7FF) return sign | 0x7C00u | (f ? 0x200u : 0u);
    int E = e - 1023;
    if (E > 15) return sign | 0x7C00u;
    if (E >= -14) {
        uint32_t mant = (uint32_t)(f >> 42);
        uint64_t rem = f & ((UINT64_C(1) << 42) - 1);
        uint32_t h = ((uint32_t)(E + 15) << 10) | mant;
        const uint64_t half = UINT64_C(1) << 41;
        if (rem > half || (rem == half && (mant & 1u))) h += 1;  // carries into the exponent
        return sign | h;
    }
    if (e == 0) return sign;  // float64 subnormals are far below the binary16 range
    int sh = 28 - E;          // value in units of 2^-24 is sig53 >> sh
    if (sh > 53) return sign;
    uint64_t sig = (UINT64_C(1) << 52) | f;
    uint32_t q = (uint32_t)(sig >> sh);
    uint64_t rem = sig & ((UINT64_C(1) << sh) - 1);
    uint64_t half = UINT64_C(1) << (sh - 1);
    if (rem > half || (rem == half && (q & 1u))) q += 1;
    return sign | q;
}

// ----------------------------------------------------------------- reading segments
template <int FMT>
struct Seg;

template <>
struct Seg<CB_F64> {
    double2 x[4];
    __device__ __forceinline__ void load(const BasisView& V, int col, int row0) {
        const double2* p = reinterpret_cast<const double2*>(V.values + (int64_t)col * V.col_bytes) + (row0 >> 1);
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = p[k];
    }
    __device__ __forceinline__ double v(int q) const { return (q & 1) ? x[q >> 1].y : x[q >> 1].x; }
    __device__ __forceinline__ double dot(const double* w) const {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) s = fma(v(q), w[q], s);
        return s;
    }
    __device__ __forceinline__ void axpy(double h, double* acc) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = fma(h, v(q), acc[q]);
    }
    __device__ __forceinline__ void decode(double* out) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) out[q] = v(q);
    }
};

template <>
struct Seg<CB_F32> {
    float4 x[2];
    __device__ __forceinline__ void load(const BasisView& V, int col, int row0) {
        const float4* p = reinterpret_cast<const float4*>(V.values + (int64_t)col * V.col_bytes) + (row0 >> 2);
        x[0] = p[0];
        x[1] = p[1];
    }
    __device__ __forceinline__ double v(int q) const {
        const float4& a = x[q >> 2];
        float f = (q & 3) == 0 ? a.x : (q & 3) == 1 ? a.y : (q & 3) == 2 ? a.z : a.w;
        return (double)f;
    }
    __device__ __forceinline__ double dot(const double* w) const {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) s = fma(v(q), w[q], s);
        return s;
    }
    __device__ __forceinline__ void axpy(double h, double* acc) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = fma(h, v(q), acc[q]);
    }
    __device__ __forceinline__ void decode(double* out) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) out[q] = v(q);
    }
};

template <>
struct Seg<CB_F16> {
    uint4 x;
    __device__ __forceinline__ void load(const BasisView& V, int col, int row0) {
        x = *(reinterpret_cast<const uint4*>(V.values + (int64_t)col * V.col_bytes) + (row0 >> 3));
    }
    __device__ __forceinline__ double v(int q) const {
        uint32_t wd = (q >> 1) == 0 ? x.x : (q >> 1) == 1 ? x.y : (q >> 1) == 2 ? x.z : x.w;
        return half_to_double((q & 1) ? (wd >> 16) : (wd & 0xFFFFu));
    }
    __device__ __forceinline__ double dot(const double* w) const {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) s = fma(v(q), w[q], s);
        return s;
    }
    __device__ __forceinline__ void axpy(double h, double* acc) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = fma(h, v(q), acc[q]);
    }
    __device__ __forceinline__ void decode(double* out) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) out[q] = v(q);
    }
};

// Common part of the FRSZ2 segments: block exponent and the code magnitudes
// as exact signed doubles.
template <int L>
struct FrszBase {
    uint32_t e;  // stored block exponent field E
    __device__ __forceinline__ int scale_exp() const {
        int Eeff = e ? (int)e : 1;
        return Eeff - 1023 - (L - 2);
    }
};

template <>
struct Seg<CB_FRSZ2_32> : FrszBase<32> {
    uint4 x[2];
    __device__ __forceinline__ void load(const BasisView& V, int col, int row0) {
        const uint4* p = reinterpret_cast<const uint4*>(V.values + (int64_t)col * V.col_bytes) + (row0 >> 2);
        x[0] = p[0];
        x[1] = p[1];
        e = V.exps[(int64_t)col * V.exp_stride + (row0 >> 5)];
    }
    __device__ __forceinline__ uint32_t code(int q) const {
        const uint4& a = x[q >> 2];
        return (q & 3) == 0 ? a.x : (q & 3) == 1 ? a.y : (q & 3) == 2 ? a.z : a.w;
    }
    __device__ __forceinline__ double m(int q) const {
        uint32_t c = code(q);
        return signed_mag(c & 0x7FFFFFFFu, c);
    }
    __device__ __forceinline__ double dot(const double* w) const {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) s = fma(m(q), w[q], s);
        return ldexp(s, scale_exp());
    }
    __device__ __forceinline__ void axpy(double h, double* acc) const {
        double hs = ldexp(h, scale_exp());
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = fma(hs, m(q), acc[q]);
    }
    __device__ __forceinline__ void decode(double* out) const {
        int se = scale_exp();
#pragma unroll
        for (int q = 0; q < 8; ++q) out[q] = ldexp(m(q), se);
    }
};

template <>
struct Seg<CB_FRSZ2_16> : FrszBase<16> {
    uint4 x;
    __device__ __forceinline__ void load(const BasisView& V, int col, int row0) {
        x = *(reinterpret_cast<const uint4*>(V.values + (int64_t)col * V.col_bytes) + (row0 >> 3));
        e = V.exps[(int64_t)col * V.exp_stride + (row0 >> 5)];
    }
    __device__ __forceinline__ double m(int q) const {
        uint32_t wd = (q >> 1) == 0 ? x.x : (q >> 1) == 1 ? x.y : (q >> 1) == 2 ? x.z : x.w;
        if (q & 1) return signed_mag((wd >> 16) & 0x7FFFu, wd);
        return signed_mag(wd & 0x7FFFu, wd << 16);
    }
    __device__ __forceinline__ double dot(const double* w) const {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) s = fma(m(q), w[q], s);
        return ldexp(s, scale_exp());
    }
    __device__ __forceinline__ void axpy(double h, double* acc) const {
        double hs = ldexp(h, scale_exp());
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = fma(hs, m(q), acc[q]);
    }
    __device__ __forceinline__ void decode(double* out) const {
        int se = scale_exp();
#pragma unroll
        for (int q = 0; q < 8; ++q) out[q] = ldexp(m(q), se);
    }
};

// l = 21: a block's 32 codes span 21 words.  The segment of 8 values that
// starts at value 8t (t = 0..3) begins at bit 168t = 32*(5t) + 8t, so the thread
// loads the 6 words from 5t and funnel-shifts the window right by 8t bits; the
// codes then sit at the fixed bit offsets 21q of the shifted 168-bit window.
template <>
struct Seg<CB_FRSZ2_21> : FrszBase<21> {
    uint32_t y[6];
    __device__ __forceinline__ void load(const BasisView& V, int col, int row0) {
        const uint32_t* base = reinterpret_cast<const uint32_t*>(V.values + (int64_t)col * V.col_bytes);
        const int t = (row0 >> 3) & 3;
        const uint32_t* p = base + (row0 >> 5) * 21 + 5 * t;
#pragma unroll
        for (int k = 0; k < 6; ++k) y[k] = p[k];
        e = V.exps[(int64_t)col * V.exp_stride + (row0 >> 5)];
    }
    __device__ __forceinline__ void codes(int row0, uint32_t* c) const {
        const uint32_t s = (uint32_t)(8 * ((row0 >> 3) & 3));
        uint32_t z[6];
#pragma unroll
        for (int k = 0; k < 5; ++k) z[k] = __builtin_amdgcn_alignbit(y[k + 1], y[k], s);
        z[5] = y[5] >> s;
        c[0] = z[0];
        c[1] = __builtin_amdgcn_alignbit(z[1], z[0], 21);
        c[2] = z[1] >> 10;
        c[3] = __builtin_amdgcn_alignbit(z[2], z[1], 31);
        c[4] = __builtin_amdgcn_alignbit(z[3], z[2], 20);
        c[5] = z[3] >> 9;
        c[6] = __builtin_amdgcn_alignbit(z[4], z[3], 30);
        c[7] = __builtin_amdgcn_alignbit(z[5], z[4], 19);
    }
    __device__ __forceinline__ static double m_of(uint32_t c) { return signed_mag(c & 0xFFFFFu, c << 11); }
    int row0_;
    __device__ __forceinline__ void set_row(int row0) { row0_ = row0; }
    __device__ __forceinline__ double dot(const double* w) const {
        uint32_t c[8];
        codes(row0_, c);
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) s = fma(m_of(c[q]), w[q], s);
        return ldexp(s, scale_exp());
    }
    __device__ __forceinline__ void axpy(double h, double* acc) const {
        uint32_t c[8];
        codes(row0_, c);
        double hs = ldexp(h, scale_exp());
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = fma(hs, m_of(c[q]), acc[q]);
    }
    __device__ __forceinline__ void decode(double* out) const {
        uint32_t c[8];
        codes(row0_, c);
        int se = scale_exp();
#pragma unroll
        for (int q = 0; q < 8; ++q) out[q] = ldexp(m_of(c[q]), se);
    }
};

// Uniform entry: load a column segment (all formats).
template <int FMT>
__device__ __forceinline__ void seg_load(Seg<FMT>& s, const BasisView& V, int col, int row0) {
    s.load(V, col, row0);
    if constexpr (FMT == CB_FRSZ2_21) s.set_row(row0);
}

// ----------------------------------------------------------------- writing blocks
// FRSZ2 code of value v inside its 32-lane group (all 32 lanes participate).
// Returns the code; *E receives the block's stored exponent field.
template <int L>
__device__ __forceinline__ uint32_t frsz2_encode_lane(double v, uint32_t* Eout) {
    uint32_t hi = hi32(v), lo = lo32(v);
    uint32_t s = hi >> 31;
    uint32_t e = (hi >> 20) & 0x7FFu;
    // step 1: block maximum of the exponent fields over the 32-lane group
    uint32_t E = e;
#pragma unroll
    for (int off = 16; off >= 1; off >>= 1) E = max(E, (uint32_t)__shfl_xor((int)E, off, 32));
    *Eout = E;
    uint32_t Eeff = E ? E : 1u;
    uint32_t eeff = e ? e : 1u;
    // step 2: significand with the leading one made explicit (53 bits)
    uint64_t sig = ((uint64_t)((hi & 0xFFFFFu) | (e ? 0x100000u : 0u)) << 32) | lo;
    // steps 3 and 5: align to E (shift by k = E - e) and keep l-1 bits
    uint32_t drop = (uint32_t)(54 - L) + (Eeff - eeff);
    uint32_t M = drop >= 53u ? 0u : (uint32_t)(sig >> drop);
    // step 4: sign to the left of the significand
    return (s << (L - 1)) | M;
}

}  // namespace dev
}  // namespace cb
