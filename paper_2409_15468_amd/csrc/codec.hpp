// Device-side storage codecs for basis columns: FRSZ2 (specialised for l = 16,
// 21, 32; any l in [3, 32] through the generic tile) and the float64 / float32
// / float16 baselines.
//
// Access pattern.  A wavefront works on a tile of 512 consecutive rows of a
// column; lane t owns 8 of them.  The lane-to-row map is chosen per format so
// that every 16-byte load instruction of the wave reads one contiguous 1 KB
// run of the column (lane t at byte 16 t of the run): float64 lanes own rows
// {128k + 2t, +1}, k < 4; float32 and frsz2_32 lanes own {256k + 4t .. +3},
// k < 2; float16, frsz2_16 and frsz2_21 lanes own 8t .. 8t+7.  Each such group
// of rows lies inside one 32-value FRSZ2 block.  frsz2_21 codes straddle words:
// a lane loads the 6 words that hold its 8 codes.  Basis loads are
// non-temporal when the columns a pass reads exceed what the Infinity Cache can
// keep between passes (the solver re-reads them up to four times per step),
// ordinary otherwise.
//
// FRSZ2 values are never materialised with their scale: a code becomes the
// exact signed integer +-M (a 32-bit convert and a sign-bit insert), products
// are accumulated, and the block scale 2^(max(E,1)-1023-(l-2)) of Eq. 2 is
// applied once per block piece with ldexp.  Scaling by a power of two is
// exact, so this equals decoding first up to the order of the sums.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cb_internal.hpp"

namespace cb {
namespace dev {

constexpr int kTile = 512;  // rows of a column per wavefront

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// 16-byte load; NT: non-temporal (streaming, does not displace cached data)
template <bool NT>
__device__ __forceinline__ uint4 ld16(const void* p) {
    if constexpr (NT) {
        u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
        return make_uint4(v.x, v.y, v.z, v.w);
    } else {
        return *reinterpret_cast<const uint4*>(p);
    }
}
template <bool NT>
__device__ __forceinline__ uint32_t ld4(const uint32_t* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
// Load mode of a tile: bit 0 the tile lies wholly inside the column (no row
// checks), bit 1 non-temporal loads.
constexpr int kFull = 1, kStream = 2;
__device__ __forceinline__ uint32_t word_of(const uint4& a, int i) {
    return i == 0 ? a.x : i == 1 ? a.y : i == 2 ? a.z : a.w;
}
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

// ----------------------------------------------------------------- lane-to-row maps
template <int FMT>
struct Map {
    // rows of lane t: 8 values in NG groups of GS consecutive rows, group k
    // starting at k * GSTRIDE + GS * t (relative to the tile)
    static constexpr int GS = FMT == CB_F64 ? 2 : (FMT == CB_F32 || FMT == CB_FRSZ2_32 || FMT == CB_FRSZ2_32_B64) ? 4 : 8;
    static constexpr int NG = 8 / GS;
    static constexpr int GSTRIDE = 64 * GS;
    __device__ static int row(int t, int q) { return (q / GS) * GSTRIDE + GS * t + (q % GS); }
    __device__ static int group_row(int t, int k) { return k * GSTRIDE + GS * t; }
};

// w (float64) at the lane's 8 rows; rows >= n read as 0.
template <int FMT>
__device__ __forceinline__ void load_rows(const double* __restrict__ w, int tile0, int lane, int n,
                                          double* wv) {
    using M = Map<FMT>;
#pragma unroll
    for (int k = 0; k < M::NG; ++k) {
        const int r = tile0 + M::group_row(lane, k);
        if (r + M::GS <= n) {
#pragma unroll
            for (int p = 0; p < M::GS; p += 2) {
                double2 t = *reinterpret_cast<const double2*>(w + r + p);
                wv[k * M::GS + p] = t.x;
                wv[k * M::GS + p + 1] = t.y;
            }
        } else {
#pragma unroll
            for (int p = 0; p < M::GS; ++p) wv[k * M::GS + p] = (r + p < n) ? w[r + p] : 0.0;
        }
    }
}

// NT: non-temporal 16-byte stores, for outputs that no later kernel of the
// same pass reads back soon (they do not fill the caches with dirty lines).
template <int FMT, bool NT = false>
__device__ __forceinline__ void store_rows(double* __restrict__ w, int tile0, int lane, int n,
                                           const double* wv) {
    using M = Map<FMT>;
    typedef double d2v __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int k = 0; k < M::NG; ++k) {
        const int r = tile0 + M::group_row(lane, k);
        if (r + M::GS <= n) {
#pragma unroll
            for (int p = 0; p < M::GS; p += 2) {
                if constexpr (NT) {
                    const d2v v = {wv[k * M::GS + p], wv[k * M::GS + p + 1]};
                    __builtin_nontemporal_store(v, reinterpret_cast<d2v*>(w + r + p));
                } else {
                    *reinterpret_cast<double2*>(w + r + p) = make_double2(wv[k * M::GS + p], wv[k * M::GS + p + 1]);
                }
            }
        } else {
#pragma unroll
            for (int p = 0; p < M::GS; ++p)
                if (r + p < n) w[r + p] = wv[k * M::GS + p];
        }
    }
}

// store_rows through the wave's LDS scratch `lds` (kTile doubles): the lane's
// values go to LDS at their tile row and come back in the float64 map, so
// that every 16-byte store instruction of the wave writes one contiguous 1 KB
// run of w (lane t at byte 16 t).  With the 4- and 8-row maps a direct store
// instruction scatters 16-byte pieces 32 or 64 bytes apart over 2 or 4 KB,
// which costs the memory pipeline 2-4 times as many cache-line visits per
// byte stored.  Whole waves call it; only this wave touches `lds`.
template <int FMT, bool NT = false>
__device__ __forceinline__ void store_rows_lds(double* __restrict__ w, int tile0, int lane, int n,
                                               const double* wv, double* lds) {
    using M = Map<FMT>;
    if constexpr (M::GS == 2) {
        store_rows<FMT, NT>(w, tile0, lane, n, wv);
    } else {
#pragma unroll
        for (int k = 0; k < M::NG; ++k) {
#pragma unroll
            for (int p = 0; p < M::GS; p += 2)
                *reinterpret_cast<double2*>(lds + M::group_row(lane, k) + p) =
                    make_double2(wv[k * M::GS + p], wv[k * M::GS + p + 1]);
        }
        __builtin_amdgcn_wave_barrier();
        using F = Map<CB_F64>;
        double out[8];
#pragma unroll
        for (int k = 0; k < F::NG; ++k) {
            const double2 t = *reinterpret_cast<const double2*>(lds + F::group_row(lane, k));
            out[2 * k] = t.x;
            out[2 * k + 1] = t.y;
        }
        __builtin_amdgcn_wave_barrier();
        store_rows<CB_F64, NT>(w, tile0, lane, n, out);
    }
}

// ----------------------------------------------------------------- reading tiles
// Tile<FMT>: one column's data for the lane's 8 rows.
//   load(V, col, tile0, lane)       issue the loads
//   dot(w)                          sum_q D(v)[q] * w[q]
//   axpy(h, acc)                    acc[q] += h * D(v)[q]
//   decode(out)                     out[q] = D(v)[q]
// Groups of rows past the padded length np are not loaded and read as 0.
template <int FMT>
struct Tile;

template <int FMT>
struct FloatTile {
    using M = Map<FMT>;
    uint4 x[M::NG];
    template <int LM>
    __device__ __forceinline__ void load(const BasisView& V, int col, int tile0, int lane) {
        const unsigned char* base = V.values + (int64_t)col * V.col_bytes;
        constexpr int esz = FMT == CB_F64 ? 8 : FMT == CB_F32 ? 4 : 2;
#pragma unroll
        for (int k = 0; k < M::NG; ++k) {
            const int r = tile0 + M::group_row(lane, k);
            x[k] = ((LM & kFull) || r < V.np) ? ld16<(LM & kStream) != 0>(base + (int64_t)r * esz)
                                              : make_uint4(0, 0, 0, 0);
        }
    }
    __device__ __forceinline__ double v(int q) const {
        const uint4& a = x[q / M::GS];
        const int i = q % M::GS;
        if constexpr (FMT == CB_F64) {
            return i == 0 ? make_double(a.y, a.x) : make_double(a.w, a.z);
        } else if constexpr (FMT == CB_F32) {
            return (double)__uint_as_float(word_of(a, i));
        } else {
            uint32_t wd = word_of(a, i >> 1);
            return half_to_double((i & 1) ? (wd >> 16) : (wd & 0xFFFFu));
        }
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
template <> struct Tile<CB_F64> : FloatTile<CB_F64> {};
template <> struct Tile<CB_F32> : FloatTile<CB_F32> {};
template <> struct Tile<CB_F16> : FloatTile<CB_F16> {};

__device__ __forceinline__ int scale_exp(uint32_t E, int L) { return (E ? (int)E : 1) - 1023 - (L - 2); }

// frsz2_32 with blocks of 2^LOGBS values: code q is word q of the block, so
// row r's code is word r of the column whatever the block size.
template <int LOGBS>
struct Frsz2Tile32 {
    using M = Map<CB_FRSZ2_32>;
    uint4 x[2];
    uint32_t e[2];
    template <int LM>
    __device__ __forceinline__ void load(const BasisView& V, int col, int tile0, int lane) {
        const unsigned char* base = V.values + (int64_t)col * V.col_bytes;
        const uint32_t* ex = V.exps + (int64_t)col * V.exp_stride;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int r = tile0 + M::group_row(lane, k);
            const bool live = (LM & kFull) || r < V.np;
            x[k] = live ? ld16<(LM & kStream) != 0>(base + (int64_t)r * 4) : make_uint4(0, 0, 0, 0);
            e[k] = live ? ex[r >> LOGBS] : 0u;
        }
    }
    __device__ __forceinline__ double m(int q) const {
        uint32_t c = word_of(x[q >> 2], q & 3);
        return signed_mag(c & 0x7FFFFFFFu, c);
    }
    __device__ __forceinline__ double dot(const double* w) const {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) t = fma(m(4 * k + i), w[4 * k + i], t);
            s += ldexp(t, scale_exp(e[k], 32));
        }
        return s;
    }
    __device__ __forceinline__ void axpy(double h, double* acc) const {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const double hs = ldexp(h, scale_exp(e[k], 32));
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[4 * k + i] = fma(hs, m(4 * k + i), acc[4 * k + i]);
        }
    }
    __device__ __forceinline__ void decode(double* out) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) out[q] = ldexp(m(q), scale_exp(e[q >> 2], 32));
    }
};
template <> struct Tile<CB_FRSZ2_32> : Frsz2Tile32<5> {};
template <> struct Tile<CB_FRSZ2_32_B64> : Frsz2Tile32<6> {};

// frsz2_16 with blocks of 2^LOGBS values: row r's code is half-word r.
template <int LOGBS>
struct Frsz2Tile16 {
    using M = Map<CB_FRSZ2_16>;
    uint4 x;
    uint32_t e;
    template <int LM>
    __device__ __forceinline__ void load(const BasisView& V, int col, int tile0, int lane) {
        const unsigned char* base = V.values + (int64_t)col * V.col_bytes;
        const int r = tile0 + M::group_row(lane, 0);
        const bool live = (LM & kFull) || r < V.np;
        x = live ? ld16<(LM & kStream) != 0>(base + (int64_t)r * 2) : make_uint4(0, 0, 0, 0);
        e = live ? V.exps[(int64_t)col * V.exp_stride + (r >> LOGBS)] : 0u;
    }
    __device__ __forceinline__ double m(int q) const {
        uint32_t wd = word_of(x, q >> 1);
        if (q & 1) return signed_mag((wd >> 16) & 0x7FFFu, wd);
        return signed_mag(wd & 0x7FFFu, wd << 16);
    }
    __device__ __forceinline__ double dot(const double* w) const {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) s = fma(m(q), w[q], s);
        return ldexp(s, scale_exp(e, 16));
    }
    __device__ __forceinline__ void axpy(double h, double* acc) const {
        const double hs = ldexp(h, scale_exp(e, 16));
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = fma(hs, m(q), acc[q]);
    }
    __device__ __forceinline__ void decode(double* out) const {
        const int se = scale_exp(e, 16);
#pragma unroll
        for (int q = 0; q < 8; ++q) out[q] = ldexp(m(q), se);
    }
};
template <> struct Tile<CB_FRSZ2_16> : Frsz2Tile16<5> {};
template <> struct Tile<CB_FRSZ2_16_B64> : Frsz2Tile16<6> {};

// frsz2_21.  The lane's 8 values 8t .. 8t+7 are codes 8s .. 8s+7 (s = t % 4)
// of block t / 4 of the tile; they start at bit 168 s = 32 (5 s) + 8 s of the
// block, so the lane needs the block's words 5s .. 5s+5 and shifts the 6-word
// window right by 8 s bits; code q then sits at bit 21 q of the window.  The
// tile's codes are 1344 contiguous bytes (16-byte aligned): the wave loads them
// as 84 pieces of 16 bytes (lane t: pieces t and 64 + t), two load
// instructions instead of six word loads per lane, and hands them to the lanes
// that need them through a per-wave slot of LDS when the codes are used.
// Whole waves call dot, axpy and decode.
__shared__ uint32_t xch21[8][336];  // one 1344-byte tile per wave, 8 waves at most

template <>
struct Tile<CB_FRSZ2_21> {
    uint4 a, b;  // pieces lane and 64 + lane of the tile (b: lanes < 20)
    uint32_t e;
    bool live;
    template <int LM>
    __device__ __forceinline__ void load(const BasisView& V, int col, int tile0, int lane) {
        const unsigned char* base = V.values + (int64_t)col * V.col_bytes + (int64_t)(tile0 >> 5) * 84;
        // bytes of whole blocks below np (a piece that straddles their end
        // stays inside the column's 256-byte-rounded storage)
        const int vbytes = (LM & kFull) ? 1344 : min(max((V.np - tile0) >> 5, 0), 16) * 84;
        a = 16 * lane < vbytes ? ld16<(LM & kStream) != 0>(base + 16 * lane) : make_uint4(0, 0, 0, 0);
        b = (lane < 20 && 1024 + 16 * lane < vbytes) ? ld16<(LM & kStream) != 0>(base + 1024 + 16 * lane)
                                                      : make_uint4(0, 0, 0, 0);
        const int r = tile0 + 8 * lane;
        live = (LM & kFull) || r < V.np;
        e = live ? V.exps[(int64_t)col * V.exp_stride + (r >> 5)] : 0u;
    }
    __device__ __forceinline__ void codes(uint32_t* c) const {
        const int lane = threadIdx.x & 63;
        uint32_t* x = xch21[threadIdx.x >> 6];
        __builtin_amdgcn_wave_barrier();  // the slot's previous tile has been read
        *reinterpret_cast<uint4*>(x + 4 * lane) = a;
        if (lane < 20) *reinterpret_cast<uint4*>(x + 256 + 4 * lane) = b;
        __builtin_amdgcn_wave_barrier();
        const uint32_t* p = x + (lane >> 2) * 21 + 5 * (lane & 3);
        uint32_t y[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) y[k] = live ? p[k] : 0u;
        const uint32_t s = 8u * (lane & 3);
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
    __device__ __forceinline__ double dot(const double* w) const {
        uint32_t c[8];
        codes(c);
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) sum = fma(m_of(c[q]), w[q], sum);
        return ldexp(sum, scale_exp(e, 21));
    }
    __device__ __forceinline__ void axpy(double h, double* acc) const {
        uint32_t c[8];
        codes(c);
        const double hs = ldexp(h, scale_exp(e, 21));
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = fma(hs, m_of(c[q]), acc[q]);
    }
    __device__ __forceinline__ void decode(double* out) const {
        uint32_t c[8];
        codes(c);
        const int se = scale_exp(e, 21);
#pragma unroll
        for (int q = 0; q < 8; ++q) out[q] = ldexp(m_of(c[q]), se);
    }
};

// Any l in [3, 32] (the generic formats), blocks of 32 or 64 values.  Lane t
// owns rows 8t .. 8t+7, i.e. codes 8s .. 8s+7 (s = t mod P, P = 4 or 8 lanes
// per block) of block t / P, which start at bit 8 s l of the block's words:
// word 8 s l / 32, bit 8 s l % 32 of it.  The lane loads the (at most 9) words
// that hold its 8 codes -- as words, or for wide codes as up to three aligned
// 16-byte pieces -- and walks them with a two-word window that advances by one word whenever the bit
// position passes 32; the window shifts use fixed register indices, so
// nothing spills.
template <bool WIDE>
struct GenTile {
    uint32_t y[9];
    uint32_t e;
    uint32_t off;  // bit of the lane's first code in y[0]
    int L;
    template <int LM>
    __device__ __forceinline__ void load(const BasisView& V, int col, int tile0, int lane) {
        L = V.bits;
        const int lb = V.bs_log;
        const uint32_t* base = reinterpret_cast<const uint32_t*>(V.values + (int64_t)col * V.col_bytes);
        const int r = tile0 + 8 * lane;
        const bool live = (LM & kFull) || r < V.np;
        const uint32_t start = 8u * (uint32_t)(lane & ((1 << (lb - 3)) - 1)) * (uint32_t)L;
        off = start & 31u;
        // the codes end at bit start + 8 l - 1 <= 2^lb l - 1: inside the block
        const int nw = (int)((off + 8u * (uint32_t)L + 31u) >> 5);
        const int64_t w0 = (int64_t)(r >> lb) * (L << (lb - 5)) + (start >> 5);  // first word in the column
        // Up to three 16-byte loads from the aligned word at or below w0, when
        // the last of them ends inside the column's data (np l / 32 words);
        // otherwise (the column's last lanes) word loads.
        const int sh = (int)(w0 & 3);
        const int nq = (sh + nw + 3) >> 2;
        const bool wide = WIDE && (w0 - sh) + 4 * nq <= (((int64_t)V.np * L) >> 5);
        if (WIDE && live && wide) {
            const uint4* q = reinterpret_cast<const uint4*>(base + (w0 - sh));
            uint32_t z[12];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const uint4 a = k < nq ? ld16<(LM & kStream) != 0>(q + k) : make_uint4(0, 0, 0, 0);
                z[4 * k] = a.x;
                z[4 * k + 1] = a.y;
                z[4 * k + 2] = a.z;
                z[4 * k + 3] = a.w;
            }
            // drop the sh words below w0: shifts by 2 and 1 with fixed indices,
            // written as masks so that they stay register moves
            const uint32_t m2 = (sh & 2) ? 0xFFFFFFFFu : 0u, m1 = (sh & 1) ? 0xFFFFFFFFu : 0u;
#pragma unroll
            for (int i = 0; i < 10; ++i) z[i] = (z[i] & ~m2) | (z[i + 2] & m2);
#pragma unroll
            for (int i = 0; i < 9; ++i) z[i] = (z[i] & ~m1) | (z[i + 1] & m1);
#pragma unroll
            for (int k = 0; k < 9; ++k) y[k] = z[k];
        } else {
            const uint32_t* p = base + w0;
#pragma unroll
            for (int k = 0; k < 9; ++k) y[k] = (live && k < nw) ? ld4<(LM & kStream) != 0>(p + k) : 0u;
        }
        e = live ? V.exps[(int64_t)col * V.exp_stride + (r >> lb)] : 0u;
    }
    __device__ __forceinline__ void codes(uint32_t* c) const {
        uint32_t w[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) w[k] = y[k];
        const uint32_t mask = L == 32 ? 0xFFFFFFFFu : ((1u << L) - 1u);
        uint32_t pos = off;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            c[q] = __builtin_amdgcn_alignbit(w[1], w[0], pos) & mask;
            if (q < 7) {
                pos += (uint32_t)L;
                const bool adv = pos >= 32u;
                // codes q+1 .. 7 need at most words 0 .. 7-q of the window
#pragma unroll
                for (int k = 0; k < 8 - q; ++k) w[k] = adv ? w[k + 1] : w[k];
                pos = adv ? pos - 32u : pos;
            }
        }
    }
    __device__ __forceinline__ double m_of(uint32_t c) const {
        return signed_mag(c & ((1u << (L - 1)) - 1u), c << (32 - L));
    }
    __device__ __forceinline__ double dot(const double* w) const {
        uint32_t c[8];
        codes(c);
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) sum = fma(m_of(c[q]), w[q], sum);
        return ldexp(sum, scale_exp(e, L));
    }
    __device__ __forceinline__ void axpy(double h, double* acc) const {
        uint32_t c[8];
        codes(c);
        const double hs = ldexp(h, scale_exp(e, L));
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = fma(hs, m_of(c[q]), acc[q]);
    }
    __device__ __forceinline__ void decode(double* out) const {
        uint32_t c[8];
        codes(c);
        const int se = scale_exp(e, L);
#pragma unroll
        for (int q = 0; q < 8; ++q) out[q] = ldexp(m_of(c[q]), se);
    }
};
template <> struct Tile<CB_FRSZ2_GEN> : GenTile<false> {};
template <> struct Tile<CB_FRSZ2_GENW> : GenTile<true> {};

// Load U columns of a tile (load mode M).
template <int FMT, int U, int LM>
__device__ __forceinline__ void load_tiles(Tile<FMT>* t, const BasisView& V, const int* cols, int tile0,
                                           int lane) {
#pragma unroll
    for (int u = 0; u < U; ++u) t[u].template load<LM>(V, cols[u], tile0, lane);
}

// ----------------------------------------------------------------- writing tiles
// FRSZ2 code of v with block exponent field E (Section IV-A steps 2-5).
template <int L>
__device__ __forceinline__ uint32_t frsz2_code(double v, uint32_t E) {
    const uint32_t hi = hi32(v), lo = lo32(v);
    const uint32_t e = (hi >> 20) & 0x7FFu;
    const uint32_t Eeff = E ? E : 1u;
    const uint32_t eeff = e ? e : 1u;
    // step 2: significand with the leading one made explicit (53 bits)
    const uint64_t sig = ((uint64_t)((hi & 0xFFFFFu) | (e ? 0x100000u : 0u)) << 32) | lo;
    // steps 3 and 5: align to E (shift right by k = E - e) and keep l-1 bits
    const uint32_t drop = (uint32_t)(54 - L) + (Eeff - eeff);
    const uint32_t M = drop >= 53u ? 0u : (uint32_t)(sig >> drop);
    // step 4: the sign to the left of the significand
    return ((hi >> 31) << (L - 1)) | M;
}

// The same code with l known only at run time (the generic formats).
__device__ __forceinline__ uint32_t frsz2_code_rt(double v, uint32_t E, int L) {
    const uint32_t hi = hi32(v), lo = lo32(v);
    const uint32_t e = (hi >> 20) & 0x7FFu;
    const uint32_t Eeff = E ? E : 1u;
    const uint32_t eeff = e ? e : 1u;
    const uint64_t sig = ((uint64_t)((hi & 0xFFFFFu) | (e ? 0x100000u : 0u)) << 32) | lo;
    const uint32_t drop = (uint32_t)(54 - L) + (Eeff - eeff);
    const uint32_t M = drop >= 53u ? 0u : (uint32_t)(sig >> drop);
    return ((hi >> 31) << (L - 1)) | M;
}

__device__ __forceinline__ uint32_t exp_field(double v) { return (hi32(v) >> 20) & 0x7FFu; }

// max over lane groups of 2^LOG lanes (LOG <= 4) with DPP moves inside rows
// (quad swaps, then the half-row and row mirrors)
template <int LOG>
__device__ __forceinline__ uint32_t group_max(uint32_t x) {
    if constexpr (LOG >= 1) x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false));
    if constexpr (LOG >= 2) x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false));
    if constexpr (LOG >= 3) x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false));
    if constexpr (LOG >= 4) x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false));
    return x;
}

}  // namespace dev
}  // namespace cb
