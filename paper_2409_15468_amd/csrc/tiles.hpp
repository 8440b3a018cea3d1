// Per-wavefront tile operations on basis columns shared by the multi-workgroup
// kernels and the one-workgroup batched solver: encode a tile of 512 rows into
// a column, the fused decode + projection over a range of columns, and the
// fused decode + multi-axpy.  Whole wavefronts call them (block maxima and
// reductions use cross-lane moves).
#pragma once

#include "cb_internal.hpp"
#include "codec.hpp"
#include "reduce.hpp"

namespace cb {
namespace dev {

// 16-byte stores of encoded data; NT: non-temporal, for a column that no
// kernel of the same pass reads back soon.  (The 4-byte stores of frsz2_21,
// the generic widths and the exponents stay ordinary: non-temporal, the
// partial lines they write cost frsz2_21's encoding 10%.)
template <bool NT>
__device__ __forceinline__ void put16(unsigned char* p, uint4 o) {
    if constexpr (NT) {
        typedef unsigned u4v __attribute__((ext_vector_type(4)));
        const u4v x = {o.x, o.y, o.z, o.w};
        __builtin_nontemporal_store(x, reinterpret_cast<u4v*>(p));
    } else {
        *reinterpret_cast<uint4*>(p) = o;
    }
}

// Encode the lane's 8 values v (rows of Map<FMT>) of the tile at row tile0
// into one column: values at `values`, FRSZ2 block exponents at `exps`
// (Section IV-A for frsz2; round-to-nearest-even casts for float32 and
// float16; float64 stored as is).  Groups of rows at or past np are not
// written.  Returns true if a stored value is not finite (for frsz2: a block
// whose exponent field is 2047).
// bits, bs_log: l and log2 of the block size of the generic FRSZ2 formats
// (ignored by the others).  NT: the 16-byte value stores are non-temporal.
template <int FMT, bool NT = false>
__device__ __forceinline__ bool encode_tile(unsigned char* __restrict__ values, uint32_t* __restrict__ exps,
                                            int np, int tile0, int lane, const double* v, int bits = 0,
                                            int bs_log = 5) {
    using M = Map<FMT>;
    bool bad = false;
    if constexpr (FMT == CB_F64 || FMT == CB_F32 || FMT == CB_F16) {
#pragma unroll
        for (int k = 0; k < M::NG; ++k) {
            const int r = tile0 + M::group_row(lane, k);
            uint4 o;
            if constexpr (FMT == CB_F64) {
                const double a = v[2 * k], b = v[2 * k + 1];
                o = make_uint4(lo32(a), hi32(a), lo32(b), hi32(b));
                bad |= !isfinite(a) || !isfinite(b);
            } else if constexpr (FMT == CB_F32) {
                float f[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    f[i] = (float)v[4 * k + i];
                    bad |= !isfinite(f[i]);
                }
                o = make_uint4(__float_as_uint(f[0]), __float_as_uint(f[1]), __float_as_uint(f[2]),
                               __float_as_uint(f[3]));
            } else {
                uint32_t h[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    h[i] = double_to_half_rne(v[i]);
                    bad |= (h[i] & 0x7C00u) == 0x7C00u;
                }
                o = make_uint4(h[0] | h[1] << 16, h[2] | h[3] << 16, h[4] | h[5] << 16, h[6] | h[7] << 16);
            }
            constexpr int esz = FMT == CB_F64 ? 8 : FMT == CB_F32 ? 4 : 2;
            if (r < np) put16<NT>(values + (int64_t)r * esz, o);
        }
    } else if constexpr (FMT == CB_FRSZ2_32 || FMT == CB_FRSZ2_32_B64) {
        // groups of 4 values; the 8 lanes 8u..8u+7 hold one block of 32 (the
        // 16 lanes 16u..16u+15 one block of 64)
        constexpr int LB = FMT == CB_FRSZ2_32 ? 5 : 6;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int r = tile0 + M::group_row(lane, k);
            uint32_t E = max(max(exp_field(v[4 * k]), exp_field(v[4 * k + 1])),
                             max(exp_field(v[4 * k + 2]), exp_field(v[4 * k + 3])));
            E = group_max<LB - 2>(E);  // step 1: block maximum
            uint4 o = make_uint4(frsz2_code<32>(v[4 * k], E), frsz2_code<32>(v[4 * k + 1], E),
                                 frsz2_code<32>(v[4 * k + 2], E), frsz2_code<32>(v[4 * k + 3], E));
            if (r < np) {
                put16<NT>(values + (int64_t)r * 4, o);
                if ((lane & ((1 << (LB - 2)) - 1)) == 0) exps[r >> LB] = E;
            }
            bad |= E == 0x7FFu;
        }
    } else {
        // 8 values per lane; the 4 lanes 4u..4u+3 hold one block of 32 (the
        // 8 lanes 8u..8u+7 one block of 64)
        const int lb = is_generic<FMT> ? bs_log : FMT == CB_FRSZ2_16_B64 ? 6 : 5;
        const int r = tile0 + 8 * lane;
        uint32_t E = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) E = max(E, exp_field(v[q]));
        E = group_max<2>(E);
        if (lb == 6) E = max(E, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)E, 0x141, 0xF, 0xF, false));
        const bool first = (lane & ((1 << (lb - 3)) - 1)) == 0;  // the block's first lane
        bad = E == 0x7FFu;
        if constexpr (is_generic<FMT>) {
            // The lane's 8 codes go to bits 8 s l .. 8 s l + 8 l - 1 of its
            // block (s = lane % 4), streamed word by word through a 64-bit
            // accumulator.  A word the lane shares with the previous lane of
            // the block (its first, when it starts mid-word) is handed to that
            // lane, which merges it into its own last word; the block's last
            // lane always ends on a word boundary.
            const int L = bits;
            uint32_t c[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = frsz2_code_rt(v[q], E, L);
            const uint32_t start = 8u * (uint32_t)(lane & ((1 << (lb - 3)) - 1)) * (uint32_t)L;
            const uint32_t off = start & 31u;
            uint32_t* blk = reinterpret_cast<uint32_t*>(values) + (int64_t)(r >> lb) * (L << (lb - 5)) + (start >> 5);
            const bool live = r < np;
            uint64_t acc = 0;
            uint32_t nb = off, head = 0;
            int wi = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                acc |= (uint64_t)c[q] << nb;
                nb += (uint32_t)L;
                if (nb >= 32u) {
                    const uint32_t wd = (uint32_t)acc;
                    if (wi == 0 && off != 0u) head = wd;
                    else if (live) blk[wi] = wd;
                    ++wi;
                    acc >>= 32;
                    nb -= 32u;
                }
            }
            // the next lane's first word (row shift by one lane: crosses quads)
            const uint32_t next_head = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)head, 0x101, 0xF, 0xF, false);
            if (live) {
                if (nb > 0u) blk[wi] = (uint32_t)acc | next_head;
                if (first) exps[r >> lb] = E;
            }
        } else if constexpr (FMT == CB_FRSZ2_16 || FMT == CB_FRSZ2_16_B64) {
            uint32_t c[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = frsz2_code<16>(v[q], E);
            if (r < np) {
                put16<NT>(values + (int64_t)r * 2,
                          make_uint4(c[0] | c[1] << 16, c[2] | c[3] << 16, c[4] | c[5] << 16, c[6] | c[7] << 16));
                if (first) exps[r >> lb] = E;
            }
        } else {
            uint32_t c[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = frsz2_code<21>(v[q], E);
            // the 8 codes as a 168-bit stream, code q at bit 21 q
            uint32_t S[6];
            S[0] = c[0] | c[1] << 21;
            S[1] = c[1] >> 11 | c[2] << 10 | c[3] << 31;
            S[2] = c[3] >> 1 | c[4] << 20;
            S[3] = c[4] >> 12 | c[5] << 9 | c[6] << 30;
            S[4] = c[6] >> 2 | c[7] << 19;
            S[5] = c[7] >> 13;
            // placed at bit 8 s of block word 5 s (s = lane % 4): W[k] is word 5 s + k
            const uint32_t sh = 8u * (lane & 3);
            uint32_t W[6];
            W[0] = S[0] << sh;
#pragma unroll
            for (int k = 1; k < 6; ++k) W[k] = sh ? ((S[k] << sh) | (S[k - 1] >> (32u - sh))) : S[k];
            // word 5 s + 5 is shared with the next lane of the block
            const uint32_t next0 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)W[0], 0xF9, 0xF, 0xF, false);
            if ((lane & 3) != 3) W[5] |= next0;
            if (r < np) {
                uint32_t* blk = reinterpret_cast<uint32_t*>(values) + (int64_t)(r >> 5) * 21 + 5 * (lane & 3);
                if ((lane & 3) == 0) {
                    blk[0] = W[0];
                    exps[r >> 5] = E;
                }
#pragma unroll
                for (int k = 1; k < 6; ++k) blk[k] = W[k];
            }
        }
    }
    return bad;
}

// One wave's columns [c0, c1) of its tile, 8 at a time, the last 8 first; the
// wave's sums for column c are added to red[c - c0].  The loads of the next 8
// columns are issued before the current 8 are reduced across the wave.  The
// passes of a step alternate direction -- projections run down the columns,
// updates up -- so that each pass starts on the columns the previous pass read
// last, which the caches still hold.  Each column's sum does not depend on the
// order in which columns are visited.
template <int FMT, int LM>
__device__ __forceinline__ void project_tile(const BasisView& V, int c0, int c1, int tile0, int lane,
                                             const double* wv, double* red) {
    const int last = c0 + ((c1 - c0 - 1) / 8) * 8;  // first column of the last group of 8
    Tile<FMT> t[8];
    int cols[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) cols[u] = min(last + u, c1 - 1);
    load_tiles<FMT, 8, LM>(t, V, cols, tile0, lane);
    for (int c = last; c >= c0; c -= 8) {
        double p[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) p[u] = t[u].dot(wv);
        if (c - 8 >= c0) {
#pragma unroll
            for (int u = 0; u < 8; ++u) cols[u] = c - 8 + u;
            load_tiles<FMT, 8, LM>(t, V, cols, tile0, lane);
        }
        const double sum = wave_sum8(p);  // lane 8u holds column c + u
        if ((lane & 7) == 0 && c + (lane >> 3) < c1) red[c + (lane >> 3) - c0] += sum;
    }
}

// The same sums as project_tile (identical bits) with 4 column tiles in
// registers at a time instead of 8, for kernels with a smaller register budget.
template <int FMT, int LM>
__device__ __forceinline__ void project_tile_narrow(const BasisView& V, int c0, int c1, int tile0, int lane,
                                                    const double* wv, double* red) {
    for (int c = c0 + ((c1 - c0 - 1) / 8) * 8; c >= c0; c -= 8) {
        double p[8];
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            Tile<FMT> t[4];
            int cols[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) cols[u] = min(c + 4 * half + u, c1 - 1);
            load_tiles<FMT, 4, LM>(t, V, cols, tile0, lane);
#pragma unroll
            for (int u = 0; u < 4; ++u) p[4 * half + u] = t[u].dot(wv);
        }
        const double sum = wave_sum8(p);
        if ((lane & 7) == 0 && c + (lane >> 3) < c1) red[c + (lane >> 3) - c0] += sum;
    }
}

// PIPE: double-buffer the next U columns' loads behind this U's multiply-adds
// (same sums in the same order).  Off for float64, whose tiles are the widest
// (measured no faster), for the generic widths, whose tiles hold up to nine
// words (measured 20-30% slower with it), and for callers short of registers.
template <int FMT, int U, int LM, bool PIPE = FMT != CB_F64 && !is_generic<FMT>>
__device__ __forceinline__ void subtract_tile(const BasisView& V, int j, const double* __restrict__ h,
                                              int tile0, int lane, double* acc) {
    if constexpr (!PIPE) {
        for (int c = 0; c < j; c += U) {
            Tile<FMT> t[U];
            int cols[U];
#pragma unroll
            for (int u = 0; u < U; ++u) cols[u] = min(c + u, j - 1);
            load_tiles<FMT, U, LM>(t, V, cols, tile0, lane);
#pragma unroll
            for (int u = 0; u < U; ++u)
                t[u].axpy(c + u < j ? h[c + u] : 0.0, acc);
        }
    } else {
        Tile<FMT> t[U], nx[U];
        int cols[U];
#pragma unroll
        for (int u = 0; u < U; ++u) cols[u] = min(u, j - 1);
        load_tiles<FMT, U, LM>(t, V, cols, tile0, lane);
        for (int c = 0; c < j; c += U) {
            const bool more = c + U < j;
            if (more) {
#pragma unroll
                for (int u = 0; u < U; ++u) cols[u] = min(c + U + u, j - 1);
                load_tiles<FMT, U, LM>(nx, V, cols, tile0, lane);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                t[u].axpy(c + u < j ? h[c + u] : 0.0, acc);
            if (more) {
#pragma unroll
                for (int u = 0; u < U; ++u) t[u] = nx[u];
            }
        }
    }
}

}  // namespace dev
}  // namespace cb
