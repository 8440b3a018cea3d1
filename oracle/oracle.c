/*
 * oracle.c -- plain, slow, single-thread FP64 CPU oracle for GMRES with an
 * FRSZ2-compressed (or low-precision) Krylov basis.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the HIP library; it depends on libc and libm alone.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math), so every
 * product and sum is a separately rounded IEEE operation in program order.
 *
 * Where the paper is silent or garbled, the readings used are the ones listed
 * in the design notes (truncation when cutting to l bits, the biased raw block
 * exponent as the stored integer, LSB-first bit packing, +0.0 tail padding,
 * the DGKS constant eta = 1/sqrt(2), the "twice is enough" breakdown test,
 * Givens rotations for the least-squares problem, the FP64 vector v fed to the
 * SpMV, IEEE division when normalising).
 */
#include <fenv.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Basis storage formats (the "basis knob").  The numbering is part of the
 * storage contract that the tests rely on. */
enum { OR_F64 = 0, OR_F32 = 1, OR_F16 = 2, OR_FRSZ2_16 = 3, OR_FRSZ2_21 = 4, OR_FRSZ2_32 = 5,
       OR_FRSZ2_16_B64 = 6, OR_FRSZ2_32_B64 = 7 };

#define OR_BS 32     /* FRSZ2 block size of the paper's runs (Section IV-C, item 2) */
#define OR_BS_MAX 64 /* the other block size offered: 64 values per exponent */

static int64_t nblocks_of(int64_t n) { return (n + OR_BS - 1) / OR_BS; }
static int64_t nblocks_bs(int64_t n, int bs) { return (n + bs - 1) / bs; }

/* ------------------------------------------------------------------------ */
/* FRSZ2 compression: the six steps of Section IV-A, Eq. (1)-(2).           */
/* ------------------------------------------------------------------------ */

/* Split an IEEE double into sign, biased exponent and 52 fraction bits
 * (Eq. 1). */
static void ieee_split(double x, unsigned* s, unsigned* e, uint64_t* f) {
    uint64_t b;
    memcpy(&b, &x, 8);
    *s = (unsigned)(b >> 63);
    *e = (unsigned)((b >> 52) & 0x7FF);
    *f = b & ((UINT64_C(1) << 52) - 1);
}

/* Encode one block of bs values, bs = 32 or 64 (missing tail values already
 * replaced by +0.0).  Writes the block's bs*l/32 words (the bit stream of the
 * codes, code q at bits [q*l, (q+1)*l), LSB first, little-endian 32-bit
 * words) and returns the stored exponent word.  *nonfinite is set when the
 * block holds Inf/NaN (its words are then meaningless). */
static uint32_t frsz2_encode_block(const double* x, int l, int bs, uint32_t* words, int* nonfinite) {
    unsigned s[OR_BS_MAX], e[OR_BS_MAX];
    uint64_t f[OR_BS_MAX];
    unsigned emax = 0;
    /* Step 1: extract every exponent and find the block maximum. */
    for (int q = 0; q < bs; ++q) {
        ieee_split(x[q], &s[q], &e[q], &f[q]);
        if (e[q] > emax) emax = e[q];
    }
    if (emax == 0x7FF) *nonfinite = 1;
    /* A block of zeros and subnormals normalises against exponent field 1,
     * the exponent at which subnormals live. */
    unsigned emax_eff = emax ? emax : 1;
    memset(words, 0, (size_t)l * 4 * (bs / 32));
    for (int q = 0; q < bs; ++q) {
        /* Step 2: significand with the usually implicit leading 1 made
         * explicit (subnormals have a leading 0 and live at exponent 1). */
        unsigned e_eff = e[q] ? e[q] : 1;
        uint64_t sig = (e[q] ? (UINT64_C(1) << 52) : 0) | f[q]; /* 53 bits: 1.b51..b0 */
        /* Step 3: prefix k = emax - e zero bits, i.e. shift right by k. */
        unsigned k = emax_eff - e_eff;
        /* Step 5 (applied to the magnitude): keep the leading l-1 bits of the
         * prefixed significand -- the integer bit and l-2 fraction bits --
         * truncating the rest.  The significand has 53 bits, so keeping l-1
         * of the (53+k) bits means dropping 54-l+k low bits. */
        unsigned drop = (unsigned)(54 - l) + k;
        uint64_t mag = drop >= 53 ? 0 : (sig >> drop);
        /* Step 4: the sign bit goes to the left of the significand. */
        uint64_t c = ((uint64_t)s[q] << (l - 1)) | mag;
        /* Step 6: store the code (bit by bit, LSB first). */
        for (int t = 0; t < l; ++t) {
            unsigned pos = (unsigned)(q * l + t);
            words[pos / 32] |= (uint32_t)((c >> t) & 1u) << (pos % 32);
        }
    }
    return emax;
}

/* Compress n values in blocks of bs (32 or 64).  exps has ceil(n/bs)
 * entries, words (bs/32)*l*ceil(n/bs).  Returns 1 if any block held a
 * non-finite value, else 0. */
int or_frsz2_encode_bs(const double* x, int64_t n, int l, int bs, uint32_t* exps, uint32_t* words) {
    int nonfinite = 0;
    double blk[OR_BS_MAX];
    const int64_t bw = (int64_t)l * (bs / 32); /* words per block */
    for (int64_t b = 0; b < nblocks_bs(n, bs); ++b) {
        for (int q = 0; q < bs; ++q) {
            int64_t i = b * bs + q;
            blk[q] = i < n ? x[i] : 0.0; /* pad the tail with +0.0 */
        }
        exps[b] = frsz2_encode_block(blk, l, bs, words + b * bw, &nonfinite);
    }
    return nonfinite;
}

int or_frsz2_encode(const double* x, int64_t n, int l, uint32_t* exps, uint32_t* words) {
    return or_frsz2_encode_bs(x, n, l, OR_BS, exps, words);
}

/* Read code q of a block's bit stream. */
static uint64_t frsz2_code(const uint32_t* blockwords, int l, int q) {
    uint64_t c = 0;
    for (int t = 0; t < l; ++t) {
        unsigned pos = (unsigned)(q * l + t);
        c |= (uint64_t)((blockwords[pos / 32] >> (pos % 32)) & 1u) << t;
    }
    return c;
}

/* Decompression, closed form of Eq. (2): the value of code c in a block with
 * stored exponent E is (-1)^sign * M * 2^(E_eff - 1023 - (l-2)), M the l-1
 * magnitude bits (integer bit plus l-2 fraction bits).  Every such value is
 * a multiple of 2^-1074 below 2^1024, hence exactly representable. */
void or_frsz2_decode_bs(const uint32_t* exps, const uint32_t* words, int64_t n, int l, int bs, double* x) {
    const int64_t bw = (int64_t)l * (bs / 32);
    for (int64_t i = 0; i < n; ++i) {
        int64_t b = i / bs;
        int q = (int)(i % bs);
        uint64_t c = frsz2_code(words + b * bw, l, q);
        uint64_t M = c & ((UINT64_C(1) << (l - 1)) - 1);
        int neg = (int)((c >> (l - 1)) & 1u);
        int E = (int)exps[b];
        int Eeff = E ? E : 1;
        double v = ldexp((double)M, Eeff - 1023 - (l - 2));
        x[i] = neg ? -v : v;
    }
}

void or_frsz2_decode(const uint32_t* exps, const uint32_t* words, int64_t n, int l, double* x) {
    or_frsz2_decode_bs(exps, words, n, l, OR_BS, x);
}

/* Random-access decompression of value i by the four steps of Section IV-B:
 * read the block exponent and the code; split off the sign and count the
 * leading zeros k of the significand; drop them and the explicit 1, giving
 * the exponent e = E - k; merge sign, exponent and significand into IEEE bits.
 * An independent route to the same value as the closed form above. */
double or_frsz2_decode_value_bs(const uint32_t* exps, const uint32_t* words, int64_t i, int l, int bs) {
    int64_t b = i / bs;
    int q = (int)(i % bs);
    /* Step 1 */
    unsigned E = exps[b];
    unsigned Eeff = E ? E : 1;
    uint64_t c = frsz2_code(words + b * (int64_t)l * (bs / 32), l, q);
    /* Step 2 */
    uint64_t sign = (c >> (l - 1)) & 1u;
    uint64_t M = c & ((UINT64_C(1) << (l - 1)) - 1);
    uint64_t bits = sign << 63;
    if (M != 0) {
        int k = 0; /* leading zeros inside the (l-1)-bit significand field */
        while (!((M >> (l - 2 - k)) & 1u)) ++k;
        int top = l - 2 - k; /* position of the leading 1 */
        /* Step 3 */
        int e = (int)Eeff - k;
        if (e >= 1) {
            uint64_t frac = M - (UINT64_C(1) << top);
            /* Step 4 */
            bits |= ((uint64_t)e << 52) | (frac << (52 - top));
        } else {
            /* The merged value lies below the normal range: it is stored as a
             * subnormal, whose field is the value in units of 2^-1074. */
            bits |= M << (Eeff + 53 - (unsigned)l);
        }
    }
    double v;
    memcpy(&v, &bits, 8);
    return v;
}

double or_frsz2_decode_value(const uint32_t* exps, const uint32_t* words, int64_t i, int l) {
    return or_frsz2_decode_value_bs(exps, words, i, l, OR_BS);
}

/* ------------------------------------------------------------------------ */
/* Baseline storage formats: IEEE float32 and float16 with one rounding.     */
/* ------------------------------------------------------------------------ */

/* float16 from float64 rounded to nearest, ties to even, in one step.  The
 * value is scaled to units of the float16 spacing of its binade (exact,
 * a power-of-two scaling), rounded to an integer by nearbyint in the default
 * round-to-nearest-even mode, and the bits are read off the rounded value. */
uint16_t or_f16_from_f64(double x) {
    uint16_t sgn = signbit(x) ? 0x8000u : 0u;
    if (isnan(x)) return (uint16_t)(sgn | 0x7E00u);
    double a = fabs(x);
    if (a >= 65520.0) return (uint16_t)(sgn | 0x7C00u); /* rounds to infinity */
    int ex;
    if (a >= ldexp(1.0, -14)) {
        frexp(a, &ex);
        ex -= 1; /* a in [2^ex, 2^(ex+1)) */
    } else {
        ex = -14; /* subnormal spacing 2^-24 */
    }
    double ulp = ldexp(1.0, ex - 10);
    double r = nearbyint(a / ulp) * ulp;
    if (r == 0.0) return sgn;
    int er;
    frexp(r, &er);
    er -= 1;
    if (er < -14) return (uint16_t)(sgn | (uint16_t)(r / ldexp(1.0, -24)));
    uint16_t mant = (uint16_t)(r / ldexp(1.0, er - 10) - 1024.0);
    return (uint16_t)(sgn | (uint16_t)((er + 15) << 10) | mant);
}

double or_f64_from_f16(uint16_t h) {
    int neg = h >> 15;
    int e = (h >> 10) & 0x1F;
    int m = h & 0x3FF;
    double v;
    if (e == 0x1F) v = m ? NAN : INFINITY;
    else if (e == 0) v = ldexp((double)m, -24);
    else v = ldexp((double)(1024 + m), e - 25);
    return neg ? -v : v;
}

/* ------------------------------------------------------------------------ */
/* Basis column storage.  Column c of an ncols-wide basis over n rows uses    */
/* col_bytes = nb*32*{8,4,2} for float64/32/16 (nb = ceil(n/32)) and          */
/* nbs*(bs/32)*l*4 for frsz2_l with blocks of bs values (nbs = ceil(n/bs));   */
/* frsz2 columns also own nbs exponent words.  Rows past n hold +0.0.         */
/* ------------------------------------------------------------------------ */

/* FRSZ2 with any l in [3, 32]: format number 64 + l with blocks of 32 values,
 * 128 + l with blocks of 64 (l is a free parameter of the format, Section
 * IV-A; the fixed widths also have the numbers above). */
#define OR_FRSZ2_ANY(l) (64 + (l))
#define OR_FRSZ2_B64_ANY(l) (128 + (l))

static int frsz2_bits(int fmt) {
    if (fmt >= OR_FRSZ2_ANY(3) && fmt <= OR_FRSZ2_ANY(32)) return fmt - 64;
    if (fmt >= OR_FRSZ2_B64_ANY(3) && fmt <= OR_FRSZ2_B64_ANY(32)) return fmt - 128;
    return fmt == OR_FRSZ2_16 || fmt == OR_FRSZ2_16_B64 ? 16 : fmt == OR_FRSZ2_21 ? 21
         : fmt == OR_FRSZ2_32 || fmt == OR_FRSZ2_32_B64 ? 32 : 0;
}

static int frsz2_bs(int fmt) {
    return fmt == OR_FRSZ2_16_B64 || fmt == OR_FRSZ2_32_B64 ||
           (fmt >= OR_FRSZ2_B64_ANY(3) && fmt <= OR_FRSZ2_B64_ANY(32)) ? 64 : 32;
}

int64_t or_basis_col_bytes(int fmt, int64_t n) {
    int64_t nb = nblocks_of(n);
    switch (fmt) {
    case OR_F64: return nb * 32 * 8;
    case OR_F32: return nb * 32 * 4;
    case OR_F16: return nb * 32 * 2;
    default: return nblocks_bs(n, frsz2_bs(fmt)) * (frsz2_bs(fmt) / 32) * frsz2_bits(fmt) * 4;
    }
}

/* exponent words of one column: ceil(n / bs) for frsz2, 0 for float formats */
int64_t or_basis_exp_words(int fmt, int64_t n) {
    return frsz2_bits(fmt) ? nblocks_bs(n, frsz2_bs(fmt)) : 0;
}

/* Q(x): store one column.  Returns 1 if a non-finite value was met. */
int or_basis_encode(int fmt, const double* x, int64_t n, void* vals, uint32_t* exps) {
    int64_t np = nblocks_of(n) * 32;
    int bad = 0;
    if (fmt == OR_F64) {
        double* o = (double*)vals;
        for (int64_t i = 0; i < np; ++i) {
            o[i] = i < n ? x[i] : 0.0;
            if (!isfinite(o[i])) bad = 1;
        }
    } else if (fmt == OR_F32) {
        float* o = (float*)vals;
        for (int64_t i = 0; i < np; ++i) {
            o[i] = i < n ? (float)x[i] : 0.0f;
            if (!isfinite(o[i])) bad = 1;
        }
    } else if (fmt == OR_F16) {
        uint16_t* o = (uint16_t*)vals;
        for (int64_t i = 0; i < np; ++i) {
            o[i] = i < n ? or_f16_from_f64(x[i]) : 0;
            if ((o[i] & 0x7C00u) == 0x7C00u) bad = 1;
        }
    } else {
        bad = or_frsz2_encode_bs(x, n, frsz2_bits(fmt), frsz2_bs(fmt), exps, (uint32_t*)vals);
    }
    return bad;
}

/* D(.): read one column back as float64. */
void or_basis_decode(int fmt, const void* vals, const uint32_t* exps, int64_t n, double* x) {
    if (fmt == OR_F64) {
        memcpy(x, vals, (size_t)n * 8);
    } else if (fmt == OR_F32) {
        for (int64_t i = 0; i < n; ++i) x[i] = (double)((const float*)vals)[i];
    } else if (fmt == OR_F16) {
        for (int64_t i = 0; i < n; ++i) x[i] = or_f64_from_f16(((const uint16_t*)vals)[i]);
    } else {
        or_frsz2_decode_bs(exps, (const uint32_t*)vals, n, frsz2_bits(fmt), frsz2_bs(fmt), x);
    }
}

/* ------------------------------------------------------------------------ */
/* FP64 kernels: compensated (Neumaier) sums, so the oracle's dot products,   */
/* norms and SpMV rows are accurate to about one rounding of the result.      */
/* ------------------------------------------------------------------------ */

typedef struct { double s, c; } nsum;

static void nsum_add(nsum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

double or_dot(int64_t n, const double* a, const double* b) {
    nsum acc = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) nsum_add(&acc, a[i] * b[i]);
    return acc.s + acc.c;
}

double or_nrm2(int64_t n, const double* a) { return sqrt(or_dot(n, a, a)); }

/* y = A x for a CSR matrix (int32 indices), each row summed in CSR order. */
void or_spmv(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
             const double* x, double* y) {
    for (int64_t i = 0; i < n; ++i) {
        nsum acc = {0.0, 0.0};
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) nsum_add(&acc, val[k] * x[col[k]]);
        y[i] = acc.s + acc.c;
    }
}

/* Classical Gram-Schmidt against j decoded basis columns (Fig. 1 step 5):
 * h_i = <v_i, w> for every i against the same w. Vdec has column stride ld. */
void or_cgs_project(int64_t n, int j, const double* Vdec, int64_t ld, const double* w, double* h) {
    for (int i = 0; i < j; ++i) h[i] = or_dot(n, Vdec + (int64_t)i * ld, w);
}

/* w := w - V h, each row's correction summed over the columns in order first
 * and then subtracted (Fig. 1 step 5, second half). */
void or_cgs_subtract(int64_t n, int j, const double* Vdec, int64_t ld, const double* h, double* w) {
    for (int64_t k = 0; k < n; ++k) {
        double s = 0.0;
        for (int i = 0; i < j; ++i) s += h[i] * Vdec[(int64_t)i * ld + k];
        w[k] = w[k] - s;
    }
}

/* ------------------------------------------------------------------------ */
/* Restarted GMRES with classical Gram-Schmidt and one conditional           */
/* re-orthogonalisation (Fig. 1), no preconditioner (M = I, Section V-C).    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t iterations;  /* Arnoldi steps in total */
    int32_t restarts;    /* cycles started */
    int32_t reorths;     /* steps that ran the second Gram-Schmidt pass */
    int32_t breakdowns;  /* cycles ended by the breakdown test */
    int32_t converged;   /* explicit residual met the tolerance */
    int32_t status;      /* 0 ok, 2 non-finite, 3 not converged */
    double rel_residual; /* last explicit ||b-Ax||/||b|| (-1: not evaluated) */
    double implicit_rel_residual; /* last |g_{j+1}|/||b|| */
} or_stats;

typedef struct {
    double eta;            /* re-orthogonalisation threshold, 1/sqrt(2) */
    int32_t max_iters;     /* cap on Arnoldi steps (0: 20000) */
    int32_t max_cycles;    /* cap on cycles; 0 = unlimited.  When reached the
                              solve returns after the x update without a final
                              explicit residual */
    int32_t literal_breakdown; /* 1: compare against the pre-orthogonalisation
                                  norm as Fig. 1 step 12 is printed */
} or_options;

/* Apply the stored rotations G_0..G_{j-1} to a new Hessenberg column. */
static void givens_apply(int j, double* hcol, const double* cs, const double* sn) {
    for (int i = 0; i < j; ++i) {
        double a = hcol[i], b = hcol[i + 1];
        hcol[i] = cs[i] * a + sn[i] * b;
        hcol[i + 1] = -sn[i] * a + cs[i] * b;
    }
}

typedef struct {
    int32_t steps;     /* Arnoldi steps taken in this cycle (m') */
    int32_t reorths;   /* steps that re-orthogonalised */
    int32_t breakdown; /* the cycle ended by the breakdown test */
    int32_t status;    /* 0 ok, 2 non-finite */
    double gabs;       /* |g_{m'+1}|, the implicit residual norm */
} or_cycle_info;

/* One GMRES cycle (Fig. 1 steps 1-17) from the residual r with norm beta.
 *   enc/exps  storage for m+1 encoded columns (column stride
 *             or_basis_col_bytes / ceil(n/32)); on return they hold Q(v_i)
 *   Vdec      n*(m+1) doubles: D(Q(v_i)), column stride n
 *   H         (m+1)*m doubles, column-major, ld m+1: on return the rotated
 *             upper-triangular R in rows 0..m'-1
 *   Hraw      nullable; the unrotated Hessenberg matrix, same layout
 *   Vfp       nullable; n*(m+1) doubles: the FP64 vectors v_i themselves
 *             (column stride n), i.e. what the SpMV reads and what Q encodes
 *   y         m doubles: the least-squares solution of R y = g
 *   hist      nullable; |g_{j+1}| per step
 * Stops after m steps, when |g_{j+1}| <= tol_abs, on breakdown, or after
 * max_steps steps. */
static void gmres_cycle(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                        const double* dinv, const double* r, double beta, int m, int fmt, double eta,
                        int literal, double tol_abs, int max_steps, unsigned char* enc, uint32_t* exps,
                        double* Vdec, double* H, double* Hraw, double* Vfp, double* y, double* hist,
                        or_cycle_info* info) {
    int64_t cb = or_basis_col_bytes(fmt, n);
    int64_t nbk = nblocks_of(n);
    double* cs = malloc((size_t)m * 8);
    double* sn = malloc((size_t)m * 8);
    double* g = malloc((size_t)(m + 1) * 8);
    double* w = malloc((size_t)n * 8);
    double* v = malloc((size_t)n * 8);
    double* u = malloc((size_t)(m + 1) * 8);
    double* z = dinv ? malloc((size_t)n * 8) : NULL;
    memset(info, 0, sizeof *info);
    memset(H, 0, (size_t)(m + 1) * m * 8);
    if (Hraw) memset(Hraw, 0, (size_t)(m + 1) * m * 8);
    /* Step 1: v = r / beta (IEEE division per entry), V_1 = [Q(v)] */
    for (int64_t k = 0; k < n; ++k) v[k] = r[k] / beta;
    if (Vfp) memcpy(Vfp, v, (size_t)n * 8);
    if (or_basis_encode(fmt, v, n, enc, exps)) { info->status = 2; goto done; }
    or_basis_decode(fmt, enc, exps, n, Vdec);
    for (int i = 0; i <= m; ++i) g[i] = 0.0;
    g[0] = beta;
    for (int j = 0; j < m; ++j) {
        double* h = H + (int64_t)j * (m + 1);
        /* Steps 3-4: w = A (M^-1 v) with the FP64 v, omega = ||w||; with a
         * Jacobi preconditioner M^-1 v is the entrywise product dinv * v */
        if (dinv) {
            for (int64_t k = 0; k < n; ++k) z[k] = dinv[k] * v[k];
            or_spmv(n, row_ptr, col, val, z, w);
        } else {
            or_spmv(n, row_ptr, col, val, v, w);
        }
        double omega = or_nrm2(n, w);
        /* Steps 5-6: classical Gram-Schmidt against the stored basis */
        or_cgs_project(n, j + 1, Vdec, n, w, h);
        or_cgs_subtract(n, j + 1, Vdec, n, h, w);
        double hn = or_nrm2(n, w);
        int breakdown = 0;
        /* Steps 7-11: one re-orthogonalisation pass when the norm fell */
        if (hn < eta * omega) {
            info->reorths += 1;
            double omega2 = hn;
            or_cgs_project(n, j + 1, Vdec, n, w, u);
            or_cgs_subtract(n, j + 1, Vdec, n, u, w);
            for (int i = 0; i <= j; ++i) h[i] += u[i];
            hn = or_nrm2(n, w);
            breakdown = literal ? (hn < eta * omega) : (hn < eta * omega2);
        }
        /* Step 12 */
        if (hn == 0.0) breakdown = 1;
        if (!isfinite(hn)) { info->status = 2; goto done; }
        h[j + 1] = hn;
        if (Hraw) memcpy(Hraw + (int64_t)j * (m + 1), h, (size_t)(j + 2) * 8);
        /* Steps 16-17: least squares by Givens rotations */
        givens_apply(j, h, cs, sn);
        double rho = sqrt(h[j] * h[j] + hn * hn);
        cs[j] = h[j] / rho;
        sn[j] = hn / rho;
        h[j] = rho;
        h[j + 1] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        info->steps = j + 1;
        info->gabs = fabs(g[j + 1]);
        if (hist) hist[j] = info->gabs;
        if (info->gabs <= tol_abs || breakdown || info->steps >= max_steps) {
            info->breakdown = breakdown;
            break;
        }
        /* Steps 13-14: normalise (IEEE division) and store the new vector */
        for (int64_t k = 0; k < n; ++k) v[k] = w[k] / hn;
        if (Vfp) memcpy(Vfp + (int64_t)(j + 1) * n, v, (size_t)n * 8);
        if (or_basis_encode(fmt, v, n, enc + (j + 1) * cb, exps + (j + 1) * nbk)) {
            info->status = 2;
            goto done;
        }
        or_basis_decode(fmt, enc + (j + 1) * cb, exps + (j + 1) * nbk, n, Vdec + (int64_t)(j + 1) * n);
    }
    /* Step 17: back-substitution R y = g */
    for (int i = info->steps - 1; i >= 0; --i) {
        double s = g[i];
        for (int k = i + 1; k < info->steps; ++k) s -= H[(int64_t)k * (m + 1) + i] * y[k];
        y[i] = s / H[(int64_t)i * (m + 1) + i];
    }
done:
    free(cs); free(sn); free(g); free(w); free(v); free(u); free(z);
}

void or_gmres_cycle(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                    const double* r, double beta, int m, int fmt, double eta, int literal,
                    double tol_abs, int max_steps, unsigned char* enc, uint32_t* exps,
                    double* Vdec, double* H, double* Hraw, double* Vfp, double* y, double* hist,
                    or_cycle_info* info) {
    gmres_cycle(n, row_ptr, col, val, NULL, r, beta, m, fmt, eta, literal, tol_abs, max_steps, enc,
                exps, Vdec, H, Hraw, Vfp, y, hist, info);
}

/* Jacobi preconditioner M = diag(A) (Fig. 1's M, the simplest choice):
 * dinv[i] = 1 / a_ii by IEEE division; a row whose diagonal entry is missing,
 * zero or not finite keeps dinv[i] = 1 (left unscaled). */
void or_jacobi_diag_inv(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                        double* dinv) {
    for (int64_t i = 0; i < n; ++i) {
        dinv[i] = 1.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col[k] == i && val[k] != 0.0 && isfinite(val[k])) dinv[i] = 1.0 / val[k];
    }
}

/* Restarted GMRES(m): cycles from the current x until the explicit relative
 * residual (Eq. 4) meets tol.  x holds x0 on entry and the iterate on return.
 * dinv (nullable) is the right preconditioner M^-1 = diag(dinv), Fig. 1 steps
 * 3 and 17: the Krylov space is that of A M^-1 and the update is
 * x = x0 + M^-1 (V y); the explicit residual stays b - A x. */
int or_gmres_pc(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                const double* dinv, const double* b, double* x, int m, double tol, int fmt,
                const or_options* opt, or_stats* st, double* hist, int64_t hist_cap) {
    double eta = opt ? opt->eta : 0.7071067811865476;
    int max_iters = (opt && opt->max_iters > 0) ? opt->max_iters : 20000;
    int max_cycles = opt ? opt->max_cycles : 0;
    int literal = opt ? opt->literal_breakdown : 0;
    memset(st, 0, sizeof *st);
    st->rel_residual = -1.0;
    st->implicit_rel_residual = -1.0;

    double nb = or_nrm2(n, b);
    if (nb == 0.0) { /* b = 0: x = 0 solves it exactly */
        memset(x, 0, (size_t)n * 8);
        st->converged = 1;
        st->rel_residual = 0.0;
        st->implicit_rel_residual = 0.0;
        return 0;
    }
    unsigned char* enc = malloc((size_t)(or_basis_col_bytes(fmt, n) * (m + 1)));
    uint32_t* exps = malloc((size_t)(nblocks_of(n) * (m + 1) * 4));
    double* Vdec = malloc((size_t)(n * (m + 1) * 8));
    double* H = malloc((size_t)(m + 1) * m * 8);
    double* y = malloc((size_t)m * 8);
    double* r = malloc((size_t)n * 8);
    double* ch = malloc((size_t)m * 8);
    int status = 0;
    for (;;) {
        /* Step 1 / 18: explicit residual and stop test (Eq. 4) */
        or_spmv(n, row_ptr, col, val, x, r);
        for (int64_t k = 0; k < n; ++k) r[k] = b[k] - r[k];
        double beta = or_nrm2(n, r);
        st->rel_residual = beta / nb;
        if (!isfinite(beta)) { status = 2; break; }
        if (beta <= tol * nb) { st->converged = 1; break; }
        if (st->iterations >= max_iters) { status = 3; break; }
        st->restarts += 1;
        or_cycle_info ci;
        gmres_cycle(n, row_ptr, col, val, dinv, r, beta, m, fmt, eta, literal, tol * nb,
                    max_iters - st->iterations, enc, exps, Vdec, H, NULL, NULL, y, ch, &ci);
        for (int j = 0; j < ci.steps; ++j) {
            if (hist && st->iterations + j < hist_cap) hist[st->iterations + j] = ch[j] / nb;
        }
        st->iterations += ci.steps;
        st->reorths += ci.reorths;
        st->breakdowns += ci.breakdown;
        if (ci.steps > 0) st->implicit_rel_residual = ci.gabs / nb;
        if (ci.status) { status = ci.status; break; }
        /* Step 17: x = x0 + M^-1 (V y), each row's correction summed first */
        for (int64_t k = 0; k < n; ++k) {
            double s = 0.0;
            for (int i = 0; i < ci.steps; ++i) s += y[i] * Vdec[(int64_t)i * n + k];
            x[k] = x[k] + (dinv ? dinv[k] * s : s);
        }
        if (max_cycles > 0 && st->restarts >= max_cycles) {
            status = 3;
            st->rel_residual = -1.0;
            break;
        }
    }
    st->status = status;
    free(enc); free(exps); free(Vdec); free(H); free(y); free(r); free(ch);
    return status;
}

int or_gmres(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
             const double* b, double* x, int m, double tol, int fmt, const or_options* opt,
             or_stats* st, double* hist, int64_t hist_cap) {
    return or_gmres_pc(n, row_ptr, col, val, NULL, b, x, m, tol, fmt, opt, st, hist, hist_cap);
}

/* ------------------------------------------------------------------------ */
/* Iterative refinement around an inner compressed-basis GMRES: the outer     */
/* residual, the correction and the update stay in FP64.                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t outer;       /* refinement steps taken */
    int32_t iterations;  /* inner Arnoldi steps in total */
    int32_t converged;
    int32_t status;
    double rel_residual; /* final explicit ||b-Ax||/||b|| */
} or_ir_stats;

int or_ir_solve(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                const double* b, double* x, int m, double inner_tol, double tol, int fmt,
                int max_outer, or_ir_stats* st) {
    memset(st, 0, sizeof *st);
    double nb = or_nrm2(n, b);
    if (nb == 0.0) {
        memset(x, 0, (size_t)n * 8);
        st->converged = 1;
        return 0;
    }
    double* r = malloc((size_t)n * 8);
    double* d = malloc((size_t)n * 8);
    or_options io = {0.7071067811865476, m, 1, 0};
    int status = 3;
    for (;;) {
        or_spmv(n, row_ptr, col, val, x, r);
        for (int64_t k = 0; k < n; ++k) r[k] = b[k] - r[k];
        double rn = or_nrm2(n, r);
        st->rel_residual = rn / nb;
        if (!isfinite(rn)) { status = 2; break; }
        if (rn <= tol * nb) { st->converged = 1; status = 0; break; }
        if (st->outer >= max_outer) break;
        memset(d, 0, (size_t)n * 8);
        or_stats is;
        or_gmres(n, row_ptr, col, val, r, d, m, inner_tol, fmt, &io, &is, NULL, 0);
        st->iterations += is.iterations;
        st->outer += 1;
        if (is.status == 2) { status = 2; break; }
        for (int64_t k = 0; k < n; ++k) x[k] = x[k] + d[k];
    }
    st->status = status;
    free(r); free(d);
    return status;
}

/* Dense LU with partial pivoting, used by tests as an independent small-system
 * solver (column-major a, overwritten; b overwritten by the solution). */
int or_dense_solve(int n, double* a, double* b) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(a[(int64_t)k * n + i]) > fabs(a[(int64_t)k * n + p])) p = i;
        if (a[(int64_t)k * n + p] == 0.0) return 1;
        if (p != k) {
            for (int c = 0; c < n; ++c) {
                double t = a[(int64_t)c * n + k];
                a[(int64_t)c * n + k] = a[(int64_t)c * n + p];
                a[(int64_t)c * n + p] = t;
            }
            double t = b[k]; b[k] = b[p]; b[p] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double l = a[(int64_t)k * n + i] / a[(int64_t)k * n + k];
            a[(int64_t)k * n + i] = l;
            for (int c = k + 1; c < n; ++c) a[(int64_t)c * n + i] -= l * a[(int64_t)c * n + k];
            b[i] -= l * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int c = i + 1; c < n; ++c) s -= a[(int64_t)c * n + i] * b[c];
        b[i] = s / a[(int64_t)i * n + i];
    }
    return 0;
}

/* Rounding mode guard: the oracle assumes round-to-nearest-even. */
int or_rounding_is_nearest(void) { return fegetround() == FE_TONEAREST; }
