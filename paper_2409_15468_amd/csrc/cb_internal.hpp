// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/cbgmres.h"

namespace cb {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
int fail(int status, const char* fmt, ...);

#define CB_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::cb::fail(CB_ERR_HIP, "%s failed: %s (%s:%d)", #call,                 \
                              hipGetErrorString(e_), __FILE__, __LINE__);                 \
    } while (0)

// NULL counts as aligned (optional arguments)
inline bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

// ---------------------------------------------------------------- geometry
constexpr int kBS = 32;           // FRSZ2 block size (values per shared exponent)
constexpr int kSeg = 8;           // rows per thread in the row-segment kernels
constexpr int kThreads = 256;     // threads per workgroup in the row kernels
constexpr int kRowsPerWG = kThreads * kSeg;  // 2048 rows = 64 FRSZ2 blocks
constexpr int kCounterBytes = 8192;  // ticket counters of the last-workgroup reductions
constexpr int kMaxRestart = 512;  // largest restart length m
// Largest row count: row indices, row-group starts and the 8-row groups past
// them (up to 2048 * row_groups(n)) all stay below 2^31 in 32-bit arithmetic.
constexpr int64_t kMaxRows = (int64_t(1) << 31) - 4096;
// one-workgroup batched solver (batch.hip)
constexpr int kBatchThreads = 512;
constexpr int kBatchMaxN = 65536;
constexpr int kBatchMaxRestart = 104;
int64_t batch_workspace_bytes(int32_t n, int32_t m, int format);

// Serving ring (batch.hip): a persistent one-workgroup-per-system launch that
// takes small systems from descriptors published while it runs.
constexpr int kRingSlots = 1024;  // descriptors in flight at most (a power of two)
struct BatchRing;
// Pinned/mapped/coherent control block, descriptors and results; NULL on failure.
BatchRing* ring_create(int grid, int idle_polls, double slice_s);
// Publish one system: q holds its device buffers (validated as for
// cbgmres_solve_batch), the h_ pointers its inputs and the output x in
// host memory that is pinned, mapped and coherent.  *seq receives the
// sequence number.  CB_ERR_WORKSPACE if every slot is busy.
int ring_publish(BatchRing* r, const cb_batch_item& q, const int32_t* h_row_ptr, const int32_t* h_col,
                 const double* h_val, const double* h_b, const double* h_x0, double* h_x, uint32_t* seq);
// true once system seq has finished; then *res and *launch (the launch that
// served it) are set and its slot is free again.
bool ring_poll(BatchRing* r, uint32_t seq, cb_result* res, uint32_t* launch);
// Launch the ring kernel on s unless a launch is still running; returns the
// new launch's number, or 0 if none was started.  CB status via *status.
uint32_t ring_kick(BatchRing* r, hipStream_t s, int* status);
bool ring_running(BatchRing* r);
// Ask the kernel to leave once nothing is left to claim, and wait for it.
void ring_stop(BatchRing* r);
void ring_destroy(BatchRing* r);

inline int64_t nblocks(int64_t n) { return (n + kBS - 1) / kBS; }
inline int64_t padded_rows(int64_t n) { return nblocks(n) * kBS; }
inline int row_groups(int64_t n) { return (int)((padded_rows(n) + kRowsPerWG - 1) / kRowsPerWG); }
__host__ __device__ inline int row_groups_dev(int np) { return (np + kRowsPerWG - 1) / kRowsPerWG; }
// workgroups of the basis kernels: one per row group, at most kProjectGroups
constexpr int kProjectGroups = 1024;
inline int project_groups(int64_t n) { int g = row_groups(n); return g < kProjectGroups ? g : kProjectGroups; }
// The projection alone (h = V^T w) runs best with half as many, longer
// workgroups: measured 2% faster at 2^24 rows, where the updates are not.
constexpr int kDotGroups = 512;
inline int dot_groups(int64_t n) { int g = project_groups(n); return g < kDotGroups ? g : kDotGroups; }

// Kernel template ids of the generic-l FRSZ2 codec (formats CB_FRSZ2_BITS(l)
// and CB_FRSZ2_B64_BITS(l)); l and the block size travel in BasisView.  GENW
// (l >= kWideBits) reads a lane's words as aligned 16-byte pieces, GEN as
// single words.
constexpr int CB_FRSZ2_GEN = 15;
constexpr int CB_FRSZ2_GENW = 14;
constexpr int kWideBits = 26;
template <int FMT> constexpr bool is_generic = FMT == CB_FRSZ2_GEN || FMT == CB_FRSZ2_GENW;
inline bool generic_b64(int f) { return f >= CB_FRSZ2_B64_BITS(3) && f <= CB_FRSZ2_B64_BITS(32); }
inline bool generic_format(int f) {
    return (f >= CB_FRSZ2_BITS(3) && f <= CB_FRSZ2_BITS(32)) || generic_b64(f);
}
inline bool valid_format(int f) { return (f >= CB_F64 && f <= CB_FRSZ2_32_B64) || generic_format(f); }
// formats the one-workgroup batched solver runs (the paper's block size 32)
inline bool batch_format(int f) { return f >= CB_F64 && f <= CB_FRSZ2_32; }
inline int frsz2_bits_of(int f) {
    return f == CB_FRSZ2_16 || f == CB_FRSZ2_16_B64 ? 16 : f == CB_FRSZ2_21 ? 21
         : f == CB_FRSZ2_32 || f == CB_FRSZ2_32_B64 ? 32
         : generic_b64(f) ? f - CB_FRSZ2_B64_GENERIC_BASE
         : generic_format(f) ? f - CB_FRSZ2_GENERIC_BASE : 0;
}
// log2 of the FRSZ2 block size (5 for float formats: rows are padded to 32)
inline int block_log_of(int f) { return f == CB_FRSZ2_16_B64 || f == CB_FRSZ2_32_B64 || generic_b64(f) ? 6 : 5; }
// the template instance that runs format f
inline int kernel_format(int f) {
    return generic_format(f) ? (frsz2_bits_of(f) >= kWideBits ? CB_FRSZ2_GENW : CB_FRSZ2_GEN) : f;
}
// rows a basis column of format f stores: n rounded up to its block size
inline int64_t padded_rows_of(int f, int64_t n) {
    const int64_t bs = int64_t(1) << block_log_of(f);
    return (n + bs - 1) / bs * bs;
}
int64_t column_bytes(int f, int64_t n);       // column stride (256-byte multiple)
int64_t column_data_bytes(int f, int64_t n);  // bytes of one column's values
int64_t exponent_words(int f, int64_t n);

// Device view of a basis (column-major, see cbgmres.h).
struct BasisView {
    const unsigned char* values;
    const uint32_t* exps;
    int64_t col_bytes;
    int64_t exp_stride;  // exponent words per column
    int32_t n;
    int32_t np;          // rows stored: n rounded up to the block size
    int32_t bits;        // FRSZ2 l (0 for float formats)
    int32_t bs_log;      // log2 of the FRSZ2 block size (5 or 6)
};
inline BasisView view_of(const cb_basis& V) {
    BasisView b;
    b.values = static_cast<const unsigned char*>(V.values);
    b.exps = V.exps;
    b.col_bytes = column_bytes(V.format, V.n);
    b.exp_stride = exponent_words(V.format, V.n);
    b.n = V.n;
    b.np = (int32_t)padded_rows_of(V.format, V.n);
    b.bits = frsz2_bits_of(V.format);
    b.bs_log = block_log_of(V.format);
    return b;
}

// SpMV geometry: lanes per row and rows per workgroup depend on the matrix only.
constexpr int kSpmvGroups = 2048;
constexpr int kXcds = 8;  // accelerator dies (XCDs), each with its own L2; workgroup w runs on XCD w % 8
int spmv_lanes_per_row(int32_t n, int32_t nnz);
int spmv_groups(int32_t n, int32_t nnz);
int64_t reduce_workspace_bytes(int32_t n, int32_t ncols, int32_t nnz);

struct Epi;  // last-workgroup reduction / solver step logic (epilogue.hpp)

// ---------------------------------------------------------------- launchers (no validation)
// `guard` (nullable device int): a kernel whose guard reads 0 does nothing.
// `jdev` (nullable device int): column count read on the device (overrides j).
void launch_store(int fmt, const cb_basis& V, int col, const double* w, const double* divisor,
                  double* v_out, int32_t* flag, const int* guard, hipStream_t s);
void launch_load(int fmt, const cb_basis& V, int col, double* x, hipStream_t s);
// h = V^T w: partials[c * G + g] for c < j, then the epilogue e (its counter
// must read 0) forms and uses the sums.
void launch_project(int fmt, const cb_basis& V, int j, const double* w, double* partials,
                    const int* guard, const Epi& e, hipStream_t s);
// w += sign * V h (h device); with partials != NULL also ||w||^2 per
// workgroup and the epilogue e on it.
void launch_subtract(int fmt, const cb_basis& V, int j, const int* jdev, const double* h,
                     double* w, double* partials, const int* guard, int accumulate_sign,
                     const Epi& e, hipStream_t s);
// w -= V h (h device, j coefficients), then partials of u = V^T w (c < j) and
// ||w||^2 (c = j), and the epilogue e (FUSED_CHECK).
void launch_subtract_project(int fmt, const cb_basis& V, int j, const double* h, double* w, double* partials,
                             const int* guard, const Epi& e, hipStream_t s);
void launch_zero_counter(unsigned* counter, hipStream_t s);
// Stage 2: out[c] (op 0: =, op 1: +=) = sum_g partials[c * G + g], c < ncols.
void launch_reduce(const double* partials, int G, int ncols, double* out, int op,
                   const int* guard, hipStream_t s);
// y = A x (mode 0) or y = b - A x (mode 1); with partials != NULL also
// ||y||^2 per workgroup (spmv_groups of them, summed by the consumer).
// plan (optional, from launch_spmv_plan): per 512-row block the range of
// columns, so that rows longer than 8 entries on average gather x from LDS.
void launch_spmv(const cb_csr& A, const double* x, const double* b, double* y, double* partials,
                 int mode, const int* guard, hipStream_t s, const void* plan = nullptr);
// The SpMV plan: bytes, whether the matrix's SpMV uses it, and its kernel.
int64_t spmv_plan_bytes(int32_t n);
bool spmv_uses_plan(int32_t n, int32_t nnz);
void launch_spmv_plan(const cb_csr& A, void* plan, hipStream_t s);
void launch_fill(double* x, double v, int64_t n, hipStream_t s);
// Column col := Q(w / *divisor) and y = A (w / *divisor), ||y||^2 partials
// (spmv_groups of them); flag (device, required) set on a non-finite store.
void launch_spmv_store(int fmt, const cb_csr& A, const cb_basis& V, int col, const double* w,
                       const double* divisor, double* y, double* partials, int32_t* flag, const int* guard,
                       hipStream_t s, const void* plan = nullptr);

}  // namespace cb
