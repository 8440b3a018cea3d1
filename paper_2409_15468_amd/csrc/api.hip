// C ABI: argument checks and launches for the codec, basis and SpMV entry
// points, plus the thread-local error text.
#include <cstdarg>
#include <cstring>
#include <mutex>

#include "cb_internal.hpp"
#include "epilogue.hpp"

namespace cb {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

int fail(int status, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return status;
}

int64_t column_data_bytes(int f, int64_t n) {
    const int64_t nb = nblocks(n);
    switch (f) {
    case CB_F64: return nb * 32 * 8;
    case CB_F32: return nb * 32 * 4;
    case CB_F16: return nb * 32 * 2;
    default:  // frsz2: l words per 32 rows of the padded column
        return valid_format(f) ? padded_rows_of(f, n) / 32 * frsz2_bits_of(f) * 4 : -1;
    }
}

// Column stride: the data rounded up to 256 bytes, so every column starts
// aligned for 16-byte loads (frsz2_21 tiles are 1344-byte runs).
int64_t column_bytes(int f, int64_t n) {
    const int64_t d = column_data_bytes(f, n);
    return d < 0 ? d : (d + 255) / 256 * 256;
}

int64_t exponent_words(int f, int64_t n) { return frsz2_bits_of(f) ? padded_rows_of(f, n) >> block_log_of(f) : 0; }

// Workspace of the primitives: a header holding the ticket counters of the
// last-workgroup reduction, then the partial sums.
int64_t reduce_workspace_bytes(int32_t n, int32_t ncols, int32_t nnz) {
    int64_t a = (int64_t)project_groups(n) * (ncols > 0 ? ncols : 1);
    int64_t b = nnz > 0 ? spmv_groups(n, nnz) : 0;
    return kCounterBytes + 8 * (a > b ? a : b);
}

static Epi store_epi(double* out, void* work) {
    Epi e{};
    e.mode = EPI_STORE;
    e.out = out;
    e.counter = static_cast<unsigned*>(work);
    return e;
}
static double* partials_of(void* work) {
    return reinterpret_cast<double*>(static_cast<unsigned char*>(work) + kCounterBytes);
}

static bool bad_n(int64_t n) { return n < 1 || n > kMaxRows; }

static int check_basis(const cb_basis* V, int need_cols) {
    if (!V) return fail(CB_ERR_INVALID_ARG, "basis descriptor is NULL");
    if (!valid_format(V->format)) return fail(CB_ERR_INVALID_ARG, "unknown basis format %d", V->format);
    if (bad_n(V->n)) return fail(CB_ERR_INVALID_ARG, "basis rows n=%d out of range", V->n);
    if (V->ncols < need_cols) return fail(CB_ERR_INVALID_ARG, "basis has %d columns, %d needed", V->ncols, need_cols);
    if (!V->values) return fail(CB_ERR_INVALID_ARG, "basis values pointer is NULL");
    if (frsz2_bits_of(V->format) && !V->exps) return fail(CB_ERR_INVALID_ARG, "frsz2 basis needs exps");
    if (!aligned(V->values, 16) || !aligned(V->exps, 4))
        return fail(CB_ERR_INVALID_ARG, "basis values must be 16-byte and exps 4-byte aligned");
    return CB_OK;
}

// the FP64 vectors the row kernels read or write in 16-byte pairs
static int check_vec16(const void* a, const void* b = nullptr, const void* c = nullptr) {
    if (!aligned(a, 16) || !aligned(b, 16) || !aligned(c, 16))
        return fail(CB_ERR_INVALID_ARG, "device vectors must be 16-byte aligned");
    return CB_OK;
}

// ----------------------------------------------------------------- projection without allocation
// Reduction workspace of cb_cgs_project_noalloc: a file-scope device array
// that covers every valid call (ticket counters, then kDotGroups partials for
// each of up to kMaxRestart + 1 columns: 2.0 MiB).  Each GPU the library runs
// on holds its own copy until the process ends.  Host code never names the
// array in a launch: it takes the device address from hipGetSymbolAddress,
// once per device, and passes that.
constexpr int64_t kNoAllocScratchBytes = kCounterBytes + 8 * (int64_t)kDotGroups * (kMaxRestart + 1);
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices];

// The scratch array's device address on the current device (looked up on the
// first call there), or NULL with the error text set.
static void* scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        fail(CB_ERR_HIP, "no usable current device (%d)", dev);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fail(CB_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_dev[dev] = p;
    }
    return g_scratch_dev[dev];
}

}  // namespace cb

using namespace cb;

extern "C" {

const char* cb_status_string(int status) {
    switch (status) {
    case CB_OK: return "ok";
    case CB_ERR_INVALID_ARG: return "invalid argument";
    case CB_ERR_UNSUPPORTED_BITS: return "unsupported FRSZ2 bit width";
    case CB_ERR_NONFINITE: return "non-finite value";
    case CB_ERR_NOT_CONVERGED: return "not converged";
    case CB_ERR_WORKSPACE: return "workspace too small";
    case CB_ERR_OVER_BUDGET: return "request exceeds the HBM budget";
    case CB_ERR_HIP: return "HIP runtime error";
    case CB_PENDING: return "pending";
    case CB_ERR_NOT_FOUND: return "unknown ticket";
    default: return "unknown status";
    }
}

const char* cb_last_error(void) { return g_err; }

int64_t frsz2_exponent_words(int64_t n) { return n < 0 ? -1 : nblocks(n); }

int64_t frsz2_value_words(int64_t n, int bits) {
    if (n < 0 || bits < 3 || bits > 32) return -1;
    return (int64_t)bits * nblocks(n);
}

static int format_of_bits(int bits) {
    return bits == 16 ? CB_FRSZ2_16 : bits == 21 ? CB_FRSZ2_21 : bits == 32 ? CB_FRSZ2_32
         : (bits >= 3 && bits <= 32) ? CB_FRSZ2_BITS(bits) : -1;
}

int frsz2_compress(const double* x, int64_t n, int bits, uint32_t* exps, uint32_t* words,
                   int32_t* nonfinite_flag, void* stream) {
    const int f = format_of_bits(bits);
    if (f < 0) return fail(CB_ERR_UNSUPPORTED_BITS, "frsz2 bits=%d (3 to 32)", bits);
    if (bad_n(n)) return fail(CB_ERR_INVALID_ARG, "n=%lld out of range", (long long)n);
    if (!x || !exps || !words) return fail(CB_ERR_INVALID_ARG, "NULL pointer");
    if (int st = check_vec16(x, words)) return st;
    if (!aligned(exps, 4)) return fail(CB_ERR_INVALID_ARG, "exps must be 4-byte aligned");
    cb_basis V{f, (int32_t)n, 1, 0, words, exps};
    int32_t* flag = nonfinite_flag;
    launch_store(f, V, 0, x, nullptr, nullptr, flag, nullptr, (hipStream_t)stream);
    CB_HIP(hipGetLastError());
    return CB_OK;
}

int frsz2_decompress(const uint32_t* exps, const uint32_t* words, int64_t n, int bits, double* x,
                     void* stream) {
    const int f = format_of_bits(bits);
    if (f < 0) return fail(CB_ERR_UNSUPPORTED_BITS, "frsz2 bits=%d (3 to 32)", bits);
    if (bad_n(n)) return fail(CB_ERR_INVALID_ARG, "n=%lld out of range", (long long)n);
    if (!x || !exps || !words) return fail(CB_ERR_INVALID_ARG, "NULL pointer");
    if (int st = check_vec16(x, words)) return st;
    if (!aligned(exps, 4)) return fail(CB_ERR_INVALID_ARG, "exps must be 4-byte aligned");
    cb_basis V{f, (int32_t)n, 1, 0, const_cast<uint32_t*>(words), const_cast<uint32_t*>(exps)};
    launch_load(f, V, 0, x, (hipStream_t)stream);
    CB_HIP(hipGetLastError());
    return CB_OK;
}

int64_t cb_basis_column_bytes(int format, int64_t n) {
    if (!valid_format(format) || n < 0) return -1;
    return column_bytes(format, n);
}

int64_t cb_basis_exponent_words(int format, int64_t n) {
    if (!valid_format(format) || n < 0) return -1;
    return exponent_words(format, n);
}

int cb_basis_store(const cb_basis* V, int32_t col, const double* w, const double* divisor,
                   double* v_out, int32_t* nonfinite_flag, void* stream) {
    if (int st = check_basis(V, col + 1)) return st;
    if (col < 0 || !w) return fail(CB_ERR_INVALID_ARG, "bad column or NULL w");
    if (int st = check_vec16(w, v_out)) return st;
    launch_store(V->format, *V, col, w, divisor, v_out, nonfinite_flag, nullptr, (hipStream_t)stream);
    CB_HIP(hipGetLastError());
    return CB_OK;
}

int cb_basis_load(const cb_basis* V, int32_t col, double* x, void* stream) {
    if (int st = check_basis(V, col + 1)) return st;
    if (col < 0 || !x) return fail(CB_ERR_INVALID_ARG, "bad column or NULL x");
    if (int st = check_vec16(x)) return st;
    launch_load(V->format, *V, col, x, (hipStream_t)stream);
    CB_HIP(hipGetLastError());
    return CB_OK;
}

int64_t cb_reduce_workspace_bytes(int32_t n, int32_t ncols) {
    if (bad_n(n) || ncols < 0) return -1;
    return reduce_workspace_bytes(n, ncols, 0);
}

int cb_cgs_project(const cb_basis* V, int32_t j, const double* w, double* h, void* work,
                   size_t work_bytes, void* stream) {
    if (int st = check_basis(V, j)) return st;
    if (j < 1 || !w || !h || !work) return fail(CB_ERR_INVALID_ARG, "bad j or NULL pointer");
    if (int st = check_vec16(w)) return st;
    if (j > kMaxRestart + 1)
        return fail(CB_ERR_INVALID_ARG, "j=%d columns exceeds the limit of %d", j, kMaxRestart + 1);
    if ((int64_t)work_bytes < reduce_workspace_bytes(V->n, j, 0))
        return fail(CB_ERR_WORKSPACE, "workspace %zu < %lld bytes", work_bytes,
                    (long long)reduce_workspace_bytes(V->n, j, 0));
    hipStream_t s = (hipStream_t)stream;
    launch_zero_counter(static_cast<unsigned*>(work), s);
    launch_project(V->format, *V, j, w, partials_of(work), nullptr, store_epi(h, work), s);
    CB_HIP(hipGetLastError());
    return CB_OK;
}

int64_t cb_cgs_project_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

int cb_cgs_project_noalloc(const cb_basis* V, int32_t j, const double* w, double* h, void* stream) {
    if (int st = check_basis(V, j)) return st;
    if (j < 1 || !w || !h) return fail(CB_ERR_INVALID_ARG, "bad j or NULL pointer");
    if (int st = check_vec16(w)) return st;
    if (j > kMaxRestart + 1)
        return fail(CB_ERR_INVALID_ARG, "j=%d columns exceeds the limit of %d", j, kMaxRestart + 1);
    // the projection writes dot_groups(n) partials per column after the counters
    const int64_t need = kCounterBytes + 8 * (int64_t)dot_groups(V->n) * j;
    if (need > kNoAllocScratchBytes)
        return fail(CB_ERR_WORKSPACE, "n=%d, j=%d needs %lld bytes of scratch, more than the fixed %lld",
                    V->n, j, (long long)need, (long long)kNoAllocScratchBytes);
    void* ws = scratch_on_current_device();
    if (!ws) return CB_ERR_HIP;
    hipStream_t s = (hipStream_t)stream;
    launch_zero_counter(static_cast<unsigned*>(ws), s);  // a fill kernel, no memset node
    launch_project(V->format, *V, j, w, partials_of(ws), nullptr, store_epi(h, ws), s);
    CB_HIP(hipGetLastError());
    return CB_OK;
}

int cb_cgs_subtract(const cb_basis* V, int32_t j, const double* h, double* w, double* norm2,
                    void* work, size_t work_bytes, void* stream) {
    if (int st = check_basis(V, j)) return st;
    if (j < 1 || !w || !h) return fail(CB_ERR_INVALID_ARG, "bad j or NULL pointer");
    if (int st = check_vec16(w)) return st;
    if (j > kMaxRestart + 1)
        return fail(CB_ERR_INVALID_ARG, "j=%d columns exceeds the limit of %d", j, kMaxRestart + 1);
    if (norm2 && (!work || (int64_t)work_bytes < reduce_workspace_bytes(V->n, 1, 0)))
        return fail(CB_ERR_WORKSPACE, "norm needs a workspace of %lld bytes",
                    (long long)reduce_workspace_bytes(V->n, 1, 0));
    hipStream_t s = (hipStream_t)stream;
    if (norm2) launch_zero_counter(static_cast<unsigned*>(work), s);
    launch_subtract(V->format, *V, j, nullptr, h, w, norm2 ? partials_of(work) : nullptr, nullptr, -1,
                    store_epi(norm2, work), s);
    CB_HIP(hipGetLastError());
    return CB_OK;
}

int cb_cgs_subtract_project(const cb_basis* V, int32_t j, const double* h, double* w, double* out,
                            void* work, size_t work_bytes, void* stream) {
    if (int st = check_basis(V, j)) return st;
    if (j < 1 || !w || !h || !out || !work) return fail(CB_ERR_INVALID_ARG, "bad j or NULL pointer");
    if (int st = check_vec16(w)) return st;
    if (j > kMaxRestart)
        return fail(CB_ERR_INVALID_ARG, "j=%d columns exceeds the limit of %d", j, kMaxRestart);
    if ((int64_t)work_bytes < reduce_workspace_bytes(V->n, j + 1, 0))
        return fail(CB_ERR_WORKSPACE, "workspace %zu < %lld bytes", work_bytes,
                    (long long)reduce_workspace_bytes(V->n, j + 1, 0));
    hipStream_t s = (hipStream_t)stream;
    launch_zero_counter(static_cast<unsigned*>(work), s);
    launch_subtract_project(V->format, *V, j, h, w, partials_of(work), nullptr, store_epi(out, work), s);
    CB_HIP(hipGetLastError());
    return CB_OK;
}

int cb_basis_combine(const cb_basis* V, int32_t j, const double* y, double* x, void* stream) {
    if (int st = check_basis(V, j)) return st;
    if (j < 1 || !y || !x) return fail(CB_ERR_INVALID_ARG, "bad j or NULL pointer");
    if (int st = check_vec16(x)) return st;
    if (j > kMaxRestart + 1)
        return fail(CB_ERR_INVALID_ARG, "j=%d columns exceeds the limit of %d", j, kMaxRestart + 1);
    launch_subtract(V->format, *V, j, nullptr, y, x, nullptr, nullptr, +1, Epi{}, (hipStream_t)stream);
    CB_HIP(hipGetLastError());
    return CB_OK;
}

static int check_csr(const cb_csr* A) {
    if (!A) return fail(CB_ERR_INVALID_ARG, "matrix descriptor is NULL");
    if (bad_n(A->n) || A->nnz < 0) return fail(CB_ERR_INVALID_ARG, "bad matrix size n=%d nnz=%d", A->n, A->nnz);
    if (!A->row_ptr || (A->nnz > 0 && (!A->col || !A->val)))
        return fail(CB_ERR_INVALID_ARG, "NULL matrix array");
    return CB_OK;
}

// cb_spmv / cb_residual workspace: the norm's partial sums, then (rows of more
// than 8 entries on average) the column windows of the 512-row blocks.
static int64_t spmv_partials_bytes(const cb_csr* A) { return (8 * (int64_t)spmv_groups(A->n, A->nnz) + 255) & ~int64_t(255); }

int64_t cb_spmv_workspace_bytes(int32_t n, int32_t nnz) {
    if (bad_n(n) || nnz < 0) return -1;
    cb_csr A{n, nnz, nullptr, nullptr, nullptr};
    return spmv_partials_bytes(&A) + (spmv_uses_plan(n, nnz) ? spmv_plan_bytes(n) : 0);
}

static int spmv_common(const cb_csr* A, const double* x, const double* b, double* y, double* norm2, void* work,
                       size_t work_bytes, int mode, void* stream) {
    const int G = spmv_groups(A->n, A->nnz);
    const int64_t need = 8 * (int64_t)G;
    if (norm2 && (!work || (int64_t)work_bytes < need))
        return fail(CB_ERR_WORKSPACE, "norm needs a workspace of %lld bytes", (long long)need);
    hipStream_t s = (hipStream_t)stream;
    double* part = norm2 ? static_cast<double*>(work) : nullptr;
    void* plan = nullptr;
    if (work && spmv_uses_plan(A->n, A->nnz) &&
        (int64_t)work_bytes >= cb_spmv_workspace_bytes(A->n, A->nnz) && aligned(work, 8)) {
        plan = static_cast<unsigned char*>(work) + spmv_partials_bytes(A);
        launch_spmv_plan(*A, plan, s);
    }
    launch_spmv(*A, x, b, y, part, mode, nullptr, s, plan);
    if (norm2) launch_reduce(part, G, 1, norm2, 0, nullptr, s);
    CB_HIP(hipGetLastError());
    return CB_OK;
}

int cb_spmv(const cb_csr* A, const double* x, double* y, double* norm2, void* work,
            size_t work_bytes, void* stream) {
    if (int st = check_csr(A)) return st;
    if (!x || !y) return fail(CB_ERR_INVALID_ARG, "NULL vector");
    return spmv_common(A, x, nullptr, y, norm2, work, work_bytes, 0, stream);
}

int cb_residual(const cb_csr* A, const double* b, const double* x, double* r, double* norm2,
                void* work, size_t work_bytes, void* stream) {
    if (int st = check_csr(A)) return st;
    if (!x || !r || !b) return fail(CB_ERR_INVALID_ARG, "NULL vector");
    return spmv_common(A, x, b, r, norm2, work, work_bytes, 1, stream);
}

}  // extern "C"
