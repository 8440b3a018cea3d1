// Continuous-batching solve server on one GPU.
//
// Requests enter a FIFO queue.  A request is admitted when its device
// footprint (basis columns, CSR arrays, work vectors, reduction partials) fits
// in what is left of the HBM budget; admitted requests run concurrently, one
// per lane, each lane a host worker thread with its own HIP stream, so solves
// of different sizes overlap on the device.  When a solve ends its memory is
// returned to the budget and the next queued requests are admitted.  Each
// solve calls the same solver entry point (and so the same kernels with the
// same reduction order) as a stand-alone cbgmres_solve, so a result does not
// depend on the mix it ran in.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cb_internal.hpp"

namespace cb {

struct Request {
    uint64_t ticket;
    int32_t n, nnz, m, format;
    double tol;
    std::vector<int32_t> row_ptr, col;
    std::vector<double> val, b, x;
    int64_t bytes;
    double t_submit = 0, t_start = 0, t_end = 0;
    int status = CB_PENDING;
    cb_result result{};
};

}  // namespace cb

struct cb_server {
    size_t budget;
    int device;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<cb::Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<cb::Request>> all;
    int64_t charged = 0;
    int running = 0;
    bool stopping = false;
    uint64_t next_ticket = 1;
    std::vector<std::thread> workers;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace cb {

static int64_t request_bytes(int32_t n, int32_t nnz, int32_t m, int format) {
    int64_t ws = cbgmres_workspace_bytes(n, m, format);
    if (ws < 0) return -1;
    // CSR + b + x on the device, plus the solver workspace
    return ws + (int64_t)(n + 1) * 4 + (int64_t)nnz * 12 + 2 * padded_rows(n) * 8 + 4096;
}

static int run_request(Request& r, hipStream_t s) {
    const int n = r.n;
    unsigned char* mem = nullptr;
    const int64_t ws = cbgmres_workspace_bytes(n, r.m, r.format);
    auto al = [](int64_t x) { return (x + 255) & ~int64_t(255); };
    const int64_t o_rp = 0;
    const int64_t o_ci = o_rp + al((int64_t)(n + 1) * 4);
    const int64_t o_va = o_ci + al((int64_t)r.nnz * 4);
    const int64_t o_b = o_va + al((int64_t)r.nnz * 8);
    const int64_t o_x = o_b + al((int64_t)n * 8);
    const int64_t o_ws = o_x + al((int64_t)n * 8);
    const int64_t total = o_ws + ws;
    if (hipMallocAsync(reinterpret_cast<void**>(&mem), (size_t)total, s) != hipSuccess)
        return fail(CB_ERR_HIP, "device allocation of %lld bytes failed", (long long)total);
    int st = CB_OK;
    if (hipMemcpyAsync(mem + o_rp, r.row_ptr.data(), (size_t)(n + 1) * 4, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(mem + o_ci, r.col.data(), (size_t)r.nnz * 4, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(mem + o_va, r.val.data(), (size_t)r.nnz * 8, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(mem + o_b, r.b.data(), (size_t)n * 8, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(mem + o_x, r.x.data(), (size_t)n * 8, hipMemcpyHostToDevice, s)) {
        st = fail(CB_ERR_HIP, "input copy failed");
    } else {
        cb_csr A{n, r.nnz, reinterpret_cast<int32_t*>(mem + o_rp), reinterpret_cast<int32_t*>(mem + o_ci),
                 reinterpret_cast<double*>(mem + o_va)};
        st = cbgmres_solve(&A, reinterpret_cast<double*>(mem + o_b), reinterpret_cast<double*>(mem + o_x),
                           r.m, r.tol, r.format, nullptr, mem + o_ws, (size_t)ws, nullptr, 0, &r.result, s);
        if (hipMemcpyAsync(r.x.data(), mem + o_x, (size_t)n * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
            st = fail(CB_ERR_HIP, "result copy failed");
    }
    (void)hipFreeAsync(mem, s);
    (void)hipStreamSynchronize(s);
    return st;
}

static void worker_main(cb_server* S) {
    (void)hipSetDevice(S->device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
        std::shared_ptr<Request> r;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // FIFO admission: the head of the queue runs once it fits
            S->cv.wait(lk, [&] {
                return S->stopping ||
                       (!S->queue.empty() && S->charged + S->queue.front()->bytes <= (int64_t)S->budget);
            });
            if (S->queue.empty()) {
                if (S->stopping) break;
                continue;
            }
            if (S->charged + S->queue.front()->bytes > (int64_t)S->budget) continue;
            r = S->queue.front();
            S->queue.pop_front();
            S->charged += r->bytes;
            S->running += 1;
            r->t_start = S->now();
        }
        int st = run_request(*r, s);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            r->t_end = S->now();
            r->status = st == CB_PENDING ? CB_ERR_HIP : st;
            r->result.status = r->status;
            S->charged -= r->bytes;
            S->running -= 1;
            r->row_ptr.clear(); r->row_ptr.shrink_to_fit();
            r->col.clear(); r->col.shrink_to_fit();
            r->val.clear(); r->val.shrink_to_fit();
            r->b.clear(); r->b.shrink_to_fit();
        }
        S->cv.notify_all();
    }
    (void)hipStreamDestroy(s);
}

}  // namespace cb

using namespace cb;

extern "C" {

int64_t cb_server_request_bytes(int32_t n, int32_t nnz, int32_t m, int format) {
    if (n < 1 || nnz < 0 || m < 1 || !valid_format(format)) return -1;
    return request_bytes(n, nnz, m, format);
}

cb_server* cb_server_create(size_t hbm_budget_bytes, int device, int lanes) {
    if (lanes < 1 || lanes > 64) {
        set_error("lanes=%d out of range [1, 64]", lanes);
        return nullptr;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        set_error("device %d not available", device);
        return nullptr;
    }
    cb_server* S = new cb_server();
    S->budget = hbm_budget_bytes;
    S->device = device;
    S->t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < lanes; ++i) S->workers.emplace_back(worker_main, S);
    return S;
}

int cb_server_submit(cb_server* S, int32_t n, int32_t nnz, const int32_t* row_ptr_host,
                     const int32_t* col_host, const double* val_host, const double* b_host,
                     const double* x0_host, int32_t m, double tol, int format, uint64_t* ticket) {
    if (!S || !row_ptr_host || !b_host || !ticket || (nnz > 0 && (!col_host || !val_host)))
        return fail(CB_ERR_INVALID_ARG, "NULL argument");
    if (n < 1 || nnz < 0 || m < 1 || m > kMaxRestart || !(tol > 0) || !valid_format(format))
        return fail(CB_ERR_INVALID_ARG, "bad request shape");
    const int64_t bytes = request_bytes(n, nnz, m, format);
    if (bytes > (int64_t)S->budget)
        return fail(CB_ERR_OVER_BUDGET, "request needs %lld bytes, budget %zu", (long long)bytes, S->budget);
    auto r = std::make_shared<Request>();
    r->n = n; r->nnz = nnz; r->m = m; r->format = format; r->tol = tol; r->bytes = bytes;
    r->row_ptr.assign(row_ptr_host, row_ptr_host + n + 1);
    r->col.assign(col_host, col_host + nnz);
    r->val.assign(val_host, val_host + nnz);
    r->b.assign(b_host, b_host + n);
    if (x0_host) r->x.assign(x0_host, x0_host + n);
    else r->x.assign((size_t)n, 0.0);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        r->ticket = S->next_ticket++;
        r->t_submit = S->now();
        S->queue.push_back(r);
        S->all[r->ticket] = r;
        *ticket = r->ticket;
    }
    S->cv.notify_all();
    return CB_OK;
}

int cb_server_poll(cb_server* S, uint64_t ticket, double* x_host, cb_result* result_host,
                   double* times_host) {
    if (!S) return fail(CB_ERR_INVALID_ARG, "NULL server");
    std::shared_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(ticket);
        if (it == S->all.end()) return fail(CB_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
        r = it->second;
        if (r->status == CB_PENDING) return CB_PENDING;
        S->all.erase(it);
    }
    if (x_host) std::memcpy(x_host, r->x.data(), (size_t)r->n * 8);
    if (result_host) *result_host = r->result;
    if (times_host) {
        times_host[0] = r->t_submit;
        times_host[1] = r->t_start;
        times_host[2] = r->t_end;
    }
    return r->status;
}

int cb_server_stats(cb_server* S, int64_t* charged_bytes, int32_t* queued, int32_t* running) {
    if (!S) return fail(CB_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    if (charged_bytes) *charged_bytes = S->charged;
    if (queued) *queued = (int32_t)S->queue.size();
    if (running) *running = S->running;
    return CB_OK;
}

void cb_server_destroy(cb_server* S) {
    if (!S) return;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv.wait(lk, [&] { return S->queue.empty() && S->running == 0; });
        S->stopping = true;
    }
    S->cv.notify_all();
    for (auto& t : S->workers) t.join();
    delete S;
}

}  // extern "C"
