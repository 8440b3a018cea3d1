// Continuous-batching solve server on one GPU.
//
// Requests enter a queue.  A request is admitted when its device footprint
// (basis columns, CSR arrays, work vectors, reduction partials) fits in what
// is left of the HBM budget.  Two kinds of lanes (host worker threads, each
// with its own HIP stream) take admitted requests, so solves overlap on the
// device:
//  * solve lanes take large requests in arrival order, one at a time, and run
//    the multi-workgroup solver on them;
//  * batch lanes take every small request waiting (in arrival order, up to
//    kMaxBatch, as far as the budget allows) and solve them in ONE persistent
//    launch of the one-workgroup batched solver; small requests that arrive
//    meanwhile are picked up by the next free batch lane.
// Small requests never wait behind large ones for a lane (they use a few CUs
// each).  When a solve ends its memory is returned to the budget and waiting
// requests are admitted while the other lanes keep running.  Which path a
// request takes depends on its own shape only, and neither path's arithmetic
// depends on what runs beside it, so a result does not depend on the mix it
// ran in.
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

// Requests up to this size go to the batched one-workgroup solver.
constexpr int32_t kSmallN = 16384;
constexpr int kMaxBatch = 512;
constexpr int kBatchLanes = 2;

// The batched solver runs the block-32 fixed formats only; other FRSZ2
// requests go to the solve lanes whatever their size.
static bool is_small(int32_t n, int32_t m, int format) {
    return n <= kSmallN && m <= kBatchMaxRestart && batch_format(format);
}

static int64_t al256(int64_t x) { return (x + 255) & ~int64_t(255); }

static int64_t request_bytes(int32_t n, int32_t nnz, int32_t m, int format) {
    int64_t ws = is_small(n, m, format) ? batch_workspace_bytes(n, m, format) : cbgmres_workspace_bytes(n, m, format);
    if (ws < 0) return -1;
    // CSR + b + x on the device, plus the solver workspace
    return ws + al256((int64_t)(n + 1) * 4) + al256((int64_t)nnz * 4) + al256((int64_t)nnz * 8) +
           2 * al256((int64_t)n * 8) + 4096;
}

// Device copies of a request's inputs inside one allocation, workspace last.
struct Placed {
    int64_t rp, ci, va, b, x, ws, total;
};
static Placed place(const Request& r, int64_t ws_bytes) {
    Placed p;
    p.rp = 0;
    p.ci = p.rp + al256((int64_t)(r.n + 1) * 4);
    p.va = p.ci + al256((int64_t)r.nnz * 4);
    p.b = p.va + al256((int64_t)r.nnz * 8);
    p.x = p.b + al256((int64_t)r.n * 8);
    p.ws = p.x + al256((int64_t)r.n * 8);
    p.total = p.ws + al256(ws_bytes);
    return p;
}
static bool upload(const Request& r, unsigned char* mem, const Placed& p, hipStream_t s) {
    return hipMemcpyAsync(mem + p.rp, r.row_ptr.data(), (size_t)(r.n + 1) * 4, hipMemcpyHostToDevice, s) ==
               hipSuccess &&
           (r.nnz == 0 ||
            (hipMemcpyAsync(mem + p.ci, r.col.data(), (size_t)r.nnz * 4, hipMemcpyHostToDevice, s) ==
                 hipSuccess &&
             hipMemcpyAsync(mem + p.va, r.val.data(), (size_t)r.nnz * 8, hipMemcpyHostToDevice, s) ==
                 hipSuccess)) &&
           hipMemcpyAsync(mem + p.b, r.b.data(), (size_t)r.n * 8, hipMemcpyHostToDevice, s) == hipSuccess &&
           hipMemcpyAsync(mem + p.x, r.x.data(), (size_t)r.n * 8, hipMemcpyHostToDevice, s) == hipSuccess;
}
static cb_csr csr_at(const Request& r, unsigned char* mem, const Placed& p) {
    return cb_csr{r.n, r.nnz, reinterpret_cast<int32_t*>(mem + p.rp), reinterpret_cast<int32_t*>(mem + p.ci),
                  reinterpret_cast<double*>(mem + p.va)};
}

static int run_request(Request& r, hipStream_t s) {
    const int64_t ws = cbgmres_workspace_bytes(r.n, r.m, r.format);
    const Placed p = place(r, ws);
    unsigned char* mem = nullptr;
    if (hipMallocAsync(reinterpret_cast<void**>(&mem), (size_t)p.total, s) != hipSuccess)
        return fail(CB_ERR_HIP, "device allocation of %lld bytes failed", (long long)p.total);
    int st = CB_OK;
    if (!upload(r, mem, p, s)) {
        st = fail(CB_ERR_HIP, "input copy failed");
    } else {
        const cb_csr A = csr_at(r, mem, p);
        st = cbgmres_solve(&A, reinterpret_cast<double*>(mem + p.b), reinterpret_cast<double*>(mem + p.x),
                           r.m, r.tol, r.format, nullptr, mem + p.ws, (size_t)ws, nullptr, 0, &r.result, s);
        if (hipMemcpyAsync(r.x.data(), mem + p.x, (size_t)r.n * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
            st = fail(CB_ERR_HIP, "result copy failed");
    }
    (void)hipFreeAsync(mem, s);
    (void)hipStreamSynchronize(s);
    return st;
}

// Small requests: one allocation for all of them, one batched launch.
// Statuses land in each request's result.
static int run_batch(std::vector<std::shared_ptr<Request>>& rs, hipStream_t s) {
    const int count = (int)rs.size();
    std::vector<Placed> ps(count);
    std::vector<int64_t> base(count);
    int64_t total = 0;
    for (int i = 0; i < count; ++i) {
        ps[i] = place(*rs[i], batch_workspace_bytes(rs[i]->n, rs[i]->m, rs[i]->format));
        base[i] = total;
        total += ps[i].total;
    }
    unsigned char* mem = nullptr;
    if (hipMallocAsync(reinterpret_cast<void**>(&mem), (size_t)total, s) != hipSuccess)
        return fail(CB_ERR_HIP, "device allocation of %lld bytes failed", (long long)total);
    int st = CB_OK;
    std::vector<cb_batch_item> items(count);
    std::vector<cb_result> res(count);
    for (int i = 0; i < count && st == CB_OK; ++i) {
        const Request& r = *rs[i];
        unsigned char* m = mem + base[i];
        if (!upload(r, m, ps[i], s)) {
            st = fail(CB_ERR_HIP, "input copy failed");
            break;
        }
        items[i].A = csr_at(r, m, ps[i]);
        items[i].b = reinterpret_cast<double*>(m + ps[i].b);
        items[i].x = reinterpret_cast<double*>(m + ps[i].x);
        items[i].workspace = m + ps[i].ws;
        items[i].workspace_bytes = (size_t)(ps[i].total - ps[i].ws);
        items[i].m = r.m;
        items[i].format = r.format;
        items[i].tol = r.tol;
    }
    if (st == CB_OK) {
        const int bst = cbgmres_solve_batch(items.data(), count, nullptr, res.data(), s);
        if (bst == CB_ERR_HIP || bst == CB_ERR_INVALID_ARG || bst == CB_ERR_WORKSPACE) st = bst;
    }
    for (int i = 0; i < count && st == CB_OK; ++i)
        if (hipMemcpyAsync(rs[i]->x.data(), mem + base[i] + ps[i].x, (size_t)rs[i]->n * 8,
                           hipMemcpyDeviceToHost, s) != hipSuccess)
            st = fail(CB_ERR_HIP, "result copy failed");
    (void)hipFreeAsync(mem, s);
    (void)hipStreamSynchronize(s);
    for (int i = 0; i < count; ++i) {
        rs[i]->result = st == CB_OK ? res[i] : cb_result{};
        rs[i]->result.status = st == CB_OK ? res[i].status : st;
    }
    return st;
}

// Under the lock: the requests a lane of this kind may take now.
static std::vector<std::shared_ptr<Request>> take_work(cb_server* S, bool batch_lane) {
    std::vector<std::shared_ptr<Request>> take;
    int64_t charged = S->charged;
    for (auto it = S->queue.begin(); it != S->queue.end();) {
        const bool small = is_small((*it)->n, (*it)->m, (*it)->format);
        if (small != batch_lane) {
            ++it;
            continue;
        }
        // arrival order within the kind: stop at the first that does not fit
        if (charged + (*it)->bytes > (int64_t)S->budget) break;
        charged += (*it)->bytes;
        take.push_back(*it);
        it = S->queue.erase(it);
        if ((int)take.size() >= (batch_lane ? kMaxBatch : 1)) break;
    }
    return take;
}

static bool has_kind(const cb_server* S, bool batch_lane) {
    for (const auto& r : S->queue)
        if (is_small(r->n, r->m, r->format) == batch_lane) return true;
    return false;
}

static void worker_main(cb_server* S, bool batch_lane) {
    (void)hipSetDevice(S->device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
        std::vector<std::shared_ptr<Request>> take;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                take = take_work(S, batch_lane);
                if (!take.empty()) break;
                if (S->stopping && !has_kind(S, batch_lane)) break;
                S->cv.wait(lk);
            }
            if (take.empty()) break;
            const double t = S->now();
            for (auto& r : take) {
                S->charged += r->bytes;
                r->t_start = t;
            }
            S->running += (int)take.size();
        }
        if (!batch_lane) {
            int st = run_request(*take[0], s);
            if (st == CB_PENDING) st = CB_ERR_HIP;
            take[0]->result.status = st;
        } else {
            run_batch(take, s);
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            const double t = S->now();
            for (auto& r : take) {
                r->t_end = t;
                r->status = r->result.status == CB_PENDING ? CB_ERR_HIP : r->result.status;
                r->result.status = r->status;
                S->charged -= r->bytes;
                S->running -= 1;
                r->row_ptr.clear(); r->row_ptr.shrink_to_fit();
                r->col.clear(); r->col.shrink_to_fit();
                r->val.clear(); r->val.shrink_to_fit();
                r->b.clear(); r->b.shrink_to_fit();
            }
        }
        S->cv.notify_all();
    }
    (void)hipStreamDestroy(s);
}

}  // namespace cb

using namespace cb;

extern "C" {

int64_t cb_server_request_bytes(int32_t n, int32_t nnz, int32_t m, int format) {
    if (n < 1 || n > kMaxRows || nnz < 0 || m < 1 || !valid_format(format)) return -1;
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
    for (int i = 0; i < lanes; ++i) S->workers.emplace_back(worker_main, S, false);
    for (int i = 0; i < kBatchLanes; ++i) S->workers.emplace_back(worker_main, S, true);
    return S;
}

int cb_server_submit(cb_server* S, int32_t n, int32_t nnz, const int32_t* row_ptr_host,
                     const int32_t* col_host, const double* val_host, const double* b_host,
                     const double* x0_host, int32_t m, double tol, int format, uint64_t* ticket) {
    if (!S || !row_ptr_host || !b_host || !ticket || (nnz > 0 && (!col_host || !val_host)))
        return fail(CB_ERR_INVALID_ARG, "NULL argument");
    if (n < 1 || n > kMaxRows || nnz < 0 || m < 1 || m > kMaxRestart || !(tol > 0) || !valid_format(format))
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
