// Continuous-batching solve server on one GPU.
//
// Requests enter a queue.  A request is admitted when its device footprint
// (basis columns, CSR arrays, work vectors, reduction partials) fits in what
// is left of the HBM budget; admission is in arrival order within each kind.
//  * Large requests go to solve lanes (host worker threads, each with its own
//    HIP stream), one at a time per lane, through the multi-workgroup solver.
//  * Small requests go to a device-resident request loop: a persistent
//    launch of the one-workgroup solver (batch.hip, k_batch_ring) whose
//    workgroups take systems from a ring of descriptors while it runs.  The
//    ring thread admits small requests by budget, places each in a device
//    arena (its CSR, b, x and Krylov workspace stay on the GPU for the whole
//    solve, every restart included), stages its inputs in pinned host memory
//    and publishes its descriptor; a request that arrives while the launch
//    runs is picked up by the next free workgroup of that same launch.  The
//    ring thread collects finished systems from their done words and returns
//    their memory to the budget.  The launch leaves when it has been idle for
//    a while or has run for a time slice (streams sharing its hardware queue
//    then get their turn) and is started again while work is pending.
// Which path a request takes depends on its own shape only, and neither
// path's arithmetic depends on what runs beside it, so a result does not
// depend on the mix it ran in.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
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
    // device-resident loop for small requests (under mu)
    int64_t ring_published = 0, ring_joined = 0, ring_launches = 0;
    int ring_status = 0;  // CB_OK, or the error that disabled the ring

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace cb {

// Requests up to this size go to the device-resident loop of the one-workgroup
// solver.
constexpr int32_t kSmallN = 16384;
// The loop's launch: workgroups (systems solved at once), idle polls before a
// workgroup leaves (~8 us apart: ~20 ms), time slice, and the host staging
// memory for the small systems' inputs and outputs.
constexpr int kRingGrid = 128;
constexpr int kRingIdlePolls = 2500;
constexpr double kRingSlice = 0.05;
constexpr int64_t kStagingBytes = int64_t(256) << 20;
constexpr int64_t kRingArenaMax = int64_t(4) << 30;

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

// Under the lock: a request's end -- status, time, memory back to the budget,
// host copies of its inputs released.
static void finish(cb_server* S, Request& r, double t) {
    r.t_end = t;
    r.status = r.result.status == CB_PENDING ? CB_ERR_HIP : r.result.status;
    r.result.status = r.status;
    S->charged -= r.bytes;
    S->running -= 1;
    r.row_ptr.clear(); r.row_ptr.shrink_to_fit();
    r.col.clear(); r.col.shrink_to_fit();
    r.val.clear(); r.val.shrink_to_fit();
    r.b.clear(); r.b.shrink_to_fit();
}

// Under the lock: the requests a lane of this kind may take now (at most
// `limit`).
static std::vector<std::shared_ptr<Request>> take_work(cb_server* S, bool batch_lane, int limit) {
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
        if ((int)take.size() >= limit) break;
    }
    return take;
}

static bool has_kind(const cb_server* S, bool batch_lane) {
    for (const auto& r : S->queue)
        if (is_small(r->n, r->m, r->format) == batch_lane) return true;
    return false;
}

static void worker_main(cb_server* S) {
    (void)hipSetDevice(S->device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    const bool batch_lane = false;
    for (;;) {
        std::vector<std::shared_ptr<Request>> take;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                take = take_work(S, batch_lane, 1);
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
        int st = run_request(*take[0], s);
        if (st == CB_PENDING) st = CB_ERR_HIP;
        take[0]->result.status = st;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            finish(S, *take[0], S->now());
        }
        S->cv.notify_all();
    }
    (void)hipStreamDestroy(s);
}

// ----------------------------------------------------------------- the device-resident loop
// First fit over [0, size) in 256-byte units, neighbours merged on release.
class Arena {
  public:
    void init(int64_t size) {
        free_.clear();
        if (size > 0) free_[0] = size;
    }
    int64_t alloc(int64_t bytes) {
        bytes = al256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const int64_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            return off;
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes) {
        bytes = al256(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && off + bytes == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<int64_t, int64_t> free_;
};

// Host staging of one small system: inputs, then the output x.
struct Staged {
    int64_t rp, ci, va, b, x0, x, total;
};
static Staged stage_layout(const Request& r) {
    Staged t;
    t.rp = 0;
    t.ci = al256((int64_t)(r.n + 1) * 4);
    t.va = t.ci + al256((int64_t)r.nnz * 4);
    t.b = t.va + al256((int64_t)r.nnz * 8);
    t.x0 = t.b + al256((int64_t)r.n * 8);
    t.x = t.x0 + al256((int64_t)r.n * 8);
    t.total = t.x + al256((int64_t)r.n * 8);
    return t;
}

struct InFlight {
    std::shared_ptr<Request> r;
    uint32_t seq;
    int64_t doff, dbytes, soff;
    Staged st;
    uint32_t launch_at_publish;  // the launch running when it was published (0: none)
};

static void fail_all_small(cb_server* S, int status) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->ring_status = status;
}

static void ring_main(cb_server* S) {
    (void)hipSetDevice(S->device);
    hipStream_t ks = nullptr;
    BatchRing* ring = nullptr;
    unsigned char* dev = nullptr;
    unsigned char* stg = nullptr;
    unsigned char* stg_dev = nullptr;
    const int64_t arena_bytes = std::min<int64_t>((int64_t)S->budget, kRingArenaMax);
    if (hipStreamCreateWithFlags(&ks, hipStreamNonBlocking) != hipSuccess ||
        !(ring = ring_create(kRingGrid, kRingIdlePolls, kRingSlice)) ||
        hipMalloc(reinterpret_cast<void**>(&dev), (size_t)arena_bytes) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&stg), (size_t)kStagingBytes,
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer(reinterpret_cast<void**>(&stg_dev), stg, 0) != hipSuccess) {
        fail_all_small(S, CB_ERR_HIP);
    }
    Arena darena, sarena;
    darena.init(arena_bytes);
    sarena.init(kStagingBytes);
    std::deque<InFlight> fl;
    uint32_t cur_launch = 0;
    for (;;) {
        bool progressed = false;
        // finished systems: results back to their requests, memory to the budget
        for (auto it = fl.begin(); it != fl.end();) {
            cb_result res;
            uint32_t launch = 0;
            if (!ring_poll(ring, it->seq, &res, &launch)) {
                ++it;
                continue;
            }
            Request& r = *it->r;
            std::memcpy(r.x.data(), stg + it->soff + it->st.x, (size_t)r.n * 8);
            r.result = res;
            darena.release(it->doff, it->dbytes);
            sarena.release(it->soff, it->st.total);
            {
                std::lock_guard<std::mutex> lk(S->mu);
                if (it->launch_at_publish && launch == it->launch_at_publish) S->ring_joined += 1;
                finish(S, r, S->now());
            }
            S->cv.notify_all();
            it = fl.erase(it);
            progressed = true;
        }
        // admission by budget, in arrival order
        std::vector<std::shared_ptr<Request>> take;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stopping && !has_kind(S, true) && fl.empty()) break;
            if (S->ring_status != CB_OK) {
                // the loop could not be set up: fail the small requests
                take = take_work(S, true, 1 << 30);
                const double t = S->now();
                for (auto& r : take) {
                    r->t_start = t;
                    r->result = cb_result{};
                    r->result.status = S->ring_status;
                    S->charged += r->bytes;
                    S->running += 1;
                    finish(S, *r, t);
                }
                take.clear();
            } else {
                take = take_work(S, true, kRingSlots - (int)fl.size());
                const double t = S->now();
                for (auto& r : take) {
                    S->charged += r->bytes;
                    r->t_start = t;
                }
                S->running += (int)take.size();
            }
        }
        for (size_t i = 0; i < take.size(); ++i) {
            auto& rp = take[i];
            Request& r = *rp;
            const int64_t ws = batch_workspace_bytes(r.n, r.m, r.format);
            const Placed p = place(r, ws);
            const Staged st = stage_layout(r);
            const int64_t doff = darena.alloc(p.total);
            const int64_t soff = doff < 0 ? -1 : sarena.alloc(st.total);
            if (doff < 0 || soff < 0) {
                // fragmented: back to the front of the queue until memory frees up
                if (doff >= 0) darena.release(doff, p.total);
                std::lock_guard<std::mutex> lk(S->mu);
                for (size_t k = take.size(); k-- > i;) {
                    S->charged -= take[k]->bytes;
                    S->running -= 1;
                    S->queue.push_front(take[k]);
                }
                break;
            }
            unsigned char* h = stg + soff;
            std::memcpy(h + st.rp, r.row_ptr.data(), (size_t)(r.n + 1) * 4);
            if (r.nnz) {
                std::memcpy(h + st.ci, r.col.data(), (size_t)r.nnz * 4);
                std::memcpy(h + st.va, r.val.data(), (size_t)r.nnz * 8);
            }
            std::memcpy(h + st.b, r.b.data(), (size_t)r.n * 8);
            std::memcpy(h + st.x0, r.x.data(), (size_t)r.n * 8);
            unsigned char* m = dev + doff;
            unsigned char* hd = stg_dev + soff;
            cb_batch_item q;
            q.A = csr_at(r, m, p);
            q.b = reinterpret_cast<double*>(m + p.b);
            q.x = reinterpret_cast<double*>(m + p.x);
            q.workspace = m + p.ws;
            q.workspace_bytes = (size_t)(p.total - p.ws);
            q.m = r.m;
            q.format = r.format;
            q.tol = r.tol;
            uint32_t seq = 0;
            const int pst = ring_publish(ring, q, reinterpret_cast<const int32_t*>(hd + st.rp),
                                         reinterpret_cast<const int32_t*>(hd + st.ci),
                                         reinterpret_cast<const double*>(hd + st.va),
                                         reinterpret_cast<const double*>(hd + st.b),
                                         reinterpret_cast<const double*>(hd + st.x0),
                                         reinterpret_cast<double*>(hd + st.x), &seq);
            if (pst != CB_OK) {
                darena.release(doff, p.total);
                sarena.release(soff, st.total);
                r.result = cb_result{};
                r.result.status = pst;
                std::lock_guard<std::mutex> lk(S->mu);
                finish(S, r, S->now());
                continue;
            }
            const uint32_t running_launch = ring_running(ring) ? cur_launch : 0;
            fl.push_back(InFlight{rp, seq, doff, p.total, soff, st, running_launch});
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->ring_published += 1;
            }
            progressed = true;
        }
        // a launch while systems wait (a finished launch may have left some
        // unclaimed; a fresh one with nothing to take leaves when idle)
        if (!fl.empty() && !ring_running(ring)) {
            int kst = CB_OK;
            const uint32_t id = ring_kick(ring, ks, &kst);
            if (id) {
                cur_launch = id;
                std::lock_guard<std::mutex> lk(S->mu);
                S->ring_launches += 1;
            }
            if (kst != CB_OK) fail_all_small(S, kst);
        }
        if (!progressed) {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait_for(lk, std::chrono::microseconds(fl.empty() ? 2000 : 100));
        }
    }
    if (ring) ring_destroy(ring);  // sets stop and waits for the launch
    if (dev) (void)hipFree(dev);
    if (stg) (void)hipHostFree(stg);
    if (ks) (void)hipStreamDestroy(ks);
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
    for (int i = 0; i < lanes; ++i) S->workers.emplace_back(worker_main, S);
    S->workers.emplace_back(ring_main, S);
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

int cb_server_ring_stats(cb_server* S, int64_t* published, int64_t* joined_running, int64_t* launches) {
    if (!S) return fail(CB_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    if (published) *published = S->ring_published;
    if (joined_running) *joined_running = S->ring_joined;
    if (launches) *launches = S->ring_launches;
    return S->ring_status;
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
