// Serving runtime behind octmc_server_* (include/octmc.h): registration
// requests of mixed sizes solved concurrently on one device.
//
//   admission  requests wait in arrival order; the head is admitted when a
//              worker is free and its footprint fits into the server's device
//              range (first fit over the free ranges, coalesced on release);
//              the request's pyramid, solver state and scratch all live in
//              that one slab until it completes
//   workers    one host thread, stream and set of pinned scalars per active
//              request, running the full solve (pair ingest, level loop,
//              merge)
//   batcher    (grouped mode) collects the evaluations the workers are
//              waiting for and runs each set of up to kMaxJobs as one launch
//              per kernel, every job at its own level and size; sets
//              alternate between two streams, and the next set forms while
//              up to two run on the device.  Evaluations large enough to fill
//              the device alone run on their request's stream instead.
//
// The solver of a request is the same code as octmc_register's and every
// reduction runs in a fixed order per job, so a request's result does not
// depend on what else is active.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "octmc_internal.h"

using namespace octmc;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over offsets of one device range.  Sizes are multiples
// of 256 bytes, so every range handed out stays 256-byte aligned.
class Arena {
public:
    void reset(size_t size)
    {
        free_.clear();
        free_[0] = size;
    }
    bool take(size_t bytes, size_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, next = it->first + bytes;
            free_.erase(it);
            if (rest) free_[next] = rest;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
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
    std::map<size_t, size_t> free_;  // offset -> length
};

struct Job {
    uint64_t id = 0;
    octmc_request req{};
    size_t footprint = 0;
    double t_submit = 0;
};

// One evaluation handed from a worker to the batcher.
struct Ticket {
    EvalArgs ea{};
    hipEvent_t ready = nullptr;  // recorded on the worker's stream: the inputs are ready
    hipEvent_t done = nullptr;   // recorded on the batcher's stream after the grouped launch
    bool launched = false;
    int rc = OCTMC_OK;
    std::string err;
};

struct Worker {
    hipStream_t s = nullptr;
    double* h_terms = nullptr;
    double* h_dots = nullptr;
    hipEvent_t ready = nullptr, done = nullptr;
    Ticket ticket;
    std::thread th;
};

struct DirectEval final : Evaluator {
    int eval(const EvalArgs& ea, hipStream_t s) override { return eval_group(&ea, 1, s); }
    bool enqueue_only() const override { return true; }
};

}  // namespace

struct octmc_server {
    octmc_ctx* ctx = nullptr;
    int device = 0;
    int mode = OCTMC_SERVE_GROUPED;
    int max_active = 1;
    char* base = nullptr;
    size_t budget = 0;
    Arena arena;
    Clock::time_point start;

    std::mutex mu;
    std::condition_variable cv_admit, cv_done, cv_batch, cv_ticket;
    std::deque<Job> queue;
    std::deque<octmc_completion> done;
    int active = 0;
    uint64_t next_id = 1;
    bool stop = false, stop_batcher = false;

    std::vector<Worker*> workers;
    std::vector<Ticket*> pending;
    std::thread batcher;
    hipStream_t bs[2] = {nullptr, nullptr};  // grouped launches alternate between two streams
    hipEvent_t last[2] = {nullptr, nullptr};

    double now() const { return std::chrono::duration<double>(Clock::now() - start).count(); }
};

namespace {

// Evaluations of at least this many A-scans fill the device with one launch
// per kernel (one wave per output A-scan, about 3 000 resident waves), so
// grouping them with others saves nothing and only makes the request wait for
// the batcher: they run directly on the request's stream.  Smaller ones (the
// coarse pyramid levels) are grouped, where one launch replaces several
// nearly empty ones.
constexpr int kGroupMaxAscans = 128 * 128;

struct GroupEval final : Evaluator {
    octmc_server* S;
    Worker* W;
    GroupEval(octmc_server* s, Worker* w) : S(s), W(w) {}
    int eval(const EvalArgs& ea, hipStream_t s) override
    {
        if (ea.pair && pair_level_ascans(ea.pair, ea.level) >= kGroupMaxAscans) return eval_group(&ea, 1, s);
        HIP_TRY(hipEventRecord(W->ready, s));
        Ticket& t = W->ticket;
        t.ea = ea;
        t.ready = W->ready;
        t.done = W->done;
        t.launched = false;
        t.rc = OCTMC_OK;
        t.err.clear();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->pending.push_back(&t);
        }
        S->cv_batch.notify_one();
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_ticket.wait(lk, [&] { return t.launched; });
        }
        // the worker's stream waits for the set in every case, so that a
        // synchronisation of that stream covers the batcher's work too
        const hipError_t we = hipStreamWaitEvent(s, W->done, 0);
        if (t.rc != OCTMC_OK) return fail(t.rc, t.err);
        HIP_TRY(we);
        return OCTMC_OK;
    }
};

// Launch one set of waiting evaluations (one storage type, distinct pairs).
int launch_set(hipStream_t bs, Ticket* const* t, int n)
{
    EvalArgs ea[kMaxJobs];
    for (int q = 0; q < n; ++q) {
        HIP_TRY(hipStreamWaitEvent(bs, t[q]->ready, 0));
        ea[q] = t[q]->ea;
    }
    OCTMC_TRY(eval_group(ea, n, bs));
    for (int q = 0; q < n; ++q) HIP_TRY(hipEventRecord(t[q]->done, bs));
    return OCTMC_OK;
}

void batcher_main(octmc_server* S)
{
    (void)hipSetDevice(S->device);
    std::vector<Ticket*> take;
    bool launched_before[2] = {false, false};
    for (int step = 0;; step ^= 1) {
        hipStream_t bs = S->bs[step];
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_batch.wait(lk, [&] { return S->stop_batcher || !S->pending.empty(); });
            if (S->pending.empty()) return;  // stop_batcher and nothing left
            take.swap(S->pending);
        }
        std::stable_sort(take.begin(), take.end(), [](const Ticket* a, const Ticket* b) {
            return pair_dtype(a->ea.pair) < pair_dtype(b->ea.pair);
        });
        size_t q0 = 0;
        while (q0 < take.size()) {
            size_t q1 = q0 + 1;
            const octmc_dtype dt = pair_dtype(take[q0]->ea.pair);
            while (q1 < take.size() && q1 - q0 < (size_t)kMaxJobs && pair_dtype(take[q1]->ea.pair) == dt) ++q1;
            const int rc = launch_set(bs, take.data() + q0, (int)(q1 - q0));
            if (rc != OCTMC_OK) {
                // Part of the set may already be queued on bs and still write
                // into the requests' slabs: let it finish before the workers
                // see the failure (and free their slabs), and record every
                // done event so that their streams' waits are complete.
                const std::string msg = octmc_last_error();
                (void)hipStreamSynchronize(bs);
                for (size_t q = q0; q < q1; ++q) {
                    (void)hipEventRecord(take[q]->done, bs);
                    take[q]->rc = rc;
                    take[q]->err = msg;
                }
            }
            q0 = q1;
        }
        const hipError_t e = hipEventRecord(S->last[step], bs);
        launched_before[step] = e == hipSuccess;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (Ticket* t : take) t->launched = true;
        }
        S->cv_ticket.notify_all();
        // at most two sets in flight: the next one forms while this one and
        // the one before it run; wait for the one before it
        if (launched_before[step ^ 1]) (void)hipEventSynchronize(S->last[step ^ 1]);
        take.clear();
    }
}

void run_job(octmc_server* S, Worker* W, const Job& job, size_t off, octmc_completion& c)
{
    const octmc_request& r = job.req;
    Slab slab{S->base + off, job.footprint, 0};
    octmc_pair* P = nullptr;
    DirectEval direct;
    GroupEval grouped(S, W);
    Evaluator* ev = S->mode == OCTMC_SERVE_GROUPED ? static_cast<Evaluator*>(&grouped) : &direct;
    int rc = pair_create_impl(S->ctx, &r.params, &r.shape, r.oct_x, r.oct_y, r.octa_x, r.octa_y, r.enface_x,
                              r.enface_y, r.valid_x, r.valid_y, W->s, &slab, &P);
    if (rc == OCTMC_OK)
        rc = register_impl(P, r.disp_out, r.merged_oct, r.merged_octa, &c.report, W->s, ev, &slab, W->h_terms,
                           W->h_dots);
    if (rc != OCTMC_OK) std::snprintf(c.error, sizeof(c.error), "%s", octmc_last_error());
    const hipError_t e = hipStreamSynchronize(W->s);  // the slab is free only after the request's work
    if (rc == OCTMC_OK && e != hipSuccess) {
        rc = OCTMC_E_DEVICE;
        std::snprintf(c.error, sizeof(c.error), "%s", hipGetErrorString(e));
    }
    if (P) octmc_pair_destroy(P);
    c.status = rc;
    c.bytes_used = slab.used;
}

void worker_main(octmc_server* S, Worker* W)
{
    (void)hipSetDevice(S->device);
    for (;;) {
        Job job;
        size_t off = 0;
        double t_admit = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                if (!S->queue.empty() && S->arena.take(S->queue.front().footprint, &off)) break;
                if (S->stop && S->queue.empty()) return;
                S->cv_admit.wait(lk);
            }
            job = S->queue.front();
            S->queue.pop_front();
            ++S->active;
            t_admit = S->now();  // under the lock: admission times follow admission order
        }
        S->cv_admit.notify_all();  // the next request may fit as well
        octmc_completion c{};
        c.id = job.id;
        c.tag = job.req.tag;
        c.t_submit = job.t_submit;
        c.t_admit = t_admit;
        c.bytes_reserved = job.footprint;
        run_job(S, W, job, off, c);
        c.t_done = S->now();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->arena.give(off, job.footprint);
            --S->active;
            S->done.push_back(c);
        }
        S->cv_admit.notify_all();
        S->cv_done.notify_all();
    }
}

int check_request(const octmc_request* req)
{
    if (!req) return fail(OCTMC_E_INVALID, "request is NULL");
    const octmc_params pr = resolve_levels(req->params, req->shape);
    OCTMC_TRY(validate_params(&pr));
    OCTMC_TRY(validate_shape(&pr, &req->shape));
    if (!req->oct_x || !req->oct_y || !req->disp_out) return fail(OCTMC_E_INVALID, "oct_x, oct_y, disp_out required");
    const bool octa = req->octa_x && req->octa_y, enf = req->enface_x && req->enface_y;
    if (!octa && !enf) return fail(OCTMC_E_INVALID, "need both OCTA volumes or both en face images");
    if ((req->octa_x != nullptr) != (req->octa_y != nullptr) ||
        (req->enface_x != nullptr) != (req->enface_y != nullptr) ||
        (req->valid_x != nullptr) != (req->valid_y != nullptr))
        return fail(OCTMC_E_INVALID, "inputs must be given for both scans");
    if (req->merged_octa && !octa) return fail(OCTMC_E_INVALID, "merged_octa needs OCTA volumes");
    if (req->merged_octa && !req->merged_oct) return fail(OCTMC_E_INVALID, "merged_octa needs merged_oct");
    if (req->params.flags & OCTMC_PREALIGN)
        return fail(OCTMC_E_INVALID, "OCTMC_PREALIGN is not available for served requests (prealign with "
                                     "octmc_pair_create, then submit the prealigned volumes)");
    return OCTMC_OK;
}

size_t request_footprint(const octmc_request* req)
{
    return pair_footprint(resolve_levels(req->params, req->shape), req->shape, req->octa_x != nullptr,
                          req->valid_x != nullptr, req->merged_oct != nullptr);
}

void destroy_server(octmc_server* S)
{
    for (int q = 0; q < 2; ++q) {
        if (S->bs[q]) (void)hipStreamDestroy(S->bs[q]);
        if (S->last[q]) (void)hipEventDestroy(S->last[q]);
    }
    for (Worker* W : S->workers) {
        if (W->s) (void)hipStreamDestroy(W->s);
        if (W->ready) (void)hipEventDestroy(W->ready);
        if (W->done) (void)hipEventDestroy(W->done);
        if (W->h_terms) (void)hipHostFree(W->h_terms);
        if (W->h_dots) (void)hipHostFree(W->h_dots);
        delete W;
    }
    if (S->base) (void)hipFree(S->base);
    delete S;
}

}  // namespace

extern "C" {

int octmc_request_footprint(const octmc_request* req, uint64_t* bytes)
{
    if (!bytes) return fail(OCTMC_E_INVALID, "bytes is NULL");
    OCTMC_TRY(check_request(req));
    *bytes = request_footprint(req);
    return OCTMC_OK;
}

int octmc_server_create(octmc_ctx* ctx, uint64_t hbm_budget_bytes, int32_t max_active, int32_t mode,
                        octmc_server** out)
{
    if (!ctx || !out) return fail(OCTMC_E_INVALID, "NULL argument");
    if (max_active < 1 || max_active > 64) return fail(OCTMC_E_INVALID, "max_active must lie in [1, 64]");
    if (mode != OCTMC_SERVE_GROUPED && mode != OCTMC_SERVE_STREAMS) return fail(OCTMC_E_INVALID, "unknown mode");
    if (hbm_budget_bytes < (1u << 20)) return fail(OCTMC_E_INVALID, "budget below 1 MiB");
    auto* S = new octmc_server();
    S->ctx = ctx;
    S->device = ctx_device(ctx);
    S->mode = mode;
    S->max_active = max_active;
    S->start = Clock::now();
    struct Guard {
        octmc_server* s;
        ~Guard()
        {
            if (s) destroy_server(s);
        }
    } guard{S};
    HIP_TRY(hipSetDevice(S->device));
    S->budget = (size_t)hbm_budget_bytes & ~(size_t)255;
    void* mem = nullptr;
    HIP_TRY(hipMalloc(&mem, S->budget));
    S->base = static_cast<char*>(mem);
    S->arena.reset(S->budget);
    for (int q = 0; q < 2; ++q) {
        HIP_TRY(hipStreamCreateWithFlags(&S->bs[q], hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&S->last[q], hipEventDisableTiming));
    }
    for (int k = 0; k < max_active; ++k) {
        auto* W = new Worker();
        S->workers.push_back(W);
        HIP_TRY(hipStreamCreateWithFlags(&W->s, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&W->ready, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&W->done, hipEventDisableTiming));
        HIP_TRY(hipHostMalloc(&W->h_terms, OCTMC_NTERMS * 8, hipHostMallocDefault));
        HIP_TRY(hipHostMalloc(&W->h_dots, (kMaxDots + 1) * 8, hipHostMallocDefault));
    }
    if (mode == OCTMC_SERVE_GROUPED) S->batcher = std::thread(batcher_main, S);
    for (Worker* W : S->workers) W->th = std::thread(worker_main, S, W);
    guard.s = nullptr;
    *out = S;
    return OCTMC_OK;
}

int octmc_server_submit(octmc_server* srv, const octmc_request* req, uint64_t* id)
{
    if (!srv) return fail(OCTMC_E_INVALID, "server is NULL");
    OCTMC_TRY(check_request(req));
    const size_t fp = request_footprint(req);
    if (fp > srv->budget) return fail(OCTMC_E_OOM, "request footprint exceeds the server's memory budget");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) return fail(OCTMC_E_BUSY, "server is shutting down");
        Job j;
        j.id = srv->next_id++;
        j.req = *req;
        j.req.params = resolve_levels(req->params, req->shape);
        j.footprint = fp;
        j.t_submit = srv->now();
        if (id) *id = j.id;
        srv->queue.push_back(j);
    }
    srv->cv_admit.notify_all();
    return OCTMC_OK;
}

int octmc_server_poll(octmc_server* srv, octmc_completion* out, int32_t max, int32_t wait_ms, int32_t* n)
{
    if (!srv || !n || (max > 0 && !out)) return fail(OCTMC_E_INVALID, "NULL argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto ready = [&] { return !srv->done.empty() || (srv->queue.empty() && srv->active == 0); };
    if (wait_ms < 0)
        srv->cv_done.wait(lk, ready);
    else if (wait_ms > 0)
        srv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
    int k = 0;
    while (k < max && !srv->done.empty()) {
        out[k++] = srv->done.front();
        srv->done.pop_front();
    }
    *n = k;
    return OCTMC_OK;
}

int octmc_server_status(const octmc_server* srv, int32_t* queued, int32_t* active, int32_t* done)
{
    if (!srv) return fail(OCTMC_E_INVALID, "server is NULL");
    auto* S = const_cast<octmc_server*>(srv);
    std::lock_guard<std::mutex> lk(S->mu);
    if (queued) *queued = (int32_t)S->queue.size();
    if (active) *active = S->active;
    if (done) *done = (int32_t)S->done.size();
    return OCTMC_OK;
}

int octmc_server_destroy(octmc_server* srv)
{
    if (!srv) return OCTMC_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_admit.notify_all();
    for (Worker* W : srv->workers)
        if (W->th.joinable()) W->th.join();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop_batcher = true;
    }
    srv->cv_batch.notify_all();
    if (srv->batcher.joinable()) srv->batcher.join();
    (void)hipSetDevice(srv->device);
    destroy_server(srv);
    return OCTMC_OK;
}

}  // extern "C"
