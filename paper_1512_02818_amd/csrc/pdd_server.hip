// Serving loop of the nodal solver: continuous batching of node-solve
// requests, each solved to its own standard error by the balanced-simulation
// rule (Sec. 3.1, eq. F:N_y_h): a pilot, a per-node plan, then the planned
// paths in request-determined chunks merged into the pilot's sums.
//
// One host thread runs epochs. An epoch admits waiting requests (FIFO, while
// a slot is free and the memory model fits the budget), takes the next chunk
// of every admitted request that is not in an epoch in flight as a batch
// item, and enqueues the batch on a free lane (a stream and the scratch of a
// context) through the same path as pdd_solve_batch. With up to `pipeline`
// epochs in flight, the thread waits for the first of them to end (cut short
// by a new request while a lane is free), then plans its finished pilots and
// completes its finished requests while the other lanes keep the device
// busy. Because a
// request's chunk sequence depends only on the request and the server
// options, a request is in at most one epoch in flight, and an epoch never
// exceeds one launch per group, a request gives bitwise the same statistics
// alone or in any mix, at any pipeline depth.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "pdd.h"
#include "host_runtime.hpp"

using namespace pdd;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

enum class Phase { Queued, Pilot, Planned };

struct Request {
    uint64_t id = 0;
    pdd_request req{};
    std::vector<double> nodes;          // copy of the caller's nodes
    pdd_grid u_prev{}, resid{};         // copies of the grid structs
    pdd_grid grad[3]{};                 // gradient grids of an Ito request (copies)
    bool cv = false, ito = false;
    uint64_t mem = 0;                   // memory model of the request
    Phase phase = Phase::Queued;
    pdd_status status = PDD_OK;         // of its last allocation or epoch
    pdd_node_stats *dev_out = nullptr;  // device statistics
    std::vector<uint64_t> target;       // planned paths per node
    std::vector<double> nu;             // pilot mean steps per path, per node
    double remaining = 0.0;             // path-steps still to run (estimate)
    uint64_t per_node_chunk = 0;        // paths per node in one continuation chunk
    uint64_t chunk = 0;                 // continuation chunks done
    uint64_t max_target = 0;
    Clock::time_point t_submit, t_admit;
    // batch item of its epoch in flight
    int lane = -1;                      // lane of that epoch, -1 when not in flight
    pdd_solve_opts opts{};
    std::vector<uint64_t> counts;
};

// An epoch slot: a stream, the scratch of a context, the batch it runs.
struct Lane {
    pdd_ctx *ctx = nullptr;
    bool own_ctx = false;               // created by the server (lane 0 uses the server's)
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<Request *> batch;
    std::vector<HostItem> items;
    pdd_status st = PDD_OK;             // of the enqueue
    Clock::time_point t0;
    bool busy = false;
};

uint64_t grid_bytes(const pdd_grid &g, int dim)
{
    uint64_t n = 1;
    for (int i = 0; i < dim; ++i) n *= (uint64_t)g.n[i];
    return n * (g.dtype == PDD_DTYPE_F64 ? 8 : 4);
}

}  // namespace

struct pdd_server {
    pdd_ctx *ctx = nullptr;
    pdd_server_opts o{};
    std::vector<Lane> lanes;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stopping = false;
    std::deque<std::unique_ptr<Request>> queue;   // waiting
    std::vector<std::unique_ptr<Request>> active; // admitted (worker thread only)
    std::deque<pdd_completion> done;
    uint64_t next_id = 1;
    // device statistics of finished requests, kept for reuse by size: a
    // hipFree would wait for every epoch in flight (worker thread only)
    std::multimap<size_t, void *> spare_out;
    // report (under mu)
    pdd_server_report rep{};
    bool busy_open = false;                // an epoch is in flight, since busy_since
    Clock::time_point busy_since;
    std::vector<double> latencies;         // completed requests
    std::vector<double> censored;          // cancelled requests: age at cancellation
    std::map<uint64_t, Clock::time_point> outstanding;  // submitted, not finished: submit time
    bool any_submit = false;
    Clock::time_point first_submit, last_done;

    void run();
    void launch(int lane, std::vector<Request *> &batch, uint64_t paths);
    void complete(Lane &L, std::vector<pdd_node_stats> &pilot);
    void finish(Request *r, pdd_status status, hipStream_t s);
    bool admissible();  // under mu
    pdd_node_stats *take_out(int64_t n);
    void give_out(pdd_node_stats *p, int64_t n);
    void release_lanes();
};

namespace {

pdd_status copy_stats(pdd_node_stats *dst, const pdd_node_stats *src, int64_t n, hipStream_t s)
{
    HIP_TRY(hipMemcpyAsync(dst, src, (size_t)n * sizeof(pdd_node_stats), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PDD_OK;
}

size_t out_bytes(int64_t n)
{
    size_t b = 4096;
    while (b < (size_t)n * sizeof(pdd_node_stats)) b *= 2;
    return b;
}

}  // namespace

pdd_node_stats *pdd_server::take_out(int64_t n)
{
    const size_t b = out_bytes(n);
    auto f = spare_out.find(b);
    if (f != spare_out.end()) {
        void *p = f->second;
        spare_out.erase(f);
        return static_cast<pdd_node_stats *>(p);
    }
    void *p = nullptr;
    if (hipMalloc(&p, b) != hipSuccess) return nullptr;
    return static_cast<pdd_node_stats *>(p);
}

void pdd_server::give_out(pdd_node_stats *p, int64_t n)
{
    if (p) spare_out.emplace(out_bytes(n), p);
}

bool pdd_server::admissible()
{
    return !queue.empty() && (int64_t)active.size() < o.max_inflight &&
           rep.mem_in_use + rep.mem_fixed + queue.front()->mem <= o.memory_budget;
}

// Completes a request: statistics to the caller (on success, copied on
// stream s), memory back to the budget, a completion record. Called by the
// worker without the lock.
void pdd_server::finish(Request *r, pdd_status status, hipStream_t s)
{
    pdd_completion c{};
    c.id = r->id;
    c.user_tag = r->req.user_tag;
    c.n_nodes = r->req.n_nodes;
    if (status == PDD_OK && r->dev_out) {
        std::vector<pdd_node_stats> st(r->req.n_nodes);
        status = copy_stats(st.data(), r->dev_out, r->req.n_nodes, s);
        if (status == PDD_OK) {
            std::memcpy(r->req.out, st.data(), st.size() * sizeof(pdd_node_stats));
            for (auto &x : st) {
                c.paths += (uint64_t)x.n;
                c.path_steps += (uint64_t)x.steps_sum;
            }
        }
    }
    give_out(r->dev_out, r->req.n_nodes);
    r->dev_out = nullptr;
    const auto now = Clock::now();
    c.status = status;
    c.queued_ms = r->phase == Phase::Queued ? ms_between(r->t_submit, now) : ms_between(r->t_submit, r->t_admit);
    c.latency_ms = ms_between(r->t_submit, now);
    std::lock_guard<std::mutex> lk(mu);
    if (r->phase != Phase::Queued) {
        rep.mem_in_use -= r->mem;
        --rep.inflight;
    }
    outstanding.erase(r->id);
    if (status == PDD_OK) {
        ++rep.completed;
        rep.nodes_completed += (uint64_t)r->req.n_nodes;
        rep.path_steps += c.path_steps;
        latencies.push_back(c.latency_ms);
        last_done = now;
    } else if (status == PDD_E_BUSY) {  // cancelled: its latency is at least its age
        ++rep.cancelled;
        censored.push_back(c.latency_ms);
    } else {
        ++rep.failed;
    }
    done.push_back(c);
    cv_done.notify_all();
}

// Enqueues an epoch over `batch` (each request contributes its next chunk) on
// a free lane. Runs on the worker thread.
void pdd_server::launch(int lane, std::vector<Request *> &batch, uint64_t paths)
{
    Lane &L = lanes[lane];
    L.batch = batch;
    L.items.assign(batch.size(), HostItem{});
    for (size_t q = 0; q < batch.size(); ++q) {
        Request *r = batch[q];
        HostItem &it = L.items[q];
        it.prob = r->req.problem;
        it.u_prev = r->cv ? &r->u_prev : nullptr;
        it.resid = r->cv ? &r->resid : nullptr;
        it.grad = r->ito ? r->grad : nullptr;
        it.nodes = r->nodes.data();
        it.n_nodes = r->req.n_nodes;
        it.o = &r->opts;
        it.out = r->dev_out;
        r->lane = lane;
    }
    L.t0 = Clock::now();
    {
        std::lock_guard<std::mutex> lk(mu);
        rep.paths_run += paths;
        if (!busy_open) {
            busy_open = true;
            busy_since = L.t0;
        }
    }
    // one launch per group whatever the context's tuning table caps: a
    // request's node sums then never depend on the mix it ran in
    L.st = run_items(L.ctx, L.items, L.stream, true, ctx);
    // recorded even after a failed enqueue, so that completion waits for
    // whatever did reach the stream
    if (hipEventRecord(L.done, L.stream) != hipSuccess && L.st == PDD_OK)
        L.st = fail(PDD_E_HIP, "could not record the end of an epoch");
    L.busy = true;
}

// Waits for the epoch on lane L, then plans its finished pilots and completes
// its finished requests. Runs on the worker thread.
void pdd_server::complete(Lane &L, std::vector<pdd_node_stats> &pilot)
{
    pdd_status st = L.st;
    if (hipEventSynchronize(L.done) != hipSuccess && st == PDD_OK) st = fail(PDD_E_HIP, "epoch failed on the device");
    const auto now = Clock::now();
    L.busy = false;
    bool idle = true;
    for (const Lane &x : lanes) idle &= !x.busy;
    {
        std::lock_guard<std::mutex> lk(mu);
        ++rep.epochs;
        rep.epoch_s += ms_between(L.t0, now) / 1e3;
        if (idle && busy_open) {
            rep.busy_s += ms_between(busy_since, now) / 1e3;
            busy_open = false;
        }
    }
    for (Request *r : L.batch) {
        r->lane = -1;
        r->status = st;
    }
    for (Request *r : L.batch) {
        bool end = st != PDD_OK;
        pdd_status why = st;
        if (!end && r->phase == Phase::Pilot) {
            const int64_t n = r->req.n_nodes;
            pilot.resize(n);
            why = copy_stats(pilot.data(), r->dev_out, n, L.stream);
            r->target.resize(n);
            r->nu.resize(n);
            for (int64_t i = 0; i < n; ++i) r->nu[i] = pilot[i].mean_steps;
            if (why == PDD_OK) why = pdd_plan_paths(pilot.data(), n, r->req.target_se, o.n_max, r->target.data());
            if (why != PDD_OK) {
                end = true;
            } else {
                r->phase = Phase::Planned;
                r->max_target = *std::max_element(r->target.begin(), r->target.end());
                r->per_node_chunk = std::max<uint64_t>(1, o.chunk_paths / (uint64_t)n);
                r->chunk = 0;
                end = r->max_target <= o.n_pilot;
            }
        } else if (!end) {
            ++r->chunk;
            end = o.n_pilot + r->chunk * r->per_node_chunk >= r->max_target;
        }
        if (end) {
            finish(r, why, L.stream);
            for (auto &up : active)
                if (up.get() == r) up.reset();
        }
    }
    active.erase(std::remove(active.begin(), active.end(), nullptr), active.end());
    L.batch.clear();
    L.items.clear();
}

void pdd_server::run()
{
    (void)hipSetDevice(ctx->device);
    std::vector<pdd_node_stats> pilot;
    std::deque<int> fifo;  // lanes in flight, oldest first
    auto free_lane = [&] {
        for (size_t i = 0; i < lanes.size(); ++i)
            if (!lanes[i].busy) return (int)i;
        return -1;
    };
    for (;;) {
        // admission at the epoch boundary
        {
            std::unique_lock<std::mutex> lk(mu);
            if (fifo.empty() && active.empty() && queue.empty() && !stopping)
                cv_work.wait(lk, [&] { return stopping || !queue.empty(); });
            if (stopping) break;
            while (admissible()) {
                std::unique_ptr<Request> r = std::move(queue.front());
                queue.pop_front();
                r->phase = Phase::Pilot;
                r->t_admit = Clock::now();
                rep.mem_in_use += r->mem;
                rep.mem_peak = std::max(rep.mem_peak, rep.mem_in_use);
                ++rep.admitted;
                ++rep.inflight;
                rep.queued = queue.size();
                active.push_back(std::move(r));
            }
        }
        // device statistics of newly admitted requests
        for (auto &r : active) {
            if (r->dev_out || r->phase != Phase::Pilot || r->status != PDD_OK) continue;
            r->dev_out = take_out(r->req.n_nodes);
            if (!r->dev_out)
                r->status = fail(PDD_E_NOMEM, "device statistics of request %llu", (unsigned long long)r->id);
        }
        // failed allocations end here (such a request was never in flight)
        for (auto &up : active)
            if (up->status != PDD_OK && up->lane < 0) {
                finish(up.get(), up->status, nullptr);
                up.reset();
            }
        active.erase(std::remove(active.begin(), active.end(), nullptr), active.end());
        // the next epoch on a free lane: the next chunk of the requests not in
        // flight within epoch_paths, pilots first, then the least remaining
        // work (the order decides only when a chunk runs, never what it computes)
        const int lane = free_lane();
        bool left = false;  // requests not in flight that this epoch leaves out
        if (lane >= 0) {
            std::vector<Request *> order;
            for (auto &up : active) {
                Request *r = up.get();
                if (r->lane >= 0) continue;
                if (r->phase == Phase::Planned) {
                    const uint64_t off = o.n_pilot + r->chunk * r->per_node_chunk;
                    double w = 0.0;
                    for (size_t i = 0; i < r->target.size(); ++i)
                        if (r->target[i] > off) w += (double)(r->target[i] - off) * r->nu[i];
                    r->remaining = w;
                }
                order.push_back(r);
            }
            std::stable_sort(order.begin(), order.end(), [](const Request *a, const Request *b) {
                const bool pa = a->phase == Phase::Pilot, pb = b->phase == Phase::Pilot;
                if (pa != pb) return pa;
                if (!pa && a->remaining != b->remaining) return a->remaining < b->remaining;
                return a->id < b->id;
            });
            std::vector<Request *> batch;
            uint64_t total = 0;
            for (Request *r : order) {
                const uint64_t n = (uint64_t)r->req.n_nodes;
                pdd_solve_opts &op = r->opts;
                std::memset(&op, 0, sizeof op);
                op.dt = r->req.dt;
                op.stream_id = r->req.stream_id;
                op.precision = r->req.precision;
                op.exit_mode = r->req.exit_mode;
                op.law = PDD_LAW_GAUSS;
                uint64_t size;
                if (r->phase == Phase::Pilot) {
                    op.n_paths = o.n_pilot;
                    size = n * o.n_pilot;
                } else {
                    const uint64_t off = o.n_pilot + r->chunk * r->per_node_chunk;
                    r->counts.resize(n);
                    size = 0;
                    for (uint64_t i = 0; i < n; ++i) {
                        const uint64_t t = r->target[i];
                        r->counts[i] = t > off ? std::min(t - off, r->per_node_chunk) : 0;
                        size += r->counts[i];
                    }
                    op.n_paths_per_node = r->counts.data();
                    op.path_offset = off;
                    op.flags = PDD_ACCUMULATE;
                }
                if (!batch.empty() && total + size > o.epoch_paths) {
                    left = true;
                    continue;
                }
                total += size;
                batch.push_back(r);
            }
            if (!batch.empty()) {
                launch(lane, batch, total);
                fifo.push_back(lane);
            }
        }
        if (fifo.empty()) continue;
        // what did not fit goes to the next free lane first
        const bool lane_free = free_lane() >= 0;
        if (left && lane_free) continue;
        // the first epoch in launch order that has ended; with a lane free, a
        // new request cuts the wait short
        int ready = -1;
        for (;;) {
            for (size_t k = 0; k < fifo.size() && ready < 0; ++k)
                if (hipEventQuery(lanes[fifo[k]].done) != hipErrorNotReady) ready = (int)k;
            if (ready >= 0) break;
            std::unique_lock<std::mutex> lk(mu);
            if (stopping || (lane_free && admissible())) break;
            cv_work.wait_for(lk, std::chrono::microseconds(200));
        }
        if (ready < 0) continue;
        const int li = fifo[ready];
        fifo.erase(fifo.begin() + ready);
        complete(lanes[li], pilot);
    }
    // stopping: the epochs in flight end, then every request is cancelled
    for (int i : fifo) {
        (void)hipEventSynchronize(lanes[i].done);
        lanes[i].busy = false;
        for (Request *r : lanes[i].batch) r->lane = -1;
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        if (busy_open) rep.busy_s += ms_between(busy_since, Clock::now()) / 1e3;
        busy_open = false;
    }
    for (auto &up : active) finish(up.get(), PDD_E_BUSY, nullptr);
    active.clear();
    std::deque<std::unique_ptr<Request>> rest;
    {
        std::lock_guard<std::mutex> lk(mu);
        rest.swap(queue);
        rep.queued = 0;
    }
    for (auto &up : rest) finish(up.get(), PDD_E_BUSY, nullptr);
}

// Streams, events and contexts of the lanes, and the spare statistics
// buffers (after the worker has ended).
void pdd_server::release_lanes()
{
    for (Lane &L : lanes) {
        if (L.done) (void)hipEventSynchronize(L.done);
        if (L.stream) (void)hipStreamDestroy(L.stream);
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.own_ctx) pdd_shutdown(L.ctx);
    }
    lanes.clear();
    (void)hipSetDevice(ctx->device);
    for (auto &kv : spare_out) (void)hipFree(kv.second);
    spare_out.clear();
}

extern "C" {

pdd_status pdd_server_create(pdd_ctx *ctx, const pdd_server_opts *opts, pdd_server **out)
{
    if (!ctx || !out) return fail(PDD_E_INVALID, "ctx or out is NULL");
    *out = nullptr;
    pdd_server_opts o{};
    if (opts) o = *opts;
    if (!o.memory_budget) o.memory_budget = 64ull << 30;
    if (!o.max_inflight) o.max_inflight = 1024;
    if (!o.n_pilot) o.n_pilot = 1000;
    if (!o.n_max) o.n_max = 1ull << 31;
    if (!o.chunk_paths) o.chunk_paths = 1ull << 22;
    if (!o.epoch_paths) o.epoch_paths = kScratchSlots;
    if (!o.pipeline) o.pipeline = 2;
    if (o.max_inflight < 0 || o.max_queued < 0 || o.n_pilot < 2 || o.n_max < o.n_pilot ||
        o.n_max > (1ull << 32) || o.epoch_paths > kScratchSlots || o.chunk_paths > o.epoch_paths ||
        o.pipeline < 1 || o.pipeline > 4 || o.reserved != 0)
        return fail(PDD_E_INVALID, "bad server options");
    auto sv = std::make_unique<pdd_server>();
    sv->ctx = ctx;
    sv->o = o;
    // record scratch of a full epoch per lane: phi, e (FP64) and the exit step per path
    sv->rep.mem_fixed = (uint64_t)o.pipeline * o.epoch_paths * (8 + 8 + 4);
    if (sv->rep.mem_fixed >= o.memory_budget)
        return fail(PDD_E_INVALID, "memory budget below the record scratch (%llu bytes)",
                    (unsigned long long)sv->rep.mem_fixed);
    HIP_TRY(hipSetDevice(ctx->device));
    sv->lanes.resize(o.pipeline);
    for (int i = 0; i < o.pipeline; ++i) {
        Lane &L = sv->lanes[i];
        pdd_status st = PDD_OK;
        if (i == 0) {
            L.ctx = ctx;
        } else if ((st = pdd_init(&L.ctx, ctx->device)) == PDD_OK) {
            L.own_ctx = true;
            L.ctx->tuned = ctx->tuned;  // the launch shapes of the server's context
        }
        if (st == PDD_OK && (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
                             hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess))
            st = fail(PDD_E_HIP, "could not create the streams of the server");
        if (st != PDD_OK) {
            sv->release_lanes();
            return st;
        }
    }
    try {
        sv->worker = std::thread([s = sv.get()] { s->run(); });
    } catch (...) {
        sv->release_lanes();
        return fail(PDD_E_INTERNAL, "could not start the server thread");
    }
    *out = sv.release();
    return PDD_OK;
}

pdd_status pdd_server_submit(pdd_server *sv, const pdd_request *req, uint64_t *id)
{
    if (!sv || !req || !id) return fail(PDD_E_INVALID, "NULL argument");
    if (req->n_nodes < 1 || !req->nodes || !req->out || !req->problem)
        return fail(PDD_E_INVALID, "request needs nodes, out and a problem");
    if (!(req->target_se > 0.0) || !std::isfinite(req->target_se))
        return fail(PDD_E_INVALID, "target_se must be finite and > 0");
    if (req->problem->ctx != sv->ctx) return fail(PDD_E_INVALID, "problem belongs to another context");
    auto r = std::make_unique<Request>();
    r->req = *req;
    const int dim = req->problem->desc.dim;
    r->nodes.assign(req->nodes, req->nodes + (size_t)req->n_nodes * dim);
    r->req.nodes = r->nodes.data();
    r->cv = req->u_prev || req->resid;
    if (req->u_prev) r->u_prev = *req->u_prev;
    if (req->resid) r->resid = *req->resid;
    r->ito = req->grad != nullptr;
    if (r->ito && r->cv) return fail(PDD_E_INVALID, "a request takes the correction grids or the gradient grids, not both");
    if (r->ito)
        for (int c = 0; c < dim; ++c) r->grad[c] = req->grad[c];
    // the same checks as a solve of the pilot (nodes inside, grids, options)
    pdd_solve_opts op{};
    op.dt = req->dt;
    op.n_paths = sv->o.n_pilot;
    op.stream_id = req->stream_id;
    op.precision = req->precision;
    op.exit_mode = req->exit_mode;
    HostItem it;
    it.prob = req->problem;
    it.u_prev = req->u_prev ? &r->u_prev : nullptr;
    it.resid = req->resid ? &r->resid : nullptr;
    it.grad = r->ito ? r->grad : nullptr;
    it.nodes = r->nodes.data();
    it.n_nodes = req->n_nodes;
    it.o = &op;
    it.out = req->out;
    pdd_status st = validate_item(it);
    if (st) return st;
    const uint64_t n = (uint64_t)req->n_nodes;
    if (n * sv->o.n_pilot > sv->o.epoch_paths)
        return fail(PDD_E_UNSUPPORTED, "pilot of %llu nodes exceeds epoch_paths", (unsigned long long)n);
    // memory model: device statistics + the solve's per-node tables + grids
    r->mem = n * (sizeof(pdd_node_stats) + sizeof(NodeAcc) + dim * sizeof(double) + 2 * sizeof(uint64_t));
    if (r->cv) r->mem += grid_bytes(r->u_prev, dim) + grid_bytes(r->resid, dim);
    if (r->ito) r->mem += (uint64_t)dim * grid_bytes(r->grad[0], dim);
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(sv->mu);
    ++sv->rep.submitted;
    if (r->mem + sv->rep.mem_fixed > sv->o.memory_budget) {
        ++sv->rep.shed;
        return fail(PDD_E_NOMEM, "request needs %llu bytes, more than the budget", (unsigned long long)r->mem);
    }
    if (sv->stopping || (sv->o.max_queued > 0 && (int64_t)sv->queue.size() >= sv->o.max_queued)) {
        ++sv->rep.shed;
        return fail(PDD_E_BUSY, "request shed: queue full");
    }
    if (!sv->any_submit) {
        sv->any_submit = true;
        sv->first_submit = r->t_submit;
    }
    r->id = sv->next_id++;
    *id = r->id;
    sv->outstanding[r->id] = r->t_submit;
    sv->queue.push_back(std::move(r));
    sv->rep.queued = sv->queue.size();
    sv->cv_work.notify_one();
    return PDD_OK;
}

pdd_status pdd_server_poll(pdd_server *sv, pdd_completion *out, int32_t cap, int32_t *n, int32_t wait_ms)
{
    if (!sv || !n || cap < 0 || (cap > 0 && !out)) return fail(PDD_E_INVALID, "bad arguments");
    std::unique_lock<std::mutex> lk(sv->mu);
    if (sv->done.empty() && wait_ms > 0)
        sv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !sv->done.empty(); });
    int32_t k = 0;
    while (k < cap && !sv->done.empty()) {
        out[k++] = sv->done.front();
        sv->done.pop_front();
    }
    *n = k;
    return PDD_OK;
}

pdd_status pdd_server_report_get(pdd_server *sv, pdd_server_report *out)
{
    if (!sv || !out) return fail(PDD_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    pdd_server_report r = sv->rep;
    r.queued = sv->queue.size();
    // nearest-rank percentile of sorted values
    auto pct = [](const std::vector<double> &v, double p) {
        const size_t k = (size_t)std::ceil(p / 100.0 * (double)v.size());
        return v[std::min(v.size(), std::max<size_t>(k, 1)) - 1];
    };
    std::vector<double> l = sv->latencies;
    std::sort(l.begin(), l.end());
    // every request not shed: completed at its latency, cancelled or
    // unfinished at its age (a lower bound of its latency)
    std::vector<double> cens = sv->censored;
    const auto now = Clock::now();
    for (const auto &kv : sv->outstanding) cens.push_back(ms_between(kv.second, now));
    std::vector<double> all = l;
    all.insert(all.end(), cens.begin(), cens.end());
    std::sort(all.begin(), all.end());
    r.censored = cens.size();
    if (sv->busy_open) r.busy_s += ms_between(sv->busy_since, now) / 1e3;
    r.p50_ms = r.p99_ms = r.mean_ms = r.p50_done_ms = r.p99_done_ms = 0.0;
    r.p50_censored = r.p99_censored = 0;
    if (!all.empty()) {
        r.p50_ms = pct(all, 50.0);
        r.p99_ms = pct(all, 99.0);
        // lower bounds once a censored age sits at or below them
        const double cmin = cens.empty() ? HUGE_VAL : *std::min_element(cens.begin(), cens.end());
        r.p50_censored = cmin <= r.p50_ms;
        r.p99_censored = cmin <= r.p99_ms;
    }
    if (!l.empty()) {
        r.p50_done_ms = pct(l, 50.0);
        r.p99_done_ms = pct(l, 99.0);
        double s = 0.0;
        for (double v : l) s += v;
        r.mean_ms = s / (double)l.size();
        r.wall_s = ms_between(sv->first_submit, sv->last_done) / 1e3;
        r.node_solves_per_s = r.wall_s > 0 ? (double)r.nodes_completed / r.wall_s : 0.0;
    }
    *out = r;
    return PDD_OK;
}

void pdd_server_destroy(pdd_server *sv)
{
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
    }
    sv->cv_work.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    sv->release_lanes();
    delete sv;
}

}  // extern "C"
