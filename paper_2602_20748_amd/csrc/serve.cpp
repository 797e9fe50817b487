// Serving: a request loop over one resident graph (host runtime, no kernels of its own).
//
// Requests wait in a queue; `workers` host threads each own a HIP stream and take the next
// request whose workspace fits in the free part of the caller's device pool (first-fit
// allocator).  A worker runs the request with rpq_eval / crpq_eval on its stream, so admitted
// requests overlap on the device, then returns the workspace and wakes the others.  Memory is
// the admission gate: the workspace of a dense RPQ is its per-unit visited bitmaps
// (V * states * unit width bits, times the units in flight), of a sparse RPQ or a CRPQ what the
// call asks for.  A dense RPQ that does not fit the whole pool is split (fewer units in flight,
// then narrower units).  A request that runs short of workspace re-enters the queue at the
// front with the size the library asked for.
//
// With the resident engine on, dense RPQs it can run go to a driver thread instead: it stages
// every such request that arrived into the engine (its units join the device unit queue of the
// persistent batched kernel), runs one bounded launch, completes the requests whose units have
// all retired, and repeats while anything is queued or running.
#include "internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace {

constexpr double kHeadWaitMs = 50.0;    // after this the oldest request may no longer be passed
constexpr size_t kLookahead = 64;       // queued requests considered for admission
constexpr uint64_t kAlign = 256;

// First-fit allocator over [0, size): free blocks by offset, coalesced on release.
class PoolAlloc {
public:
    explicit PoolAlloc(uint64_t size) : size_(size) {
        if (size) free_[0] = size;
    }
    bool alloc(uint64_t bytes, uint64_t* off) {
        bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const uint64_t rest = it->second - bytes;
            const uint64_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
        used_ -= bytes;
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
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }

private:
    uint64_t size_, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

struct Job {
    uint64_t id = 0;
    rpq_request req{};
    rpq_eval_opts opts{};            // dense RPQ: the split chosen at admission
    std::vector<crpq_atom> atoms;    // CRPQ: copies of the caller's host arrays
    std::vector<int64_t> binding;
    std::vector<int32_t> vlabel;
    std::vector<const uint32_t*> domain;
    std::vector<uint64_t> domain_size;
    std::vector<uint32_t> neq;
    uint64_t need = 0;               // workspace bytes to admit with
    rpq_ticket t{};
    bool resident = false;           // routed to the resident engine
};

}  // namespace

struct rpq_server {
    rpq_graph_t g = nullptr;
    char* pool = nullptr;
    std::unique_ptr<PoolAlloc> alloc;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job*> queue;
    std::vector<std::unique_ptr<Job>> jobs;   // index = ticket
    std::vector<std::thread> workers;
    bool stopping = false;
    uint64_t running = 0, completed = 0, failed = 0, eprod = 0;
    // resident engine (null when off): its queue, driver thread and pool segment
    rpq::Resident* res = nullptr;
    std::deque<Job*> res_queue;
    std::condition_variable cv_res;
    std::thread driver;
    uint64_t res_off = 0, res_bytes = 0, res_slot_bytes = 0, res_running = 0, res_completed = 0, res_launches = 0;
    uint32_t res_iters = 8;
    uint32_t res_width = 64, res_max_units = 0;
    std::chrono::steady_clock::time_point t0;

    uint64_t worker_pool() const { return alloc->size() - (res ? ((res_bytes + 255) & ~255ull) : 0); }

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// Workspace of a dense RPQ that fits `limit`, splitting the source units if needed.
int dense_plan(rpq_graph_t g, Job* j, uint64_t limit) {
    const rpq_request& r = j->req;
    const uint64_t n = (r.flags & RPQ_ALL_SOURCES) && r.n_sources == 0 ? g->V : r.n_sources;
    std::memset(&j->opts, 0, sizeof j->opts);
    uint64_t ws = 0;
    RPQ_TRY(rpq_eval_workspace_size(g, &r.nfa, n, r.flags, &j->opts, &ws));
    if (ws <= limit) {
        j->need = ws;
        return RPQ_OK;
    }
    // fewer units in flight, then narrower units
    for (uint32_t width = 4096; width >= 64; width /= 2) {
        for (uint32_t conc = 256; conc >= 1; conc /= 2) {
            rpq_eval_opts o{};
            o.batch_width = width;
            o.concurrency = conc;
            if (rpq_eval_workspace_size(g, &r.nfa, n, r.flags, &o, &ws) != RPQ_OK) continue;
            if (ws <= limit) {
                j->opts = o;
                j->need = ws;
                return RPQ_OK;
            }
        }
    }
    rpq::set_error("request needs more than the %llu-byte pool even at one 64-source unit", (unsigned long long)limit);
    return RPQ_ENOMEM;
}

void finish_job(rpq_server* s, Job* j, int rc, double end) {
    j->t.status = rc;
    j->t.end_ms = end;
    j->t.done = 1;
    if (rc == RPQ_OK || rc == RPQ_EOVERFLOW) {
        ++s->completed;
        s->eprod += j->t.product_edges;
    } else {
        ++s->failed;
    }
}

int run_job(rpq_server* s, Job* j, char* ws, hipStream_t stream, uint64_t* needed) {
    const rpq_request& r = j->req;
    *needed = 0;
    if (r.kind == RPQ_REQ_RPQ) {
        rpq_result res;
        std::memset(&res, 0, sizeof res);
        res.pairs = r.pairs;
        res.capacity = r.capacity;
        res.per_source = r.per_source;
        const int rc = rpq::eval_impl(s->g, &r.nfa, r.sources, r.n_sources, r.flags, &j->opts, nullptr, ws, j->need,
                                      &res, stream);
        if (rc == RPQ_ENOMEM) *needed = res.workspace_needed;
        j->t.count = res.count;
        j->t.hash = res.hash;
        j->t.product_edges = res.product_edges;
        j->t.written = res.written;
        return rc;
    }
    crpq_vars v;
    std::memset(&v, 0, sizeof v);
    v.n_vars = r.vars.n_vars;
    v.binding = j->binding.empty() ? nullptr : j->binding.data();
    v.vertex_label = j->vlabel.empty() ? nullptr : j->vlabel.data();
    v.domain = j->domain.empty() ? nullptr : j->domain.data();
    v.domain_size = j->domain_size.empty() ? nullptr : j->domain_size.data();
    v.neq = j->neq.empty() ? nullptr : j->neq.data();
    v.n_neq = (uint32_t)(j->neq.size() / 2);
    crpq_result res;
    std::memset(&res, 0, sizeof res);
    res.tuples = r.tuples;
    res.capacity = r.tuple_capacity;
    const int rc = crpq_eval(s->g, j->atoms.data(), (uint32_t)j->atoms.size(), &v, r.flags, ws, j->need, &res, stream);
    if (rc == RPQ_ENOMEM) *needed = res.workspace_needed;
    j->t.count = res.count;
    j->t.hash = res.hash;
    j->t.product_edges = 0;
    j->t.written = res.written;
    return rc;
}

// Next admissible job (its workspace allocated), or null.  Caller holds s->mu.
Job* admit(rpq_server* s, uint64_t* off) {
    if (s->queue.empty()) return nullptr;
    const double now = s->now_ms();
    const bool head_only = now - s->queue.front()->t.arrival_ms > kHeadWaitMs;
    const size_t n = head_only ? 1 : std::min(kLookahead, s->queue.size());
    for (size_t i = 0; i < n; ++i) {
        Job* j = s->queue[i];
        if (s->alloc->alloc(std::max<uint64_t>(j->need, kAlign), off)) {
            s->queue.erase(s->queue.begin() + (long)i);
            return j;
        }
    }
    return nullptr;
}

void worker_main(rpq_server* s) {
    int dev = s->g->device;
    (void)hipSetDevice(dev);
    hipStream_t stream = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        uint64_t off = 0;
        Job* j = nullptr;
        while (!(j = admit(s, &off))) {
            if (s->stopping && s->queue.empty()) {
                lk.unlock();
                if (have_stream) (void)hipStreamDestroy(stream);
                return;
            }
            s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
        }
        ++s->running;
        j->t.start_ms = s->now_ms();
        j->t.workspace_bytes = j->need;
        lk.unlock();
        uint64_t needed = 0;
        int rc = have_stream ? run_job(s, j, s->pool + off, stream, &needed) : RPQ_EDEVICE;
        // nothing of this request may still run on its workspace once the segment goes back to the
        // pool (the calls drain their stream on every return; this keeps the rule local too)
        if (have_stream) (void)hipStreamSynchronize(stream);
        const double end = s->now_ms();
        lk.lock();
        s->alloc->release(off, std::max<uint64_t>(j->need, kAlign));
        --s->running;
        if (rc == RPQ_ENOMEM && needed > j->need && needed <= s->worker_pool()) {
            j->need = needed;              // run again with the workspace the library asked for
            s->queue.push_front(j);
        } else {
            finish_job(s, j, rc, end);
            s->cv_done.notify_all();
        }
        s->cv_work.notify_all();
    }
}

void driver_main(rpq_server* s) {
    (void)hipSetDevice(s->g->device);
    hipStream_t stream = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
    std::vector<rpq::ResidentDone> done;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // stage every arrival that fits now (arrival order); the rest waits for the next launch
        while (!s->res_queue.empty()) {
            Job* j = s->res_queue.front();
            rpq::ResidentQuery q{};
            q.nfa = j->req.nfa;
            q.sources = j->req.sources;
            q.n_sources = (j->req.flags & RPQ_ALL_SOURCES) && j->req.n_sources == 0 ? s->g->V : j->req.n_sources;
            q.pairs = (j->req.flags & RPQ_PAIRS) ? j->req.pairs : nullptr;
            q.capacity = j->req.capacity;
            q.per_source = (j->req.flags & RPQ_PER_SOURCE) ? j->req.per_source : nullptr;
            q.max_len = 0xFFFFFFFFu;
            if (rpq::resident_admit(s->res, q, j->id) != RPQ_OK) break;
            s->res_queue.pop_front();
            j->t.start_ms = s->now_ms();
            j->t.workspace_bytes = s->res_slot_bytes;
            ++s->res_running;
        }
        if (rpq::resident_broken(s->res) && !s->res_queue.empty()) {
            // after a device error the engine takes nothing more: its queue goes to the workers
            while (!s->res_queue.empty()) {
                Job* j = s->res_queue.front();
                s->res_queue.pop_front();
                j->resident = false;
                j->t.resident = 0;
                s->queue.push_back(j);
            }
            s->cv_work.notify_all();
        }
        if (rpq::resident_idle(s->res)) {
            if (s->stopping && s->res_queue.empty()) break;
            s->cv_res.wait_for(lk, std::chrono::milliseconds(5));
            continue;
        }
        lk.unlock();
        done.clear();
        const int rc = have_stream ? rpq::resident_step(s->res, s->res_iters, stream, &done) : RPQ_EDEVICE;
        (void)rc;   // a device error completes every request in flight with it (in `done`)
        const double end = s->now_ms();
        lk.lock();
        ++s->res_launches;
        for (const rpq::ResidentDone& d : done) {
            Job* j = s->jobs[d.token].get();
            j->t.count = d.count;
            j->t.hash = d.hash;
            j->t.product_edges = d.product_edges;
            j->t.written = d.written;
            --s->res_running;
            if (d.status == RPQ_OK || d.status == RPQ_EOVERFLOW) ++s->res_completed;
            finish_job(s, j, d.status, end);
        }
        if (!done.empty()) s->cv_done.notify_all();
    }
    lk.unlock();
    if (have_stream) (void)hipStreamDestroy(stream);
}

// Whether a request goes to the resident engine: dense RPQs without reversal or length bound,
// whose automaton and source count the engine takes.
bool route_resident(const rpq_server* s, const rpq_request* r) {
    if (!s->res || r->kind != RPQ_REQ_RPQ) return false;
    if (r->flags & ~(RPQ_PAIRS | RPQ_PER_SOURCE | RPQ_ALL_SOURCES)) return false;
    rpq::ResidentQuery q{};
    q.nfa = r->nfa;
    q.n_sources = (r->flags & RPQ_ALL_SOURCES) && r->n_sources == 0 ? s->g->V : r->n_sources;
    q.pairs = (r->flags & RPQ_PAIRS) ? r->pairs : nullptr;
    if (s->res_max_units && (q.n_sources + s->res_width - 1) / s->res_width > s->res_max_units) return false;
    return rpq::resident_fits(s->res, q);
}

int check_request(rpq_server* s, const rpq_request* r) {
    if (r->kind == RPQ_REQ_RPQ) {
        if (r->flags & ~(RPQ_PAIRS | RPQ_PER_SOURCE | RPQ_ALL_SOURCES | RPQ_REVERSE | RPQ_SPARSE)) {
            rpq::set_error("unknown rpq flags 0x%x", r->flags);
            return RPQ_EINVAL;
        }
        uint64_t ws = 0;
        const uint64_t n = (r->flags & RPQ_ALL_SOURCES) && r->n_sources == 0 ? s->g->V : r->n_sources;
        return rpq_eval_workspace_size(s->g, &r->nfa, n, r->flags, nullptr, &ws);   // validates the automaton
    }
    if (r->kind == RPQ_REQ_CRPQ) {
        if (!r->atoms && r->n_atoms) {
            rpq::set_error("atoms is NULL");
            return RPQ_EINVAL;
        }
        if (r->vars.n_vars == 0 || r->vars.n_vars > CRPQ_MAX_VARS || r->n_atoms > CRPQ_MAX_ATOMS) {
            rpq::set_error("n_vars must be 1..%d and n_atoms at most %d", CRPQ_MAX_VARS, CRPQ_MAX_ATOMS);
            return RPQ_EINVAL;
        }
        return RPQ_OK;
    }
    rpq::set_error("unknown request kind %u", r->kind);
    return RPQ_EINVAL;
}

}  // namespace

extern "C" {

int rpq_serve_start(rpq_graph_t g, const rpq_server_opts* opts, void* pool, uint64_t pool_bytes, rpq_server_t* out) {
    rpq::clear_error();
    if (!g || !out || !pool || (reinterpret_cast<uintptr_t>(pool) & (kAlign - 1)) || pool_bytes < kAlign) {
        rpq::set_error("graph, out and a 256-byte aligned pool of at least 256 bytes are required");
        return RPQ_EINVAL;
    }
    const uint32_t nw = (opts && opts->workers) ? opts->workers : 4;
    if (nw > 64) {
        rpq::set_error("at most 64 workers");
        return RPQ_EINVAL;
    }
    if (opts && opts->reserved) {
        rpq::set_error("reserved server options must be 0");
        return RPQ_EINVAL;
    }
    auto* s = new (std::nothrow) rpq_server();
    if (!s) {
        rpq::set_error("out of host memory");
        return RPQ_ENOMEM;
    }
    s->g = g;
    s->pool = reinterpret_cast<char*>(pool);
    s->alloc.reset(new PoolAlloc(pool_bytes & ~(kAlign - 1)));
    s->t0 = std::chrono::steady_clock::now();
    if (opts && opts->resident_slots) {
        const uint32_t W = opts->resident_width ? opts->resident_width : 64;
        const uint32_t Q = opts->resident_states ? opts->resident_states : 12;
        const uint32_t succ = opts->resident_succ ? opts->resident_succ : 4;
        s->res_iters = opts->resident_iters ? opts->resident_iters : 8;
        s->res_width = W;
        s->res_max_units = opts->resident_max_units;
        int rc = rpq::resident_bytes(g, W, opts->resident_slots, Q, succ, &s->res_bytes);
        if (rc == RPQ_OK && !s->alloc->alloc(s->res_bytes, &s->res_off)) {
            rpq::set_error("the resident engine needs %llu bytes; the pool has %llu",
                           (unsigned long long)s->res_bytes, (unsigned long long)s->alloc->size());
            rc = RPQ_ENOMEM;
        }
        hipStream_t st = nullptr;
        if (rc == RPQ_OK && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            rpq::set_error("stream creation failed");
            rc = RPQ_EDEVICE;
        }
        if (rc == RPQ_OK) rc = rpq::resident_create(g, W, opts->resident_slots, Q, succ, s->pool + s->res_off,
                                                    s->res_bytes, st, &s->res);
        if (st) (void)hipStreamDestroy(st);
        if (rc != RPQ_OK) {
            delete s;
            return rc;
        }
        s->res_slot_bytes = s->res_bytes / opts->resident_slots;
        s->driver = std::thread(driver_main, s);
    }
    for (uint32_t i = 0; i < nw; ++i) s->workers.emplace_back(worker_main, s);
    *out = s;
    return RPQ_OK;
}

int rpq_serve_submit(rpq_server_t s, const rpq_request* r, uint64_t* ticket) {
    rpq::clear_error();
    if (!s || !r || !ticket) {
        rpq::set_error("server, request and ticket must not be NULL");
        return RPQ_EINVAL;
    }
    RPQ_TRY(check_request(s, r));
    std::unique_ptr<Job> j(new (std::nothrow) Job());
    if (!j) {
        rpq::set_error("out of host memory");
        return RPQ_ENOMEM;
    }
    j->req = *r;
    // the part of the pool the workers can ever get (the resident engine holds the rest)
    const uint64_t pool = s->worker_pool();
    j->resident = route_resident(s, r);
    j->t.resident = j->resident ? 1 : 0;
    if (r->kind == RPQ_REQ_RPQ) {
        const uint64_t n = (r->flags & RPQ_ALL_SOURCES) && r->n_sources == 0 ? s->g->V : r->n_sources;
        if (r->flags & RPQ_SPARSE) {
            RPQ_TRY(rpq_eval_workspace_size(s->g, &r->nfa, n, r->flags, nullptr, &j->need));
            // room for the search to grow without a trip back through the queue
            j->need = std::max<uint64_t>(j->need, std::min<uint64_t>(pool / 16, 512ull << 20));
            if (j->need > pool) {
                rpq::set_error("sparse request needs %llu bytes; the pool has %llu", (unsigned long long)j->need,
                               (unsigned long long)pool);
                return RPQ_ENOMEM;
            }
        } else {
            RPQ_TRY(dense_plan(s->g, j.get(), pool));
        }
    } else {
        j->atoms.assign(r->atoms, r->atoms + r->n_atoms);
        const uint32_t nv = r->vars.n_vars;
        if (r->vars.binding) j->binding.assign(r->vars.binding, r->vars.binding + nv);
        if (r->vars.vertex_label) j->vlabel.assign(r->vars.vertex_label, r->vars.vertex_label + nv);
        if (r->vars.domain) {
            j->domain.assign(r->vars.domain, r->vars.domain + nv);
            if (r->vars.domain_size) j->domain_size.assign(r->vars.domain_size, r->vars.domain_size + nv);
            else j->domain_size.assign(nv, 0);
        }
        if (r->vars.n_neq) {
            if (!r->vars.neq) {
                rpq::set_error("neq is NULL");
                return RPQ_EINVAL;
            }
            j->neq.assign(r->vars.neq, r->vars.neq + 2 * r->vars.n_neq);
        }
        // start with the domain bitmaps and a margin; the call asks for more if it needs it
        j->need = std::min<uint64_t>(pool, (uint64_t)(nv + 8) * ((s->g->V + 63) / 64) * 8 * 4 + (64ull << 20));
    }
    std::lock_guard<std::mutex> lk(s->mu);
    j->id = s->jobs.size();
    j->t.arrival_ms = r->arrival_ms >= 0 ? r->arrival_ms : s->now_ms();
    *ticket = j->id;
    if (j->resident) {
        s->res_queue.push_back(j.get());
        s->cv_res.notify_one();
    } else {
        s->queue.push_back(j.get());
        s->cv_work.notify_one();
    }
    s->jobs.push_back(std::move(j));
    return RPQ_OK;
}

int rpq_serve_poll(rpq_server_t s, uint64_t ticket, rpq_ticket* out) {
    rpq::clear_error();
    if (!s || !out) {
        rpq::set_error("server and out must not be NULL");
        return RPQ_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (ticket >= s->jobs.size()) {
        rpq::set_error("unknown ticket %llu", (unsigned long long)ticket);
        return RPQ_EINVAL;
    }
    *out = s->jobs[ticket]->t;
    return RPQ_OK;
}

int rpq_serve_wait(rpq_server_t s, uint64_t ticket, rpq_ticket* out) {
    rpq::clear_error();
    if (!s || !out) {
        rpq::set_error("server and out must not be NULL");
        return RPQ_EINVAL;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (ticket >= s->jobs.size()) {
        rpq::set_error("unknown ticket %llu", (unsigned long long)ticket);
        return RPQ_EINVAL;
    }
    Job* j = s->jobs[ticket].get();
    s->cv_done.wait(lk, [&] { return j->t.done != 0; });
    *out = j->t;
    return RPQ_OK;
}

int rpq_serve_clock_ms(rpq_server_t s, double* out) {
    if (!s || !out) {
        rpq::set_error("server and out must not be NULL");
        return RPQ_EINVAL;
    }
    *out = s->now_ms();
    return RPQ_OK;
}

int rpq_serve_stats(rpq_server_t s, rpq_server_stats* out) {
    rpq::clear_error();
    if (!s || !out) {
        rpq::set_error("server and out must not be NULL");
        return RPQ_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->jobs.size();
    out->completed = s->completed;
    out->failed = s->failed;
    out->queued = s->queue.size() + s->res_queue.size();
    out->running = s->running + s->res_running;
    out->pool_bytes = s->alloc->size();
    out->pool_in_use = s->alloc->used();
    out->pool_peak = s->alloc->peak();
    out->product_edges = s->eprod;
    out->resident_completed = s->res_completed;
    out->resident_launches = s->res_launches;
    out->resident_bytes = s->res ? s->res_bytes : 0;
    return RPQ_OK;
}

int rpq_serve_stop(rpq_server_t s) {
    rpq::clear_error();
    if (!s) return RPQ_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cv_work.notify_all();
        s->cv_res.notify_all();
    }
    if (s->driver.joinable()) s->driver.join();
    for (auto& t : s->workers) t.join();
    rpq::resident_destroy(s->res);
    delete s;
    return RPQ_OK;
}

}  // extern "C"
