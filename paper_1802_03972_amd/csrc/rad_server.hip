// Serving loop for per-step particle chunks of several independent bunches.
//
// Clients submit chunks (one time step of one bunch: particles in HOST memory plus the
// bunch's grid).  A scheduler thread
//   1. admits pending chunks in arrival order while the device chunk pool (the HBM budget)
//      has room: it reserves the chunk's bytes and starts the host-to-device copy on a copy
//      stream;
//   2. forms a batch from every admitted chunk whose copy has finished (up to max_batch)
//      and launches it with one batched persistent launch on the compute stream, while
//      earlier batches may still run (up to max_inflight batches are queued on the device);
//   3. retires batches whose completion event has fired: stamps each chunk complete, frees
//      its pool bytes (which lets new chunks in) and wakes waiters.
// Chunks are never dropped: a chunk larger than the whole budget is rejected at submit,
// every other chunk waits until it fits.  Results equal those of pushing each chunk on its
// own up to FP32 rounding of partial sums.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rad.h"
#include "rad_internal.h"

namespace {

int srv_fail(int code, const std::string& msg)
{
    rad::set_last_error(msg.c_str());
    return code;
}

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, capacity) with coalescing of free ranges.
class PoolAllocator {
public:
    void reset(size_t cap)
    {
        free_.clear();
        if (cap) free_[0] = cap;
        cap_ = cap;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
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
    size_t used() const { return used_; }
    size_t capacity() const { return cap_; }

private:
    std::map<size_t, size_t> free_;
    size_t cap_ = 0, used_ = 0;
};

constexpr size_t kFieldAlign = 256;

size_t align256(size_t x) { return (x + kFieldAlign - 1) / kFieldAlign * kFieldAlign; }

}  // namespace

struct rad_server {
    rad_server_config cfg{};
    rad_batcher* batcher = nullptr;
    hipStream_t copy_stream = nullptr, compute_stream = nullptr;
    unsigned char* pool = nullptr;
    PoolAllocator alloc;

    struct Chunk {
        uint64_t ticket = 0;
        rad_grid* grid = nullptr;
        double t = 0;
        int64_t n = 0;
        rad_particles host{};
        size_t elem = 0, bytes = 0, off = 0;
        hipEvent_t copied = nullptr;
        rad_chunk_stats st{};
        bool done = false;
    };
    struct Batch {
        std::vector<uint64_t> tickets;
        hipEvent_t done = nullptr;
    };

    std::mutex mu;
    std::condition_variable cv_client, cv_sched;
    std::deque<uint64_t> pending, admitted;
    std::deque<Batch> inflight;
    std::unordered_map<uint64_t, Chunk> chunks;
    std::vector<hipEvent_t> event_pool;
    uint64_t next_ticket = 1;
    bool stop = false;
    int error = RAD_OK;
    std::string error_msg;
    rad_server_counters counters{};
    double t0 = 0;
    std::thread worker;

    hipEvent_t take_event()
    {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }

    void set_error(int code, const std::string& msg)
    {
        if (error == RAD_OK) {
            error = code;
            error_msg = msg;
        }
    }

    // Called with mu held.
    void admit()
    {
        while (!pending.empty()) {
            Chunk& c = chunks[pending.front()];
            if ((int)admitted.size() >= cfg.max_admitted) break;
            size_t off = 0;
            if (!alloc.alloc(c.bytes, &off)) break;  // arrival order: wait for room
            c.off = off;
            c.copied = take_event();
            const void* src[10] = {c.host.x, c.host.y, c.host.z, c.host.bx, c.host.by, c.host.bz,
                                   c.host.dbx, c.host.dby, c.host.dbz, c.host.w};
            for (int f = 0; f < 10; ++f) {
                hipError_t e = hipMemcpyAsync(pool + off + f * align256(c.elem * c.n), src[f], c.elem * c.n,
                                              hipMemcpyHostToDevice, copy_stream);
                if (e != hipSuccess) set_error(RAD_ERR_DEVICE, std::string("chunk copy: ") + hipGetErrorString(e));
            }
            if (!c.copied || hipEventRecord(c.copied, copy_stream) != hipSuccess)
                set_error(RAD_ERR_DEVICE, "cannot record chunk copy event");
            c.st.t_admit = now_s() - t0;
            admitted.push_back(c.ticket);
            pending.pop_front();
            counters.admitted += 1;
        }
    }

    // Called with mu held.  Launches one batch of copied chunks if there is room.
    bool launch()
    {
        if ((int)inflight.size() >= cfg.max_inflight || admitted.empty()) return false;
        std::vector<uint64_t> ready;
        std::vector<rad_batch_item> items;
        for (auto it = admitted.begin(); it != admitted.end() && (int)ready.size() < cfg.max_batch;) {
            Chunk& c = chunks[*it];
            const hipError_t q = hipEventQuery(c.copied);
            if (q == hipErrorNotReady) break;  // copies complete in order
            if (q != hipSuccess) set_error(RAD_ERR_DEVICE, std::string("chunk copy event: ") + hipGetErrorString(q));
            rad_batch_item bi{};
            bi.grid = c.grid;
            bi.t0 = c.t;
            bi.n_steps = 1;
            bi.n_particles = c.n;
            bi.p.dtype = c.host.dtype;
            const void** dst[10] = {&bi.p.x, &bi.p.y, &bi.p.z, &bi.p.bx, &bi.p.by, &bi.p.bz,
                                    &bi.p.dbx, &bi.p.dby, &bi.p.dbz, &bi.p.w};
            for (int f = 0; f < 10; ++f) *dst[f] = pool + c.off + f * align256(c.elem * c.n);
            items.push_back(bi);
            ready.push_back(*it);
            it = admitted.erase(it);
        }
        if (ready.empty()) return false;
        const double tl = now_s() - t0;
        int rc = rad_batcher_push(batcher, items.data(), (int32_t)items.size(), compute_stream);
        Batch b;
        b.tickets = ready;
        b.done = take_event();
        if (rc != RAD_OK) set_error(rc, std::string("batched launch: ") + rad_last_error());
        if (!b.done || hipEventRecord(b.done, compute_stream) != hipSuccess)
            set_error(RAD_ERR_DEVICE, "cannot record batch event");
        counters.batches += 1;
        for (uint64_t tk : ready) {
            Chunk& c = chunks[tk];
            c.st.t_launch = tl;
            c.st.batch_size = (int32_t)ready.size();
            c.st.batch_id = counters.batches;
        }
        counters.chunks_launched += (int64_t)ready.size();
        inflight.push_back(std::move(b));
        return true;
    }

    // Called with mu held.
    bool retire()
    {
        bool any = false;
        while (!inflight.empty()) {
            Batch& b = inflight.front();
            const hipError_t q = b.done ? hipEventQuery(b.done) : hipSuccess;
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) set_error(RAD_ERR_DEVICE, std::string("batch event: ") + hipGetErrorString(q));
            const double tc = now_s() - t0;
            for (uint64_t tk : b.tickets) {
                Chunk& c = chunks[tk];
                c.st.t_complete = tc;
                c.st.status = error;
                c.done = true;
                alloc.release(c.off, c.bytes);
                if (c.copied) event_pool.push_back(c.copied);
                c.copied = nullptr;
                counters.completed += 1;
            }
            if (b.done) event_pool.push_back(b.done);
            inflight.pop_front();
            any = true;
        }
        return any;
    }

    void run()
    {
        (void)hipSetDevice(cfg.device);
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            const bool retired = retire();
            admit();
            const bool launched = launch();
            if (retired) cv_client.notify_all();
            if (stop && pending.empty() && admitted.empty() && inflight.empty()) break;
            if (!launched && !retired) {
                // nothing moved: wait briefly for a submit, a copy or a batch to finish
                cv_sched.wait_for(lk, std::chrono::microseconds(cfg.poll_us));
            }
        }
        cv_client.notify_all();
    }
};

extern "C" {

int rad_server_create(rad_server** out, const rad_server_config* cfg)
{
    if (!out || !cfg) return srv_fail(RAD_ERR_INVALID_ARG, "out and cfg must be non-NULL");
    if (cfg->hbm_budget < (1u << 20)) return srv_fail(RAD_ERR_INVALID_ARG, "hbm_budget must be >= 1 MiB");
    if (cfg->max_batch < 1 || cfg->max_inflight < 1 || cfg->max_admitted < 1 || cfg->poll_us < 1)
        return srv_fail(RAD_ERR_INVALID_ARG, "max_batch, max_inflight, max_admitted and poll_us must be >= 1");
    rad_server* s = new rad_server;
    s->cfg = *cfg;
    // one batch running and one queued keep the compute stream busy; the batcher recycles
    // its two plan buffers under that bound without blocking
    s->cfg.max_inflight = std::min(cfg->max_inflight, 2);
    if (hipSetDevice(cfg->device) != hipSuccess) {
        delete s;
        return srv_fail(RAD_ERR_INVALID_ARG, "bad device");
    }
    int rc = rad_batcher_create(&s->batcher, cfg->device, cfg->max_batch);
    if (rc == RAD_OK && cfg->use_graph) rc = rad_batcher_set_graph(s->batcher, 1);
    if (rc != RAD_OK) {
        if (s->batcher) rad_batcher_destroy(s->batcher);
        delete s;
        return srv_fail(rc, std::string("batcher: ") + rad_last_error());
    }
    if (hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->compute_stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc((void**)&s->pool, cfg->hbm_budget) != hipSuccess) {
        if (s->pool) (void)hipFree(s->pool);
        if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
        if (s->compute_stream) (void)hipStreamDestroy(s->compute_stream);
        rad_batcher_destroy(s->batcher);
        delete s;
        return srv_fail(RAD_ERR_OOM, "cannot allocate the server's streams or chunk pool");
    }
    s->alloc.reset(cfg->hbm_budget);
    s->t0 = now_s();
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return RAD_OK;
}

int rad_server_submit(rad_server* s, rad_grid* g, double t, int64_t n, const rad_particles* host_p,
                      uint64_t* ticket)
{
    if (!s || !g || !host_p || !ticket) return srv_fail(RAD_ERR_INVALID_ARG, "NULL argument");
    if (n < 1) return srv_fail(RAD_ERR_INVALID_ARG, "a chunk needs n >= 1 particles");
    if (host_p->dtype != RAD_F32 && host_p->dtype != RAD_F64) return srv_fail(RAD_ERR_INVALID_ARG, "bad dtype");
    const void* f[10] = {host_p->x, host_p->y, host_p->z, host_p->bx, host_p->by, host_p->bz,
                         host_p->dbx, host_p->dby, host_p->dbz, host_p->w};
    for (const void* p : f)
        if (!p) return srv_fail(RAD_ERR_INVALID_ARG, "a particle field is NULL");
    rad_server::Chunk c;
    c.grid = g;
    c.t = t;
    c.n = n;
    c.host = *host_p;
    c.elem = host_p->dtype == RAD_F32 ? 4 : 8;
    c.bytes = 10 * align256(c.elem * (size_t)n);
    if (c.bytes > s->cfg.hbm_budget)
        return srv_fail(RAD_ERR_INVALID_ARG, "chunk larger than the whole HBM budget");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return srv_fail(RAD_ERR_INVALID_ARG, "server is stopping");
        if ((int64_t)s->pending.size() >= s->cfg.max_pending)
            return srv_fail(RAD_ERR_QUEUE_FULL, "pending queue full");
        c.ticket = s->next_ticket++;
        c.st.t_submit = now_s() - s->t0;
        *ticket = c.ticket;
        s->chunks.emplace(c.ticket, c);
        s->pending.push_back(c.ticket);
        s->counters.submitted += 1;
    }
    s->cv_sched.notify_one();
    return RAD_OK;
}

int rad_server_poll(rad_server* s, uint64_t ticket, rad_chunk_stats* st)
{
    if (!s) return srv_fail(RAD_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->chunks.find(ticket);
    if (it == s->chunks.end()) return srv_fail(RAD_ERR_INVALID_ARG, "unknown ticket");
    if (!it->second.done) return 0;
    if (st) *st = it->second.st;
    s->chunks.erase(it);
    return 1;
}

int rad_server_wait(rad_server* s, uint64_t ticket, rad_chunk_stats* st)
{
    if (!s) return srv_fail(RAD_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->chunks.find(ticket);
    if (it == s->chunks.end()) return srv_fail(RAD_ERR_INVALID_ARG, "unknown ticket");
    // a ticket collected meanwhile by another waiter counts as unknown
    s->cv_client.wait(lk, [&] {
        auto f = s->chunks.find(ticket);
        return f == s->chunks.end() || f->second.done;
    });
    it = s->chunks.find(ticket);
    if (it == s->chunks.end()) return srv_fail(RAD_ERR_INVALID_ARG, "ticket collected by another caller");
    if (st) *st = it->second.st;
    const int status = it->second.st.status;
    s->chunks.erase(it);
    return status == RAD_OK ? 1 : status;
}

int rad_server_drain(rad_server* s)
{
    if (!s) return srv_fail(RAD_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_sched.notify_one();
    s->cv_client.wait(lk, [&] { return s->pending.empty() && s->admitted.empty() && s->inflight.empty(); });
    if (s->error != RAD_OK) return srv_fail(s->error, s->error_msg);
    return RAD_OK;
}

int rad_server_counters_read(rad_server* s, rad_server_counters* out)
{
    if (!s || !out) return srv_fail(RAD_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->counters;
    out->pending = (int64_t)s->pending.size();
    out->admitted_waiting = (int64_t)s->admitted.size();
    out->inflight_batches = (int64_t)s->inflight.size();
    out->pool_used = s->alloc.used();
    out->now = now_s() - s->t0;
    return RAD_OK;
}

int rad_server_set_tile(rad_server* s, const rad_tile* t)
{
    if (!s) return srv_fail(RAD_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);   // the scheduler pushes batches under this lock
    return rad_batcher_set_tile(s->batcher, t);
}

int rad_server_get_tile(rad_server* s, rad_tile* t)
{
    if (!s || !t) return srv_fail(RAD_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    return rad_batcher_get_tile(s->batcher, t);
}

int rad_server_profile_enable(rad_server* s, int enable)
{
    if (!s) return srv_fail(RAD_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);   // the scheduler pushes batches under this lock
    return rad_batcher_profile_enable(s->batcher, enable);
}

int rad_server_profile_read(rad_server* s, rad_profile_stats* out)
{
    if (!s || !out) return srv_fail(RAD_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    return rad_batcher_profile_read(s->batcher, out);
}

int rad_server_destroy(rad_server* s)
{
    if (!s) return RAD_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_sched.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->cfg.device);
    (void)hipStreamSynchronize(s->compute_stream);
    (void)hipStreamSynchronize(s->copy_stream);
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    for (auto& kv : s->chunks)
        if (kv.second.copied) (void)hipEventDestroy(kv.second.copied);
    (void)hipFree(s->pool);
    (void)hipStreamDestroy(s->copy_stream);
    (void)hipStreamDestroy(s->compute_stream);
    rad_batcher_destroy(s->batcher);
    delete s;
    return RAD_OK;
}

}  // extern "C"
