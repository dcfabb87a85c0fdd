// mpm_serve.hip -- request queue with continuous batching (mpm_server_* in
// include/mpm.h).
//
// Admitted fits each own one of the server's streams; every step enqueues the
// next piece of every admitted fit (at most DEPTH pieces in flight per fit),
// so fits of different sizes and modes overlap on the device and a new
// arrival starts as soon as a stream and enough of the memory budget are free.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mpm_api_internal.h"

using namespace mpm;

namespace {

constexpr int DEPTH = 2;  // pieces of one fit in flight at a time

// A MAP fit of at least this many voxels fills the device by itself for a long
// time (each of its ~13,000 kernels runs several rounds of workgroups on every
// CU): two such fits side by side only share the bandwidth and both finish
// later.  At most one of them runs at a time (FIFO among them); ML fits (one
// short launch) and smaller MAP fits fill the gaps around it.
constexpr int64_t LARGE_FIT_VOXELS = (int64_t)1 << 21;

enum State { QUEUED = 0, RUNNING = 1, DONE = 2 };

struct Entry {
    uint64_t ticket;
    mpm_request req;
    int64_t N = 0;
    size_t footprint = 0;
    State state = QUEUED;
    int stream = -1;
    FitArgs args;
    std::unique_ptr<Workspace> ws;
    std::unique_ptr<Prof> prof;
    std::unique_ptr<FitJob> job;
    std::deque<hipEvent_t> inflight;
    bool all_enqueued = false;
    bool cancel = false;  // no further pieces; released once those in flight complete
    mpm_status status = MPM_OK;
    std::string error;
    mpm_report report;
};

bool is_large(const Entry &e) { return e.req.options.mode == MPM_MAP_JTV && e.N >= LARGE_FIT_VOXELS; }

}  // namespace

struct mpm_server {
    size_t budget = 0, used = 0;
    int device = 0;
    std::vector<hipStream_t> streams;
    std::vector<uint64_t> owner;  // ticket running on each stream, 0 = free
    std::deque<uint64_t> queue;
    std::map<uint64_t, std::unique_ptr<Entry>> entries;
    uint64_t next_ticket = 1;
    std::mutex mu;
    std::thread worker;
    std::atomic<bool> stop{false};
};

namespace {

void release(mpm_server *s, Entry &e)
{
    for (hipEvent_t ev : e.inflight) (void)hipEventDestroy(ev);
    e.inflight.clear();
    e.job.reset();
    e.ws.reset();  // frees the workspace on the fit's stream and waits for it
    e.prof.reset();
    if (e.stream >= 0) s->owner[e.stream] = 0;
    e.stream = -1;
    s->used -= e.footprint;
}

void finish_failed(mpm_server *s, Entry &e, mpm_status st)
{
    e.status = st;
    e.error = mpm_last_error();
    if (e.state == RUNNING) release(s, e);
    e.state = DONE;
}

// Enqueue the next piece of a running fit if fewer than DEPTH are in flight.
void advance(mpm_server *s, Entry &e)
{
    while (!e.inflight.empty() && hipEventQuery(e.inflight.front()) == hipSuccess) {
        (void)hipEventDestroy(e.inflight.front());
        e.inflight.pop_front();
    }
    if (e.cancel) {
        if (!e.inflight.empty()) return;
        release(s, e);
        e.status = MPM_ERR_CANCELLED;
        e.error = "cancelled while running";
        e.state = DONE;
        return;
    }
    if (e.all_enqueued) {
        if (!e.inflight.empty()) return;
        // every piece has completed
        e.prof->collect();
        e.status = e.job->collect(e.report, nullptr, 0);
        if (e.status) e.error = mpm_last_error();
        release(s, e);
        e.state = DONE;
        return;
    }
    if ((int)e.inflight.size() >= DEPTH) return;
    bool more = true;
    mpm_status st = e.job->enqueue_next(&more);
    if (st) {
        finish_failed(s, e, st);
        return;
    }
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ev, s->streams[e.stream]) != hipSuccess) {
        finish_failed(s, e, fail(MPM_ERR_DEVICE, "server: event record failed"));
        return;
    }
    e.inflight.push_back(ev);
    e.all_enqueued = !more;
}

mpm_status admit(mpm_server *s, Entry &e, int stream)
{
    hipStream_t hs = s->streams[stream];
    e.stream = stream;
    s->owner[stream] = e.ticket;
    s->used += e.footprint;
    e.state = RUNNING;
    e.args = FitArgs{&e.req.protocol, to_dev(&e.req.protocol), e.req.dtype, e.req.echoes, e.req.b1,
                     &e.req.options, e.req.maps, e.N, e.req.grid.nx, e.req.grid.ny, e.req.grid.nz, hs};
    e.ws.reset(new Workspace(hs));
    e.prof.reset(new Prof(hs));
    mpm_status st = MPM_OK;
    e.job = e.req.options.mode == MPM_ML ? make_ml_job(e.args, *e.ws, *e.prof, &st)
                                         : make_map_job(e.args, *e.ws, *e.prof, &st);
    return st;
}

void step_locked(mpm_server *s)
{
    // progress the running fits
    for (auto &kv : s->entries) {
        Entry &e = *kv.second;
        if (e.state == RUNNING) advance(s, e);
    }
    // admit in submission order; a large fit waits while another large one
    // runs and smaller ones may pass it, but none passes a fit that waits for
    // memory (so a large request cannot starve)
    int large_running = 0;
    for (auto &kv : s->entries)
        if (kv.second->state == RUNNING && is_large(*kv.second)) large_running++;
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Entry &e = *s->entries[*it];
        if (e.footprint > s->budget) {
            it = s->queue.erase(it);
            finish_failed(s, e, fail(MPM_ERR_OUT_OF_MEMORY, "request needs %zu bytes, server budget is %zu",
                                     e.footprint, s->budget));
            continue;
        }
        const bool large = is_large(e);
        if (large && large_running > 0) {
            ++it;
            continue;
        }
        int free_stream = -1;
        for (size_t i = 0; i < s->owner.size(); i++)
            if (!s->owner[i]) {
                free_stream = (int)i;
                break;
            }
        if (free_stream < 0 || s->used + e.footprint > s->budget) break;
        it = s->queue.erase(it);
        mpm_status st = admit(s, e, free_stream);
        if (st) {
            finish_failed(s, e, st);
            continue;
        }
        if (large) large_running++;
        advance(s, e);
    }
}

int pending_locked(mpm_server *s)
{
    int n = 0;
    for (auto &kv : s->entries)
        if (kv.second->state != DONE) n++;
    return n;
}

void worker_loop(mpm_server *s)
{
    (void)hipSetDevice(s->device);
    while (!s->stop.load()) {
        int pending;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            step_locked(s);
            pending = pending_locked(s);
        }
        std::this_thread::sleep_for(std::chrono::microseconds(pending ? 20 : 500));
    }
}

}  // namespace

extern "C" {

mpm_status mpm_server_create(size_t hbm_budget, int32_t max_active, int32_t flags, mpm_server **out)
{
    clear_error();
    if (!out) return fail(MPM_ERR_INVALID_ARG, "out is NULL");
    if (max_active < 1 || max_active > 64) return fail(MPM_ERR_INVALID_ARG, "max_active must be in [1, 64]");
    if (flags & ~MPM_SERVER_THREAD) return fail(MPM_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (hbm_budget == 0) return fail(MPM_ERR_INVALID_ARG, "hbm_budget must be > 0");
    std::unique_ptr<mpm_server> s(new mpm_server);
    s->budget = hbm_budget;
    if (hipGetDevice(&s->device) != hipSuccess) return fail(MPM_ERR_DEVICE, "no HIP device");
    for (int i = 0; i < max_active; i++) {
        hipStream_t hs;
        if (hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
            return fail(MPM_ERR_DEVICE, "stream creation failed");
        }
        s->streams.push_back(hs);
    }
    s->owner.assign(max_active, 0);
    if (flags & MPM_SERVER_THREAD) s->worker = std::thread(worker_loop, s.get());
    *out = s.release();
    return MPM_OK;
}

mpm_status mpm_server_submit(mpm_server *s, const mpm_request *r, uint64_t *ticket)
{
    clear_error();
    if (!s || !r || !ticket) return fail(MPM_ERR_INVALID_ARG, "server, request and ticket must be non-NULL");
    int64_t N;
    mpm_status st = check_fit_args(&r->protocol, &r->grid, r->dtype, r->echoes, &r->options, r->maps, &N);
    if (st) return st;
    if (r->reserved != 0) return fail(MPM_ERR_INVALID_ARG, "reserved must be 0");
    std::unique_ptr<Entry> e(new Entry);
    e->req = *r;
    e->N = N;
    e->footprint = mpm_footprint_bytes(&r->protocol, &r->grid, (mpm_dtype)r->dtype, r->options.mode);
    memset(&e->report, 0, sizeof(e->report));
    std::lock_guard<std::mutex> lk(s->mu);
    e->ticket = s->next_ticket++;
    *ticket = e->ticket;
    s->queue.push_back(e->ticket);
    s->entries[e->ticket] = std::move(e);
    return MPM_OK;
}

mpm_status mpm_server_step(mpm_server *s, int32_t *pending)
{
    clear_error();
    if (!s) return fail(MPM_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    step_locked(s);
    if (pending) *pending = pending_locked(s);
    return MPM_OK;
}

mpm_status mpm_server_poll(mpm_server *s, uint64_t ticket, int32_t *done, mpm_report *report)
{
    clear_error();
    if (!s || !done) return fail(MPM_ERR_INVALID_ARG, "server and done must be non-NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->entries.find(ticket);
    if (it == s->entries.end()) return fail(MPM_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Entry &e = *it->second;
    *done = e.state == DONE;
    if (!*done) return MPM_OK;
    if (report) *report = e.report;
    if (e.status) return fail(e.status, "%s", e.error.c_str());
    return MPM_OK;
}

mpm_status mpm_server_cancel(mpm_server *s, uint64_t ticket)
{
    clear_error();
    if (!s) return fail(MPM_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->entries.find(ticket);
    if (it == s->entries.end()) return fail(MPM_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Entry &e = *it->second;
    if (e.state == QUEUED) {
        for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
            if (*q == ticket) {
                s->queue.erase(q);
                break;
            }
        e.status = MPM_ERR_CANCELLED;
        e.error = "cancelled before it started";
        e.state = DONE;
    } else if (e.state == RUNNING) {
        e.cancel = true;
    }
    return MPM_OK;
}

mpm_status mpm_server_destroy(mpm_server *s)
{
    clear_error();
    if (!s) return MPM_OK;
    if (s->worker.joinable()) {
        s->stop.store(true);
        s->worker.join();
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto &kv : s->entries) {
            Entry &e = *kv.second;
            if (e.state == RUNNING) {
                (void)hipStreamSynchronize(s->streams[e.stream]);
                release(s, e);
                e.state = DONE;
            }
        }
        for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
    }
    delete s;
    return MPM_OK;
}

}  // extern "C"
