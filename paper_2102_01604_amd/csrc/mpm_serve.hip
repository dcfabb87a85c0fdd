// mpm_serve.hip -- request queue with continuous batching (mpm_server_* in
// include/mpm.h).
//
// Admitted work runs on the server's streams: a fit alone, or a group of small
// JTV-MAP fits of one schedule fitted together with batched launches (every
// kernel launch serves all of them: a small volume's launches each cost about
// the device's dispatch latency, which the group then pays once).  Every step
// enqueues the next piece of every running unit (at most DEPTH pieces in
// flight per unit), so fits of different sizes and modes overlap on the
// device and a new arrival starts as soon as a stream and enough of the
// memory budget are free.
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

constexpr int DEPTH = 2;  // pieces of one unit in flight at a time

// A MAP fit of at least this many voxels fills the device by itself for a long
// time (each of its ~11,000 kernels runs several rounds of workgroups on every
// CU): two such fits side by side only share the bandwidth and both finish
// later.  At most one of them runs at a time (FIFO among them); ML fits (one
// short launch) and smaller MAP fits fill the gaps around it.
constexpr int64_t LARGE_FIT_VOXELS = (int64_t)1 << 21;

// Groups of small MAP fits.  Only fits of at most GROUP_FIT_VOXELS join groups:
// their CG sweeps last about as long as a launch's dispatch latency, which a
// group pays once for all its members; a fit of 96 x 128 x 128 voxels already
// streams its sweeps at nearly the bandwidth of the part (measured: 4 of them
// batched 1.03x faster than one after another, 16 of 64^3 1.50x).  A group
// holds fits whose sizes differ by at most 2x (it finishes with its largest
// member), at most GROUP_MAX_FITS fits and GROUP_MAX_VOXELS voxels in all
// (about what fills the device in one launch of the CG sweeps).
constexpr int64_t GROUP_FIT_VOXELS = (int64_t)1 << 19;
constexpr int GROUP_MAX_FITS = 16;
constexpr int64_t GROUP_MAX_VOXELS = (int64_t)1 << 22;

enum State { QUEUED = 0, RUNNING = 1, DONE = 2 };

struct Entry;

// What runs on one stream: one fit (job) or a group of fits (batch).
struct Unit {
    int stream = -1;
    std::vector<Entry *> members;
    std::vector<FitArgs> args;
    std::unique_ptr<Workspace> ws;
    std::unique_ptr<Prof> prof;
    std::unique_ptr<FitJob> job;
    std::unique_ptr<BatchJob> batch;
    std::deque<hipEvent_t> inflight;
    bool all_enqueued = false;
    bool cancel = false;  // no further pieces; released once those in flight complete
    size_t footprint = 0;
};

struct Entry {
    uint64_t ticket;
    mpm_request req;
    int64_t N = 0;
    size_t footprint = 0;
    State state = QUEUED;
    std::shared_ptr<Unit> unit;
    bool cancelled = false;  // cancelled while running in a group: finishes as cancelled
    mpm_status status = MPM_OK;
    std::string error;
    mpm_report report;
    float echo_offset[MPM_MAX_IMAGES];  // copy of the request's echo offsets (if any)
};

bool is_large(const Entry &e) { return e.req.options.mode == MPM_MAP_JTV && e.N >= LARGE_FIT_VOXELS; }
bool groupable(const Entry &e) { return e.req.options.mode == MPM_MAP_JTV && e.N <= GROUP_FIT_VOXELS; }

}  // namespace

struct mpm_server {
    size_t budget = 0, used = 0;
    int device = 0;
    int32_t flags = 0;
    std::vector<hipStream_t> streams;
    std::vector<bool> busy;  // stream in use
    std::deque<uint64_t> queue;
    std::map<uint64_t, std::unique_ptr<Entry>> entries;
    std::vector<std::shared_ptr<Unit>> units;
    uint64_t next_ticket = 1;
    std::mutex mu;
    std::thread worker;
    std::atomic<bool> stop{false};
};

namespace {

FitArgs args_of(Entry &e, hipStream_t hs)
{
    return FitArgs{&e.req.protocol, to_dev(&e.req.protocol, e.req.options.echo_offset), e.req.dtype, e.req.echoes,
                   e.req.b1, &e.req.options, e.req.maps, e.N, e.req.grid.nx, e.req.grid.ny, e.req.grid.nz, hs};
}

void release(mpm_server *s, Unit &u)
{
    for (hipEvent_t ev : u.inflight) (void)hipEventDestroy(ev);
    u.inflight.clear();
    // the workspace first: freeing it waits for the unit's stream, so pieces
    // still in flight after an error have ended before the jobs' pinned
    // staging buffers go
    u.ws.reset();
    u.job.reset();
    u.batch.reset();
    u.prof.reset();
    if (u.stream >= 0) s->busy[u.stream] = false;
    u.stream = -1;
    s->used -= u.footprint;
    u.footprint = 0;
}

void finish(Entry &e, mpm_status st, const std::string &msg)
{
    e.status = st;
    e.error = msg;
    e.state = DONE;
    e.unit.reset();
}

void finish_unit(mpm_server *s, Unit &u, mpm_status st)
{
    const std::string msg = mpm_last_error();
    release(s, u);
    for (Entry *e : u.members) finish(*e, st, msg);
}

// Enqueue the next piece of a running unit if fewer than DEPTH are in flight;
// finish its fits once every piece has completed.  Returns false once done.
bool advance(mpm_server *s, Unit &u)
{
    while (!u.inflight.empty() && hipEventQuery(u.inflight.front()) == hipSuccess) {
        (void)hipEventDestroy(u.inflight.front());
        u.inflight.pop_front();
    }
    if (u.cancel) {
        if (!u.inflight.empty()) return true;
        release(s, u);
        for (Entry *e : u.members) finish(*e, MPM_ERR_CANCELLED, "cancelled while running");
        return false;
    }
    if (u.all_enqueued) {
        if (!u.inflight.empty()) return true;
        // every piece has completed
        u.prof->collect();
        for (size_t i = 0; i < u.members.size(); i++) {
            Entry &e = *u.members[i];
            mpm_status st = u.batch ? u.batch->collect_item((int)i, e.report, nullptr, 0)
                                    : u.job->collect(e.report, nullptr, 0);
            if (e.cancelled) finish(e, MPM_ERR_CANCELLED, "cancelled while running");
            else finish(e, st, st ? mpm_last_error() : "");
        }
        release(s, u);
        return false;
    }
    if ((int)u.inflight.size() >= DEPTH) return true;
    // the default initialisation's image means are still on their way to the
    // host: come back on a later step instead of waiting under the lock
    if (!(u.batch ? u.batch->ready() : u.job->ready())) return true;
    bool more = true;
    mpm_status st = u.batch ? u.batch->enqueue_next(&more) : u.job->enqueue_next(&more);
    if (st) {
        finish_unit(s, u, st);
        return false;
    }
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ev, s->streams[u.stream]) != hipSuccess) {
        fail(MPM_ERR_DEVICE, "server: event record failed");
        finish_unit(s, u, MPM_ERR_DEVICE);
        return false;
    }
    u.inflight.push_back(ev);
    u.all_enqueued = !more;
    return true;
}

// Start a unit of fits on a free stream.
void start_unit(mpm_server *s, std::vector<Entry *> members, int stream)
{
    std::shared_ptr<Unit> u(new Unit);
    hipStream_t hs = s->streams[stream];
    u->stream = stream;
    u->members = members;
    s->busy[stream] = true;
    for (Entry *e : members) {
        u->footprint += e->footprint;
        e->state = RUNNING;
        e->unit = u;
        u->args.push_back(args_of(*e, hs));
    }
    s->used += u->footprint;
    u->ws.reset(new Workspace(hs));
    u->prof.reset(new Prof(hs));
    mpm_status st = MPM_OK;
    if (members.size() > 1)
        u->batch = make_batch_job(u->args, *u->ws, *u->prof, &st);
    else
        u->job = members[0]->req.options.mode == MPM_ML ? make_ml_job(u->args[0], *u->ws, *u->prof, &st)
                                                         : make_map_job(u->args[0], *u->ws, *u->prof, &st);
    if (st) {
        finish_unit(s, *u, st);
        return;
    }
    s->units.push_back(u);
    advance(s, *u);
}

void step_locked(mpm_server *s)
{
    // progress the running units
    for (size_t i = 0; i < s->units.size();) {
        if (advance(s, *s->units[i])) i++;
        else s->units.erase(s->units.begin() + (long)i);
    }
    // admit in submission order; a large fit waits while another large one
    // runs and smaller ones may pass it, but none passes a fit that waits for
    // memory (so a large request cannot starve)
    int large_running = 0;
    for (auto &u : s->units)
        for (Entry *e : u->members)
            if (is_large(*e)) large_running++;
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Entry &e = *s->entries[*it];
        if (e.footprint > s->budget) {
            it = s->queue.erase(it);
            const mpm_status st = fail(MPM_ERR_OUT_OF_MEMORY, "request needs %zu bytes, server budget is %zu",
                                       e.footprint, s->budget);
            finish(e, st, mpm_last_error());
            continue;
        }
        const bool large = is_large(e);
        if (large && large_running > 0) {
            ++it;
            continue;
        }
        int free_stream = -1;
        for (size_t i = 0; i < s->busy.size(); i++)
            if (!s->busy[i]) {
                free_stream = (int)i;
                break;
            }
        if (free_stream < 0 || s->used + e.footprint > s->budget) break;
        std::vector<Entry *> group{&e};
        it = s->queue.erase(it);
        if (groupable(e) && !(s->flags & MPM_SERVER_NO_GROUPS)) {
            // (erasing from the queue invalidates its iterators: the scan restarts below)
            // later small MAP fits that can share launches with this one join it
            FitArgs a0 = args_of(e, nullptr);
            int64_t vox = e.N;
            size_t mem = s->used + e.footprint;
            for (auto jt = it; jt != s->queue.end() && (int)group.size() < GROUP_MAX_FITS;) {
                Entry &f = *s->entries[*jt];
                const bool similar = f.N <= 2 * e.N && e.N <= 2 * f.N;
                if (groupable(f) && similar && vox + f.N <= GROUP_MAX_VOXELS && mem + f.footprint <= s->budget &&
                    batch_compatible(a0, args_of(f, nullptr))) {
                    group.push_back(&f);
                    vox += f.N;
                    mem += f.footprint;
                    jt = s->queue.erase(jt);
                } else {
                    ++jt;
                }
            }
            it = s->queue.begin();  // the queue changed: restart the scan
        }
        if (large) large_running++;
        start_unit(s, group, free_stream);
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
    if (flags & ~(MPM_SERVER_THREAD | MPM_SERVER_NO_GROUPS))
        return fail(MPM_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (hbm_budget == 0) return fail(MPM_ERR_INVALID_ARG, "hbm_budget must be > 0");
    std::unique_ptr<mpm_server> s(new mpm_server);
    s->budget = hbm_budget;
    s->flags = flags;
    if (hipGetDevice(&s->device) != hipSuccess) return fail(MPM_ERR_DEVICE, "no HIP device");
    for (int i = 0; i < max_active; i++) {
        hipStream_t hs;
        if (hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
            return fail(MPM_ERR_DEVICE, "stream creation failed");
        }
        s->streams.push_back(hs);
    }
    s->busy.assign(max_active, false);
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
    if (r->options.echo_offset) {  // the request keeps its own copy
        memcpy(e->echo_offset, r->options.echo_offset, sizeof(float) * (size_t)n_images(&r->protocol));
        e->req.options.echo_offset = e->echo_offset;
    }
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
        finish(e, MPM_ERR_CANCELLED, "cancelled before it started");
    } else if (e.state == RUNNING) {
        e.cancelled = true;
        bool all = true;  // a unit whose fits are all cancelled stops
        for (Entry *m : e.unit->members) all = all && m->cancelled;
        if (all) e.unit->cancel = true;
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
        for (auto &u : s->units) {
            (void)hipStreamSynchronize(s->streams[u->stream]);
            release(s, *u);
            for (Entry *e : u->members) finish(*e, MPM_ERR_CANCELLED, "server destroyed");
        }
        s->units.clear();
        for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
    }
    delete s;
    return MPM_OK;
}

}  // extern "C"
