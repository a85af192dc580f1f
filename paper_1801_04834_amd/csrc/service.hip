// Streaming service: ~1 s blocks from several concurrent observations through the FX chain.
//
// Memory.  The service allocates its whole HBM budget once, as one device arena, and carves
// each observation's working set (plan workspace, one device input block, one visibility
// buffer) out of it with a first-fit free list that merges neighbouring free ranges; closing
// an observation returns its range.  The paper's pipeline likewise allocates its buffers once
// and recycles them through pools of free blocks ("Software architecture", sec. 7.1).
//
// Admission.  An observation whose working set fits is admitted at once.  One that does not
// fit now (but would fit the empty arena) waits in a FIFO of pending observations and is
// admitted as soon as closes free enough of the arena, in arrival order; its blocks queue in
// the meantime.
//
// Continuous batching.  n_slots worker threads, each with its own stream, take the next
// queued block of any admitted observation that has no block on the device (round robin over
// observations) and run it: host -> device copy, cobalt_correlate, device -> host copy, wait
// for the stream.  Blocks of different observations therefore overlap on the device while
// each observation's blocks run in arrival order, one at a time (the FIR history carries from
// block to block).  A full per-observation FIFO drops the new block rather than stalling the
// producer, as the paper's pipeline drops data instead of waiting ("Dealing with jitter and
// hardware failure", sec. 7.2); bounded queues with condition variables mirror its task
// pipeline ("Parallelization libraries", sec. 7.4).  Latency is measured from submit to the
// completion of the block's device-to-host visibility copy.
//
// Locking.  One mutex guards the service's tables; it is never held across a HIP call, so a
// slow (e.g. pageable) host copy in one worker holds up neither submits nor other workers.
// Observations are held by pointer (their addresses never move) and tickets are looked up
// by id after every wait.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/cobalt.h"
#include "cobalt_internal.h"

namespace {

using clock_type = std::chrono::steady_clock;

double now_s() { return std::chrono::duration<double>(clock_type::now().time_since_epoch()).count(); }

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with merging of neighbouring free ranges.
struct Arena {
    std::map<size_t, size_t> free_ranges;    // offset -> length
    void reset(size_t size) {
        free_ranges.clear();
        if (size) free_ranges[0] = size;
    }
    bool alloc(size_t n, size_t* off) {
        for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, at = it->first + n;
            free_ranges.erase(it);
            if (rest) free_ranges[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        auto next = free_ranges.lower_bound(off);
        if (next != free_ranges.end() && off + n == next->first) {   // merge with the range after
            n += next->second;
            next = free_ranges.erase(next);
        }
        if (next != free_ranges.begin()) {                              // merge with the range before
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_ranges[off] = n;
    }
};

enum ObsState { kPending = 0, kAdmitted = 1, kClosed = 2, kFailed = 3, kAdmitting = 4 };
enum TicketState { kQueued = 0, kRunning = 1, kDone = 2 };

struct Ticket {
    int obs = -1;
    const void* h_in = nullptr;
    void* h_vis = nullptr;
    std::vector<double> delays;
    double t_submit = 0, t_done = 0;
    int state = kQueued;
    int rc = COBALT_OK;
    std::string msg;
};

struct Obs {
    int state = kPending;
    bool closing = false;
    // the setting, with its host tables copied (admission may happen after open returns)
    cobalt_config cfg{};
    std::vector<float> fir, bandpass;
    std::vector<double> freqs;
    size_t plan_bytes = 0, in_bytes = 0, vis_bytes = 0, need = 0, off = 0;
    int S = 0;
    cobalt_plan* plan = nullptr;
    void* d_in = nullptr;
    void* d_vis = nullptr;
    std::deque<int64_t> queue;
    bool busy = false;                // a block of this observation is on the device
    std::string err;                  // why admission failed
};

thread_local std::string t_err;
int sfail(int code, const std::string& msg) {
    t_err = msg;
    return code;
}

}  // namespace

struct cobalt_service {
    std::mutex mu;
    std::condition_variable cv_work;      // workers wake on submit / admission / close / stop
    std::condition_variable cv_done;      // waiters wake on completion
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    bool stop = false;
    bool paused = false;
    int device = 0;
    char* d_arena = nullptr;
    Arena arena;
    size_t budget = 0, used = 0;
    int depth = 1;
    double deadline = 1.0;
    std::vector<std::unique_ptr<Obs>> obs;
    std::deque<int> pending;              // observations waiting for admission, in arrival order
    bool admitting = false;               // an admission is being set up (outside the lock)
    std::unordered_map<int64_t, Ticket> tickets;
    int64_t next_ticket = 1;
    int rr = 0;                           // round-robin start over observations
    int64_t submitted = 0, completed = 0, dropped = 0, late = 0;
    std::vector<double> latencies;
};

namespace {

// Complete every queued block of `o` without running it (caller holds the lock).
void cancel_queue(cobalt_service* s, Obs* o, int rc, const char* why) {
    while (!o->queue.empty()) {
        auto it = s->tickets.find(o->queue.front());
        o->queue.pop_front();
        if (it == s->tickets.end()) continue;
        it->second.state = kDone;
        it->second.rc = rc;
        it->second.msg = why;
        it->second.t_done = now_s();
        ++s->dropped;
    }
    s->cv_done.notify_all();
}

// Create the observation's plan in its arena range (no lock held).
int setup_obs(cobalt_service* s, Obs* o) {
    char* base = s->d_arena + o->off;
    o->d_in = base + o->plan_bytes;
    o->d_vis = base + o->plan_bytes + align_up(o->in_bytes);
    return cobalt::plan_create_impl(&o->cfg, base, &o->plan);
}

// Admit the head of the pending FIFO if its working set fits (caller holds `lk`; the lock is
// released while the plan is created).  Returns true when it did any work.
bool try_admit(cobalt_service* s, std::unique_lock<std::mutex>& lk) {
    if (s->admitting || s->pending.empty()) return false;
    Obs* o = s->obs[s->pending.front()].get();
    size_t off = 0;
    if (!s->arena.alloc(o->need, &off)) return false;
    s->pending.pop_front();
    s->admitting = true;
    o->off = off;
    o->state = kAdmitting;
    s->used += o->need;
    lk.unlock();
    const int rc = setup_obs(s, o);
    const std::string msg = rc == COBALT_OK ? std::string() : std::string(cobalt_last_error());
    lk.lock();
    s->admitting = false;
    if (rc == COBALT_OK) {
        o->state = kAdmitted;
    } else {
        o->state = kFailed;
        o->err = msg;
        s->arena.release(o->off, o->need);
        s->used -= o->need;
        cancel_queue(s, o, rc, "observation could not be admitted");
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    return true;
}

// Start the next queued block of some admitted observation on this worker's stream (caller
// holds `lk`; released while the block runs).  Returns true when it ran one.
bool try_run(cobalt_service* s, std::unique_lock<std::mutex>& lk, hipStream_t st) {
    if (s->paused) return false;
    const int n = (int)s->obs.size();
    for (int k = 0; k < n; ++k) {
        const int oi = (s->rr + k) % n;
        Obs* o = s->obs[oi].get();
        if (o->state != kAdmitted || o->busy || o->queue.empty()) continue;
        const int64_t id = o->queue.front();
        o->queue.pop_front();
        Ticket& t = s->tickets[id];        // references into an unordered_map survive inserts
        t.state = kRunning;
        o->busy = true;
        s->rr = (oi + 1) % n;
        const void* h_in = t.h_in;
        void* h_vis = t.h_vis;
        const std::vector<double> delays = t.delays;
        lk.unlock();
        int rc = COBALT_OK;
        std::string msg;
        hipError_t e = hipMemcpyAsync(o->d_in, h_in, o->in_bytes, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) {
            rc = cobalt_correlate(o->plan, o->d_in, delays.data(), o->d_vis, st);
            if (rc != COBALT_OK) msg = cobalt_last_error();
        }
        if (e == hipSuccess && rc == COBALT_OK) e = hipMemcpyAsync(h_vis, o->d_vis, o->vis_bytes, hipMemcpyDeviceToHost, st);
        const hipError_t es = hipStreamSynchronize(st);
        if (e == hipSuccess) e = es;
        if (e != hipSuccess && rc == COBALT_OK) {
            rc = COBALT_EDEVICE;
            msg = hipGetErrorString(e);
        }
        const double t_done = now_s();
        lk.lock();
        Ticket& u = s->tickets[id];
        u.t_done = t_done;
        u.state = kDone;
        u.rc = rc;
        u.msg = msg;
        const double lat = t_done - u.t_submit;
        s->latencies.push_back(lat);
        ++s->completed;
        if (lat > s->deadline) ++s->late;
        o->busy = false;
        s->cv_done.notify_all();
        s->cv_work.notify_all();
        return true;
    }
    return false;
}

void worker(cobalt_service* s, int slot) {
    (void)hipSetDevice(s->device);
    const hipStream_t st = s->streams[slot];
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        if (try_admit(s, lk)) continue;
        if (try_run(s, lk, st)) continue;
        s->cv_work.wait(lk);
    }
}

Obs* find_obs(cobalt_service* s, int obs_id) {
    if (obs_id < 0 || obs_id >= (int)s->obs.size()) return nullptr;
    return s->obs[obs_id].get();
}

}  // namespace

extern "C" {

const char* cobalt_service_last_error(void) { return t_err.c_str(); }

int cobalt_service_create(size_t hbm_budget_bytes, int n_slots, int queue_depth, double deadline_s, cobalt_service** out) {
    t_err.clear();
    if (!out) return sfail(COBALT_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_slots < 1 || n_slots > 64 || queue_depth < 1 || !(deadline_s > 0))
        return sfail(COBALT_EINVAL, "need 1 <= n_slots <= 64, queue_depth >= 1, deadline_s > 0");
    if (hbm_budget_bytes < kAlign) return sfail(COBALT_EINVAL, "hbm_budget_bytes must be at least 256");
    cobalt_service* s = new (std::nothrow) cobalt_service();
    if (!s) return sfail(COBALT_ENOMEM, "host allocation failed");
    s->budget = hbm_budget_bytes / kAlign * kAlign;
    s->depth = queue_depth;
    s->deadline = deadline_s;
    if (hipGetDevice(&s->device) != hipSuccess) { delete s; return sfail(COBALT_EDEVICE, "hipGetDevice failed"); }
    if (hipMalloc((void**)&s->d_arena, s->budget) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return sfail(COBALT_ENOMEM, "cannot allocate the HBM budget as one arena");
    }
    s->arena.reset(s->budget);
    s->streams.assign(n_slots, nullptr);
    for (auto& st : s->streams) {
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto& x : s->streams)
                if (x) (void)hipStreamDestroy(x);
            (void)hipFree(s->d_arena);
            delete s;
            return sfail(COBALT_EDEVICE, "stream creation failed");
        }
    }
    for (int i = 0; i < n_slots; ++i) s->workers.emplace_back(worker, s, i);
    *out = s;
    return COBALT_OK;
}

int cobalt_service_open(cobalt_service* s, const cobalt_config* cfg, int* obs_id) {
    t_err.clear();
    if (!s || !cfg || !obs_id) return sfail(COBALT_EINVAL, "NULL argument");
    size_t plan_bytes = 0;
    int rc = cobalt_estimate_bytes(cfg, &plan_bytes);
    if (rc != COBALT_OK) return sfail(rc, cobalt_last_error());
    std::unique_ptr<Obs> o(new (std::nothrow) Obs());
    if (!o) return sfail(COBALT_ENOMEM, "host allocation failed");
    const int64_t M = 2LL * cfg->n_stations, B = (int64_t)cfg->n_stations * (cfg->n_stations + 1) / 2;
    const int64_t sb = cfg->sample_type == COBALT_CI8 ? 2 : cfg->sample_type == COBALT_CI16 ? 4 : 8;
    o->plan_bytes = align_up(plan_bytes);
    o->in_bytes = (size_t)(M * cfg->n_subbands * cfg->samples_per_block * sb);
    o->vis_bytes = (size_t)((int64_t)cfg->n_subbands * cfg->n_channels * B * 4 * 8);
    o->need = o->plan_bytes + align_up(o->in_bytes) + align_up(std::max<size_t>(o->vis_bytes, 16));
    o->S = cfg->n_stations;
    o->cfg = *cfg;
    o->fir.assign(cfg->h_fir, cfg->h_fir + (size_t)cfg->n_taps * cfg->n_channels);
    if (cfg->h_bandpass) o->bandpass.assign(cfg->h_bandpass, cfg->h_bandpass + cfg->n_channels);
    o->freqs.assign(cfg->h_subband_freq_hz, cfg->h_subband_freq_hz + cfg->n_subbands);
    o->cfg.h_fir = o->fir.data();
    o->cfg.h_bandpass = cfg->h_bandpass ? o->bandpass.data() : nullptr;
    o->cfg.h_subband_freq_hz = o->freqs.data();
    if (o->need > s->budget) return sfail(COBALT_ENOMEM, "not admitted: the observation needs more than the whole HBM budget");

    std::unique_lock<std::mutex> lk(s->mu);
    const int id = (int)s->obs.size();
    Obs* op = o.get();
    s->obs.push_back(std::move(o));
    *obs_id = id;
    size_t off = 0;
    if (s->pending.empty() && !s->admitting && s->arena.alloc(op->need, &off)) {
        // fits now: admit in the caller's thread
        s->admitting = true;
        op->off = off;
        op->state = kAdmitting;
        s->used += op->need;
        lk.unlock();
        rc = setup_obs(s, op);
        const std::string msg = rc == COBALT_OK ? std::string() : std::string(cobalt_last_error());
        lk.lock();
        s->admitting = false;
        if (rc != COBALT_OK) {
            op->state = kClosed;
            s->arena.release(op->off, op->need);
            s->used -= op->need;
            s->cv_work.notify_all();
            return sfail(rc, msg);
        }
        op->state = kAdmitted;
        s->cv_work.notify_all();
        return COBALT_OK;
    }
    op->state = kPending;                  // admitted by a worker once closes free enough memory
    s->pending.push_back(id);
    s->cv_work.notify_all();
    return COBALT_OK;
}

int cobalt_service_query(cobalt_service* s, int obs_id, int* state) {
    t_err.clear();
    if (!s || !state) return sfail(COBALT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    Obs* o = find_obs(s, obs_id);
    if (!o) return sfail(COBALT_EINVAL, "unknown observation");
    *state = o->state == kAdmitting ? kPending : o->state;
    if (o->state == kFailed) t_err = o->err;
    return COBALT_OK;
}

int cobalt_service_submit(cobalt_service* s, int obs_id, const void* h_block, const double* h_delays, void* h_vis,
                          int64_t* ticket) {
    t_err.clear();
    if (!s || !h_delays || !h_vis || !ticket) return sfail(COBALT_EINVAL, "NULL argument");
    *ticket = -1;
    std::lock_guard<std::mutex> lk(s->mu);
    Obs* o = find_obs(s, obs_id);
    if (!o || o->closing || o->state == kClosed) return sfail(COBALT_EINVAL, "unknown or closed observation");
    if (o->state == kFailed) return sfail(COBALT_EDEVICE, "observation could not be admitted: " + o->err);
    if (!h_block && o->in_bytes > 0) return sfail(COBALT_EINVAL, "h_block is NULL");
    ++s->submitted;
    if ((int)o->queue.size() >= s->depth) {
        ++s->dropped;
        return sfail(COBALT_EBUSY, "queue full: block dropped");
    }
    const int64_t id = s->next_ticket++;
    Ticket& t = s->tickets[id];
    t.obs = obs_id;
    t.h_in = h_block;
    t.h_vis = h_vis;
    t.delays.assign(h_delays, h_delays + 2 * o->S);
    t.t_submit = now_s();
    o->queue.push_back(id);
    *ticket = id;
    s->cv_work.notify_all();
    return COBALT_OK;
}

int cobalt_service_wait(cobalt_service* s, int64_t ticket, double* latency_s) {
    t_err.clear();
    if (!s) return sfail(COBALT_EINVAL, "service is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->tickets.find(ticket) == s->tickets.end()) return sfail(COBALT_EINVAL, "unknown ticket");
    s->cv_done.wait(lk, [&] {
        auto it = s->tickets.find(ticket);
        return it == s->tickets.end() || it->second.state == kDone || s->stop;
    });
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return sfail(COBALT_EINVAL, "ticket was waited for by another thread");
    if (it->second.state != kDone) return sfail(COBALT_EDEVICE, "service stopped");
    if (latency_s) *latency_s = it->second.t_done - it->second.t_submit;
    const int rc = it->second.rc;
    const std::string msg = it->second.msg;
    s->tickets.erase(it);
    return rc == COBALT_OK ? COBALT_OK : sfail(rc, msg);
}

int cobalt_service_pause(cobalt_service* s, int paused) {
    t_err.clear();
    if (!s) return sfail(COBALT_EINVAL, "service is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    s->paused = paused != 0;
    s->cv_work.notify_all();
    return COBALT_OK;
}

int cobalt_service_get_stats(cobalt_service* s, cobalt_service_stats* out) {
    t_err.clear();
    if (!s || !out) return sfail(COBALT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> l = s->latencies;
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) -> double {
        if (l.empty()) return 0.0;
        const size_t i = (size_t)std::min<double>((double)l.size() - 1, std::ceil(p * l.size()) - 1);
        return l[i];
    };
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->dropped = s->dropped;
    out->late = s->late;
    out->p50_latency_s = pct(0.50);
    out->p99_latency_s = pct(0.99);
    out->max_latency_s = l.empty() ? 0.0 : l.back();
    out->hbm_used_bytes = (int64_t)s->used;
    out->hbm_budget_bytes = (int64_t)s->budget;
    int64_t adm = 0;
    for (auto& o : s->obs) adm += o->state == kAdmitted || o->state == kAdmitting;
    out->obs_admitted = adm;
    out->obs_pending = (int64_t)s->pending.size();
    return COBALT_OK;
}

int cobalt_service_close(cobalt_service* s, int obs_id) {
    t_err.clear();
    if (!s) return sfail(COBALT_EINVAL, "service is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    Obs* o = find_obs(s, obs_id);
    if (!o || o->closing || o->state == kClosed) return sfail(COBALT_EINVAL, "unknown or closed observation");
    o->closing = true;
    if (o->state == kPending) {
        // never admitted: its queued blocks are dropped
        s->pending.erase(std::find(s->pending.begin(), s->pending.end(), obs_id));
        cancel_queue(s, o, COBALT_EBUSY, "observation closed before admission: block dropped");
        o->state = kClosed;
        s->cv_work.notify_all();
        return COBALT_OK;
    }
    s->paused = false;                      // queued blocks of this observation still run
    s->cv_work.notify_all();
    s->cv_done.wait(lk, [&] { return o->state != kAdmitting && ((o->queue.empty() && !o->busy) || s->stop); });
    if (o->state == kFailed) {
        o->state = kClosed;
        return COBALT_OK;
    }
    cobalt_plan* plan = o->plan;
    o->plan = nullptr;
    lk.unlock();
    const int rc = cobalt_plan_destroy(plan);
    const std::string msg = rc == COBALT_OK ? std::string() : std::string(cobalt_last_error());
    lk.lock();
    s->arena.release(o->off, o->need);
    s->used -= o->need;
    o->state = kClosed;
    s->cv_work.notify_all();                // pending observations may fit now
    return rc == COBALT_OK ? COBALT_OK : sfail(rc, msg);
}

int cobalt_service_destroy(cobalt_service* s) {
    t_err.clear();
    if (!s) return COBALT_OK;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->paused = false;
        for (int id : s->pending) {
            Obs* o = s->obs[id].get();
            cancel_queue(s, o, COBALT_EBUSY, "service destroyed before admission: block dropped");
            o->state = kClosed;
        }
        s->pending.clear();
        s->cv_work.notify_all();
        // let queued and running blocks finish
        s->cv_done.wait(lk, [&] {
            if (s->admitting) return false;
            for (auto& o : s->obs)
                if (o->state == kAdmitted && (!o->queue.empty() || o->busy)) return false;
            return true;
        });
        s->stop = true;
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    for (auto& th : s->workers) th.join();
    for (auto& o : s->obs)
        if (o->state == kAdmitted && o->plan) cobalt_plan_destroy(o->plan);
    for (auto& st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    (void)hipFree(s->d_arena);
    delete s;
    return COBALT_OK;
}

}  // extern "C"
