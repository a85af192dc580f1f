// Streaming service: ~1 s blocks from several concurrent observations through the FX chain.
//
// Observations are admitted against an HBM budget (plan workspace + the observation's device
// input and visibility buffers).  Blocks arrive through cobalt_service_submit into a bounded
// per-observation FIFO; a dispatcher thread gives each waiting block a free stream slot as soon
// as one frees up, so blocks of different observations run concurrently on the device
// (continuous batching).  Blocks of one observation run in arrival order, one at a time (the
// FIR history carries from block to block).  A full FIFO drops the new block rather than
// waiting, as the paper's pipeline drops data instead of stalling ("Dealing with jitter and
// hardware failure", sec. 7.2); bounded queues with condition variables mirror its task
// pipeline ("Parallelization libraries", sec. 7.4).  Latency is measured from submit to the
// completion of the block's device-to-host visibility copy.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/cobalt.h"
#include "cobalt_internal.h"

namespace {

using clock_type = std::chrono::steady_clock;

double now_s() { return std::chrono::duration<double>(clock_type::now().time_since_epoch()).count(); }

struct Ticket {
    int obs = -1;
    const void* h_in = nullptr;
    void* h_vis = nullptr;
    std::vector<double> delays;
    double t_submit = 0, t_dispatch = 0, t_done = 0;
    int state = 0;                    // 0 queued, 1 running, 2 done
    int slot = -1;
};

struct Obs {
    cobalt_plan* plan = nullptr;
    cobalt_plan_info info{};
    size_t bytes = 0;                 // counted against the budget
    int S = 0;
    void* d_in = nullptr;
    void* d_vis = nullptr;
    std::deque<int64_t> queue;
    bool busy = false;
    bool open = false;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    int64_t ticket = -1;
};

thread_local std::string t_err;
int sfail(int code, const char* msg) {
    t_err = msg;
    return code;
}

}  // namespace

struct cobalt_service {
    std::mutex mu;
    std::condition_variable cv_work;      // dispatcher wakes on submit / stop
    std::condition_variable cv_done;      // waiters wake on completion
    std::thread th;
    bool stop = false;
    bool paused = false;
    int device = 0;
    size_t budget = 0, used = 0;
    int depth = 1;
    double deadline = 1.0;
    std::vector<Obs> obs;
    std::vector<Slot> slots;
    std::unordered_map<int64_t, Ticket> tickets;
    int64_t next_ticket = 1;
    int rr = 0;                           // round-robin start over observations
    int64_t submitted = 0, completed = 0, dropped = 0, late = 0;
    std::vector<double> latencies;
    std::string err;                      // first asynchronous device error
};

namespace {

// Dispatcher: retire finished slots, then start queued blocks on free slots.
void dispatcher(cobalt_service* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        bool progress = false;
        for (size_t i = 0; i < s->slots.size(); ++i) {
            Slot& sl = s->slots[i];
            if (sl.ticket < 0) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            Ticket& t = s->tickets[sl.ticket];
            t.t_done = now_s();
            t.state = 2;
            if (q != hipSuccess && s->err.empty()) s->err = hipGetErrorString(q);
            const double lat = t.t_done - t.t_submit;
            s->latencies.push_back(lat);
            ++s->completed;
            if (lat > s->deadline) ++s->late;
            s->obs[t.obs].busy = false;
            sl.ticket = -1;
            progress = true;
        }
        if (progress) s->cv_done.notify_all();
        if (!s->paused) {
            const int n = (int)s->obs.size();
            for (int k = 0; k < n; ++k) {
                const int oi = (s->rr + k) % n;
                Obs& o = s->obs[oi];
                if (!o.open || o.busy || o.queue.empty()) continue;
                int free_slot = -1;
                for (size_t i = 0; i < s->slots.size(); ++i)
                    if (s->slots[i].ticket < 0) { free_slot = (int)i; break; }
                if (free_slot < 0) break;
                const int64_t id = o.queue.front();
                o.queue.pop_front();
                Ticket& t = s->tickets[id];
                Slot& sl = s->slots[free_slot];
                t.t_dispatch = now_s();
                t.state = 1;
                t.slot = free_slot;
                o.busy = true;
                sl.ticket = id;
                hipError_t e = hipMemcpyAsync(o.d_in, t.h_in, (size_t)o.info.input_bytes, hipMemcpyHostToDevice, sl.st);
                int rc = e == hipSuccess ? cobalt_correlate(o.plan, o.d_in, t.delays.data(), o.d_vis, sl.st) : COBALT_EDEVICE;
                if (rc == COBALT_OK)
                    e = hipMemcpyAsync(t.h_vis, o.d_vis, (size_t)o.info.vis_bytes, hipMemcpyDeviceToHost, sl.st);
                if ((rc != COBALT_OK || e != hipSuccess) && s->err.empty())
                    s->err = rc != COBALT_OK ? cobalt_last_error() : hipGetErrorString(e);
                (void)hipEventRecord(sl.done, sl.st);
                s->rr = (oi + 1) % n;
                progress = true;
            }
        }
        if (!progress) {
            bool any_busy = false;
            for (auto& sl : s->slots) any_busy |= sl.ticket >= 0;
            // poll running work every 50 us; otherwise sleep until a submit or stop
            if (any_busy) s->cv_work.wait_for(lk, std::chrono::microseconds(50));
            else s->cv_work.wait_for(lk, std::chrono::milliseconds(20));
        }
    }
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
    cobalt_service* s = new (std::nothrow) cobalt_service();
    if (!s) return sfail(COBALT_ENOMEM, "host allocation failed");
    s->budget = hbm_budget_bytes;
    s->depth = queue_depth;
    s->deadline = deadline_s;
    if (hipGetDevice(&s->device) != hipSuccess) { delete s; return sfail(COBALT_EDEVICE, "hipGetDevice failed"); }
    s->slots.resize(n_slots);
    for (auto& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            for (auto& x : s->slots) {
                if (x.done) (void)hipEventDestroy(x.done);
                if (x.st) (void)hipStreamDestroy(x.st);
            }
            delete s;
            return sfail(COBALT_EDEVICE, "stream/event creation failed");
        }
    }
    s->th = std::thread(dispatcher, s);
    *out = s;
    return COBALT_OK;
}

int cobalt_service_open(cobalt_service* s, const cobalt_config* cfg, int* obs_id) {
    t_err.clear();
    if (!s || !cfg || !obs_id) return sfail(COBALT_EINVAL, "NULL argument");
    size_t plan_bytes = 0;
    int rc = cobalt_estimate_bytes(cfg, &plan_bytes);
    if (rc != COBALT_OK) return sfail(rc, cobalt_last_error());
    const int64_t M = 2LL * cfg->n_stations, B = (int64_t)cfg->n_stations * (cfg->n_stations + 1) / 2;
    const int64_t sb = cfg->sample_type == COBALT_CI8 ? 2 : cfg->sample_type == COBALT_CI16 ? 4 : 8;
    const size_t io = (size_t)(M * cfg->n_subbands * cfg->samples_per_block * sb) +
                      (size_t)((int64_t)cfg->n_subbands * cfg->n_channels * B * 4 * 8);
    const size_t need = plan_bytes + io + 1024;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->used + need > s->budget) return sfail(COBALT_ENOMEM, "not admitted: HBM budget exceeded");
        s->used += need;            // reserve before allocating outside the lock
    }
    Obs o;
    o.bytes = need;
    o.S = cfg->n_stations;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != s->device) (void)hipSetDevice(s->device);
    rc = cobalt_plan_create(cfg, &o.plan);
    if (rc == COBALT_OK) rc = cobalt_plan_query(o.plan, &o.info);
    if (rc == COBALT_OK && (hipMalloc(&o.d_in, (size_t)std::max<int64_t>(o.info.input_bytes, 16)) != hipSuccess ||
                            hipMalloc(&o.d_vis, (size_t)std::max<int64_t>(o.info.vis_bytes, 16)) != hipSuccess))
        rc = COBALT_ENOMEM;
    if (prev >= 0 && prev != s->device) (void)hipSetDevice(prev);
    std::lock_guard<std::mutex> lk(s->mu);
    if (rc != COBALT_OK) {
        s->used -= need;
        if (o.d_in) (void)hipFree(o.d_in);
        if (o.d_vis) (void)hipFree(o.d_vis);
        if (o.plan) cobalt_plan_destroy(o.plan);
        return sfail(rc, rc == COBALT_ENOMEM ? "device allocation failed" : cobalt_last_error());
    }
    o.open = true;
    s->obs.push_back(std::move(o));
    *obs_id = (int)s->obs.size() - 1;
    return COBALT_OK;
}

int cobalt_service_submit(cobalt_service* s, int obs_id, const void* h_block, const double* h_delays, void* h_vis,
                          int64_t* ticket) {
    t_err.clear();
    if (!s || !h_delays || !h_vis || !ticket) return sfail(COBALT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (obs_id < 0 || obs_id >= (int)s->obs.size() || !s->obs[obs_id].open) return sfail(COBALT_EINVAL, "unknown observation");
    Obs& o = s->obs[obs_id];
    if (!h_block && o.info.input_bytes > 0) return sfail(COBALT_EINVAL, "h_block is NULL");
    ++s->submitted;
    if ((int)o.queue.size() >= s->depth) {
        ++s->dropped;
        *ticket = -1;
        return sfail(COBALT_EBUSY, "queue full: block dropped");
    }
    const int64_t id = s->next_ticket++;
    Ticket& t = s->tickets[id];
    t.obs = obs_id;
    t.h_in = h_block;
    t.h_vis = h_vis;
    t.delays.assign(h_delays, h_delays + 2 * o.S);
    t.t_submit = now_s();
    o.queue.push_back(id);
    *ticket = id;
    s->cv_work.notify_one();
    return COBALT_OK;
}

int cobalt_service_wait(cobalt_service* s, int64_t ticket, double* latency_s) {
    t_err.clear();
    if (!s) return sfail(COBALT_EINVAL, "service is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return sfail(COBALT_EINVAL, "unknown ticket");
    s->cv_done.wait(lk, [&] { return it->second.state == 2 || s->stop; });
    if (it->second.state != 2) return sfail(COBALT_EDEVICE, "service stopped");
    if (latency_s) *latency_s = it->second.t_done - it->second.t_submit;
    s->tickets.erase(it);
    if (!s->err.empty()) return sfail(COBALT_EDEVICE, s->err.c_str());
    return COBALT_OK;
}

int cobalt_service_pause(cobalt_service* s, int paused) {
    t_err.clear();
    if (!s) return sfail(COBALT_EINVAL, "service is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    s->paused = paused != 0;
    s->cv_work.notify_one();
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
    return COBALT_OK;
}

int cobalt_service_close(cobalt_service* s, int obs_id) {
    t_err.clear();
    if (!s) return sfail(COBALT_EINVAL, "service is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    if (obs_id < 0 || obs_id >= (int)s->obs.size() || !s->obs[obs_id].open) return sfail(COBALT_EINVAL, "unknown observation");
    Obs& o = s->obs[obs_id];
    s->paused = false;                      // queued blocks of this observation still run
    s->cv_work.notify_one();
    s->cv_done.wait(lk, [&] { return (o.queue.empty() && !o.busy) || s->stop; });
    o.open = false;
    int rc = cobalt_plan_destroy(o.plan);
    (void)hipFree(o.d_in);
    (void)hipFree(o.d_vis);
    o.plan = nullptr;
    s->used -= o.bytes;
    return rc == COBALT_OK ? COBALT_OK : sfail(rc, cobalt_last_error());
}

int cobalt_service_destroy(cobalt_service* s) {
    t_err.clear();
    if (!s) return COBALT_OK;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->paused = false;
        s->cv_work.notify_one();
        // let queued and running blocks finish
        s->cv_done.wait(lk, [&] {
            for (auto& o : s->obs)
                if (o.open && (!o.queue.empty() || o.busy)) return false;
            return true;
        });
        s->stop = true;
        s->cv_work.notify_one();
    }
    s->th.join();
    for (auto& o : s->obs) {
        if (!o.open) continue;
        cobalt_plan_destroy(o.plan);
        (void)hipFree(o.d_in);
        (void)hipFree(o.d_vis);
    }
    for (auto& sl : s->slots) {
        (void)hipStreamSynchronize(sl.st);
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.st);
    }
    delete s;
    return COBALT_OK;
}

}  // extern "C"
