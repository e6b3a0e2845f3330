// Continuous-batching server over the stepping ABI (fe_begin / fe_advance /
// fe_end).  Requests arrive at any time; a worker thread admits them in
// arrival order as device memory frees up, keeps every admitted job's
// state (u^n, u^{n-1}) resident, and runs ticks: each tick advances the
// resident jobs (oldest first, up to an optional work budget) by up to
// `iters_per_tick` iterations each in shared launches, so
// jobs of different sizes, iteration counts and precisions overlap on the
// device.  A job's result is bitwise the one fe_denoise gives it alone (the
// step's per-pixel arithmetic does not depend on the batch).
#include "fe.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fe_internal.h"
#include "fe_sched.h"

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    fe_job job;
    uint64_t tag;
    size_t bytes;
    double t_submit;
};

struct Tick {
    hipEvent_t done = nullptr;
    std::vector<uint64_t> finishing;
    int ws = 0;
};

}  // namespace

struct fe_server {
    const fe_ctx *ctx = nullptr;
    fe_server_config cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    char *arena = nullptr;
    std::vector<void *> ws;        // fe_advance workspaces (ring)
    size_t ws_bytes = 0;
    std::vector<hipEvent_t> events;
    hipEvent_t t0_event = nullptr;
    double t0_host = 0.0;
    fe::Scheduler *sched = nullptr;

    std::mutex mu;
    std::condition_variable cv_in, cv_out;
    std::deque<Request> incoming;
    std::vector<fe_completion> completions;
    std::unordered_map<uint64_t, Request> jobs;   // id -> request (worker only)
    std::deque<Tick> inflight;                    // worker only
    std::vector<int> free_ws;                     // worker only
    std::vector<hipEvent_t> free_events;          // worker only
    std::atomic<bool> stop{false};
    std::atomic<int> n_pending{0}, n_active{0};
    std::thread worker;
    std::string error;
    fe_status status = FE_OK;

    double t_rel(double t) const { return t - t0_host; }
    void run();
    bool retire_one(bool wait);
    void fail(fe_status st, const std::string &msg)
    {
        std::lock_guard<std::mutex> lk(mu);
        if (status == FE_OK) {
            status = st;
            error = msg;
        }
        cv_out.notify_all();
    }
};

bool fe_server::retire_one(bool wait)
{
    if (inflight.empty()) return false;
    Tick &t = inflight.front();
    hipError_t e = wait ? hipEventSynchronize(t.done) : hipEventQuery(t.done);
    if (e == hipErrorNotReady) return false;
    if (e != hipSuccess) {
        fail(FE_ERR_DEVICE, std::string("tick failed: ") + hipGetErrorString(e));
        return false;
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, t0_event, t.done);
    const double t_done = ms * 1e-3;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (uint64_t id : t.finishing) {
            auto it = jobs.find(id);
            const fe::SchedJob *sj = sched->find(id);
            fe_completion c{};
            c.tag = it->second.tag;
            c.status = FE_OK;
            c.iterations = it->second.job.iterations;
            c.t_submit = t_rel(it->second.t_submit);
            c.t_admit = sj ? t_rel(sj->t_admit) : c.t_submit;
            c.t_done = t_done;
            completions.push_back(c);
            jobs.erase(it);
        }
    }
    sched->retire(t.finishing);
    free_ws.push_back(t.ws);
    free_events.push_back(t.done);
    inflight.pop_front();
    cv_out.notify_all();
    return true;
}

void fe_server::run()
{
    (void)hipSetDevice(device);
    std::vector<fe_job> bj, aj, ej;
    std::vector<float *> bs, as, es;
    std::vector<int32_t> done, cnt, edone;
    while (true) {
        bool failed = false;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (incoming.empty() && sched->pending() == 0 && sched->active() == 0 &&
                inflight.empty()) {
                if (stop.load()) break;
                cv_in.wait_for(lk, std::chrono::milliseconds(2));
            }
            while (!incoming.empty()) {
                Request r = incoming.front();
                incoming.pop_front();
                const uint64_t id = sched->submit(r.bytes, r.job.iterations, r.t_submit,
                                                  (long)r.job.height * r.job.width);
                jobs.emplace(id, r);
            }
            failed = status != FE_OK;
        }
        if (failed) break;
        while (retire_one(false)) {
        }
        if ((int)inflight.size() >= cfg.ticks_in_flight) {
            retire_one(true);
            continue;
        }
        if (sched->active() == 0 && sched->pending() == 0) {
            // only in-flight ticks left: poll them without blocking new arrivals
            if (!inflight.empty()) std::this_thread::sleep_for(std::chrono::microseconds(50));
            continue;
        }
        fe::TickPlan p = sched->plan(now_s());
        n_pending = (int)sched->pending();
        n_active = (int)sched->active();
        if (p.active.empty()) {
            // nothing fits until memory frees: wait for the oldest tick
            if (!retire_one(true)) std::this_thread::sleep_for(std::chrono::microseconds(200));
            continue;
        }
        auto state_of = [&](uint64_t id) {
            return (float *)(arena + sched->find(id)->off);
        };
        bj.clear(); bs.clear();
        for (uint64_t id : p.admitted) {
            bj.push_back(jobs.at(id).job);
            bs.push_back(state_of(id));
        }
        aj.clear(); as.clear(); done.clear(); cnt.clear();
        for (size_t i = 0; i < p.active.size(); ++i) {
            if (p.count[i] <= 0) continue;
            aj.push_back(jobs.at(p.active[i]).job);
            as.push_back(state_of(p.active[i]));
            done.push_back(p.done_before[i]);
            cnt.push_back(p.count[i]);
        }
        ej.clear(); es.clear(); edone.clear();
        for (uint64_t id : p.finishing) {
            ej.push_back(jobs.at(id).job);
            es.push_back(state_of(id));
            edone.push_back(jobs.at(id).job.iterations);
        }
        const int w = free_ws.back();
        free_ws.pop_back();
        fe_status st = FE_OK;
        if (!bj.empty()) st = fe_begin(ctx, bj.data(), bs.data(), (int32_t)bj.size(), stream);
        if (st == FE_OK && !aj.empty())
            st = fe_advance(ctx, aj.data(), as.data(), done.data(), cnt.data(), (int32_t)aj.size(),
                            ws[w], ws_bytes, stream);
        if (st == FE_OK && !ej.empty())
            st = fe_end(ctx, ej.data(), es.data(), edone.data(), (int32_t)ej.size(), stream);
        if (st != FE_OK) {
            fail(st, fe_last_error());
            break;
        }
        Tick t;
        t.done = free_events.back();
        free_events.pop_back();
        t.finishing = p.finishing;
        t.ws = w;
        hipError_t e = hipEventRecord(t.done, stream);
        if (e != hipSuccess) {
            fail(FE_ERR_DEVICE, std::string("event record: ") + hipGetErrorString(e));
            break;
        }
        inflight.push_back(t);
    }
    while (!inflight.empty())
        if (!retire_one(true)) break;
    cv_out.notify_all();
}

namespace {
thread_local std::string g_srv_err;
fe_status srv_fail(fe_status st, const char *msg)
{
    g_srv_err = msg;
    return st;
}
}  // namespace

extern "C" {

const char *fe_server_last_error(void) { return g_srv_err.c_str(); }

fe_status fe_server_create(const fe_ctx *ctx, const fe_server_config *cfg, void *hip_stream,
                           fe_server **out)
{
    if (!out) return srv_fail(FE_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!ctx || !cfg) return srv_fail(FE_ERR_INVALID, "ctx and cfg must be non-NULL");
    if (cfg->hbm_budget_bytes < 4096 || cfg->iters_per_tick < 1 || cfg->max_active < 1 ||
        cfg->ticks_in_flight < 1 || cfg->ticks_in_flight > 64 || cfg->tick_pixel_iters < 0)
        return srv_fail(FE_ERR_INVALID, "bad server configuration");
    fe_server *s = new (std::nothrow) fe_server;
    if (!s) return srv_fail(FE_ERR_NOMEM, "host allocation failed");
    s->ctx = ctx;
    s->cfg = *cfg;
    if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
    hipError_t e = hipSuccess;
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        s->own_stream = true;
    }
    if (e == hipSuccess) e = hipMalloc((void **)&s->arena, cfg->hbm_budget_bytes);
    size_t wsb = 0;
    fe_advance_workspace_size(ctx, cfg->max_active, &wsb);
    s->ws_bytes = wsb;
    const int nws = cfg->ticks_in_flight + 1;
    for (int i = 0; i < nws && e == hipSuccess; ++i) {
        void *p = nullptr;
        e = hipMalloc(&p, wsb);
        s->ws.push_back(p);
        s->free_ws.push_back(i);
        hipEvent_t ev = nullptr;
        if (e == hipSuccess) e = hipEventCreate(&ev);
        s->events.push_back(ev);
        s->free_events.push_back(ev);
    }
    if (e == hipSuccess) e = hipEventCreate(&s->t0_event);
    if (e == hipSuccess) e = hipEventRecord(s->t0_event, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(s->t0_event);
    s->t0_host = now_s();
    if (e != hipSuccess) {
        fe_server_destroy(s);
        return srv_fail(e == hipErrorOutOfMemory ? FE_ERR_NOMEM : FE_ERR_DEVICE,
                        hipGetErrorString(e));
    }
    s->sched = new fe::Scheduler(cfg->hbm_budget_bytes, cfg->iters_per_tick, cfg->max_active,
                                 cfg->tick_pixel_iters);
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return FE_OK;
}

fe_status fe_server_submit(fe_server *s, const fe_job *job, uint64_t tag)
{
    if (!s || !job) return srv_fail(FE_ERR_INVALID, "server and job must be non-NULL");
    size_t bytes = 0;
    fe_status st = fe_state_bytes(s->ctx, job->height, job->width, &bytes);
    if (st != FE_OK) return srv_fail(st, fe_last_error());
    st = fe_workspace_size(s->ctx, job, 1, &bytes);  // validates the job fully
    if (st != FE_OK) return srv_fail(st, fe_last_error());
    fe_state_bytes(s->ctx, job->height, job->width, &bytes);
    if (!s->sched->fits_ever(bytes))
        return srv_fail(FE_ERR_INVALID, "job state exceeds the server's memory budget");
    // debug mode: reject bad counts here, on the caller's thread, rather than
    // failing the whole server when the worker starts the job
    st = fe::validate_job_counts(s->device, job, 1);
    if (st != FE_OK) return srv_fail(st, fe_last_error());
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->status != FE_OK) return srv_fail(s->status, s->error.c_str());
    if (s->stop.load()) return srv_fail(FE_ERR_INVALID, "server is shutting down");
    s->incoming.push_back(Request{*job, tag, bytes, now_s()});
    s->cv_in.notify_one();
    return FE_OK;
}

fe_status fe_server_poll(fe_server *s, fe_completion *out, int32_t max, int32_t *n,
                         int32_t wait_ms)
{
    if (!s || !n || (max > 0 && !out)) return srv_fail(FE_ERR_INVALID, "bad arguments");
    *n = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->completions.empty() && wait_ms > 0 && s->status == FE_OK)
        s->cv_out.wait_for(lk, std::chrono::milliseconds(wait_ms));
    const int k = std::min<int>(max, (int)s->completions.size());
    for (int i = 0; i < k; ++i) out[i] = s->completions[i];
    s->completions.erase(s->completions.begin(), s->completions.begin() + k);
    *n = k;
    if (s->status != FE_OK && k == 0) return srv_fail(s->status, s->error.c_str());
    return FE_OK;
}

fe_status fe_server_load(fe_server *s, int32_t *pending, int32_t *active, double *now)
{
    if (!s) return srv_fail(FE_ERR_INVALID, "server is NULL");
    if (pending) *pending = s->n_pending.load();
    if (active) *active = s->n_active.load();
    if (now) *now = s->t_rel(now_s());
    return FE_OK;
}

void fe_server_destroy(fe_server *s)
{
    if (!s) return;
    s->stop = true;
    s->cv_in.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (void *p : s->ws) (void)hipFree(p);
    for (hipEvent_t ev : s->events)
        if (ev) (void)hipEventDestroy(ev);
    if (s->t0_event) (void)hipEventDestroy(s->t0_event);
    (void)hipFree(s->arena);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s->sched;
    delete s;
}

}  // extern "C"
