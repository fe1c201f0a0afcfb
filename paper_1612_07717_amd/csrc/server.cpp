// server.cpp -- a request loop over the engine: continuous batching of MLMC queries.
//
// Clients enqueue queries from any thread. One worker thread owns the engine: it
// admits waiting queries into free slots (arrival order), runs an engine iteration
// over everything admitted, and completes the tickets of queries that converged. New
// arrivals join at the next iteration, so short queries do not wait for long ones and
// the device runs the tiles of all active queries together. The FIFO policy runs the
// same queries one at a time through mlmc_estimate, as the plain comparison point.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host_common.hpp"

using namespace ldm;

namespace {

double clock_seconds() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum TicketState { QUEUED = 0, RUNNING = 1, DONE = 2 };

struct Ticket {
    TicketState state = QUEUED;
    ld_query q;
    int64_t engine_handle = -1;
    int status = LD_PENDING;
    ld_estimate_result res;
    ld_request_times times;
};

}  // namespace

struct ld_server {
    ld_server_opts opts;
    int device = 0;
    ld_engine* engine = nullptr;
    void* d_ws = nullptr;            // FIFO: mlmc_estimate workspace
    hipStream_t stream = nullptr;    // FIFO: its stream
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<int64_t> queue;
    std::vector<int64_t> running;
    std::unordered_map<int64_t, Ticket> tickets;
    int64_t next_ticket = 0;
    bool stop = false;
    int failure = LD_OK;
    std::string failure_msg;
    ld_server_stats st;
};

namespace {

void complete(ld_server* s, Ticket& t, int status) {
    t.status = status;
    t.state = DONE;
    t.times.t_done = clock_seconds();
    s->st.completed += 1;
    if (status >= 0 || status == LD_ENONFINITE) s->st.fine_steps += t.res.fine_steps;
}

// The worker failed: every queued and running query completes with the error.
void fail_all(ld_server* s, int status, const std::string& msg) {
    s->failure = status;
    s->failure_msg = msg;
    for (int64_t id : s->running) complete(s, s->tickets[id], status);
    for (int64_t id : s->queue) complete(s, s->tickets[id], status);
    s->running.clear();
    s->queue.clear();
    s->cv_done.notify_all();
}

void worker_batch(ld_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // admission in arrival order while the engine has slots
        while (!s->stop && !s->queue.empty()) {
            const int64_t id = s->queue.front();
            Ticket& t = s->tickets[id];
            int64_t h = -1;
            const int rc = ld_engine_submit(s->engine, &t.q, &h);
            if (rc == LD_EBUSY) break;
            s->queue.pop_front();
            if (rc != LD_OK) {
                complete(s, t, rc);
                s->cv_done.notify_all();
                continue;
            }
            t.engine_handle = h;
            t.state = RUNNING;
            t.times.t_admit = clock_seconds();
            s->running.push_back(id);
        }
        s->st.max_running = std::max<int32_t>(s->st.max_running, (int32_t)s->running.size());
        if (s->stop) break;
        if (s->running.empty()) {
            s->cv_work.wait(lk, [s] { return s->stop || !s->queue.empty(); });
            continue;
        }
        lk.unlock();
        const double t0 = clock_seconds();
        int32_t active = 0;
        const int rc = ld_engine_step(s->engine, &active);
        const std::string msg = rc == LD_OK ? std::string() : std::string(ld_last_error());
        const double t1 = clock_seconds();
        lk.lock();
        s->st.busy_seconds += t1 - t0;
        s->st.iterations += 1;
        (void)ld_engine_stats(s->engine, &s->st.device_seconds, nullptr, nullptr);
        if (rc != LD_OK) {
            fail_all(s, rc, msg);
            break;
        }
        bool any = false;
        for (size_t i = 0; i < s->running.size();) {
            Ticket& t = s->tickets[s->running[i]];
            const int r = ld_engine_result(s->engine, t.engine_handle, &t.res);
            if (r == LD_PENDING) {
                ++i;
                continue;
            }
            (void)ld_engine_release(s->engine, t.engine_handle);
            complete(s, t, r);
            any = true;
            s->running[i] = s->running.back();
            s->running.pop_back();
        }
        if (any) s->cv_done.notify_all();
    }
}

void worker_fifo(ld_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_work.wait(lk, [s] { return s->stop || !s->queue.empty(); });
        if (s->stop) break;
        const int64_t id = s->queue.front();
        s->queue.pop_front();
        Ticket& t = s->tickets[id];
        t.state = RUNNING;
        t.times.t_admit = clock_seconds();
        s->running.assign(1, id);
        s->st.max_running = std::max<int32_t>(s->st.max_running, 1);
        const ld_query q = t.q;
        lk.unlock();
        ld_estimate_opts o;
        mlmc_estimate_default_opts(&o);
        o.release = q.problem.release;
        o.T = q.problem.T;
        o.M0 = q.problem.M0;
        o.L_min = q.L_min;
        o.L_max = q.L_max;
        o.fixed_L = q.fixed_L;
        o.fixed_N = 0;
        o.eps_is_relative = q.eps_is_relative;
        o.N_init = q.N_init;
        o.alpha = q.alpha;
        o.precision = s->opts.engine.precision;
        o.stream_id = q.problem.stream_id;
        o.seed = q.problem.seed;
        o.max_iter = q.max_iter > 0 ? q.max_iter : 100;
        o.max_fine_steps = q.max_fine_steps;
        o.x_adapt = q.problem.x_adapt;
        o.d_workspace = s->d_ws;
        o.workspace_bytes = mlmc_estimate_workspace();
        o.hip_stream = s->stream;
        ld_estimate_result res;
        std::memset(&res, 0, sizeof res);
        const double t0 = clock_seconds();
        const int rc = mlmc_estimate(q.eps, &q.problem.qoi, q.integrator, &q.problem.profile, &o, &res);
        const std::string msg = (rc == LD_EDEVICE) ? std::string(ld_last_error()) : std::string();
        const double t1 = clock_seconds();
        lk.lock();
        s->st.busy_seconds += t1 - t0;
        s->st.device_seconds += res.device_seconds;
        s->st.iterations += 1;
        s->running.clear();
        Ticket& tt = s->tickets[id];
        tt.res = res;
        complete(s, tt, rc);
        if (rc == LD_EDEVICE) {
            fail_all(s, rc, msg);
            break;
        }
        s->cv_done.notify_all();
    }
}

void free_server(ld_server* s) {
    if (s->engine) ld_engine_destroy(s->engine);
    if (s->stream) {
        (void)hipStreamSynchronize(s->stream);
        (void)hipStreamDestroy(s->stream);
    }
    if (s->d_ws) (void)hipFree(s->d_ws);
    delete s;
}

}  // namespace

extern "C" {

void ld_server_default_opts(ld_server_opts* o) {
    if (o == nullptr) return;
    std::memset(o, 0, sizeof *o);
    ld_engine_default_opts(&o->engine);
    o->policy = LD_SERVE_BATCH;
    o->max_queued = 0;
}

double ld_server_clock(void) { return clock_seconds(); }

int ld_server_create(const ld_server_opts* opts_in, ld_server** out) {
    if (out == nullptr) return fail(LD_EINVAL, "out is NULL");
    *out = nullptr;
    ld_server_opts o;
    if (opts_in)
        o = *opts_in;
    else
        ld_server_default_opts(&o);
    if (o.policy != LD_SERVE_BATCH && o.policy != LD_SERVE_FIFO) return fail(LD_EINVAL, "unknown policy");
    if (o.max_queued < 0) return fail(LD_EINVAL, "max_queued must be >= 0");
    if (o.engine.precision != LD_FP32 && o.engine.precision != LD_FP64)
        return fail(LD_EINVAL, "unknown precision");
    ld_server* s = new ld_server();
    s->opts = o;
    std::memset(&s->st, 0, sizeof s->st);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(LD_ENODEVICE, "no HIP device");
    }
    if (o.policy == LD_SERVE_BATCH) {
        const int rc = ld_engine_create(&o.engine, &s->engine);
        if (rc != LD_OK) {
            delete s;
            return rc;
        }
    } else {
        if (hipMalloc(&s->d_ws, mlmc_estimate_workspace()) != hipSuccess) {
            free_server(s);
            return fail(LD_ENOMEM, "hipMalloc of the estimate workspace failed");
        }
        if (hipStreamCreate(&s->stream) != hipSuccess) {
            free_server(s);
            return fail(LD_EDEVICE, "hipStreamCreate failed");
        }
    }
    try {
        s->worker = std::thread(o.policy == LD_SERVE_BATCH ? worker_batch : worker_fifo, s);
    } catch (...) {
        free_server(s);
        return fail(LD_EDEVICE, "could not start the worker thread");
    }
    *out = s;
    return LD_OK;
}

void ld_server_destroy(ld_server* s) {
    if (s == nullptr) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    free_server(s);
}

int ld_server_submit(ld_server* s, const ld_query* q, int64_t* ticket) {
    if (s == nullptr || ticket == nullptr) return fail(LD_EINVAL, "NULL argument");
    const int rc = validate_query(q);
    if (rc != LD_OK) return rc;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failure != LD_OK) return fail(s->failure, "server stopped after an error: " + s->failure_msg);
    if (s->opts.max_queued > 0 && (int64_t)s->queue.size() >= s->opts.max_queued)
        return fail(LD_EBUSY, "admission queue is full");
    const int64_t id = s->next_ticket++;
    Ticket& t = s->tickets[id];
    t.q = *q;
    std::memset(&t.res, 0, sizeof t.res);
    std::memset(&t.times, 0, sizeof t.times);
    t.times.t_submit = clock_seconds();
    s->queue.push_back(id);
    s->st.submitted += 1;
    s->st.max_queued = std::max<int32_t>(s->st.max_queued, (int32_t)s->queue.size());
    *ticket = id;
    s->cv_work.notify_one();
    return LD_OK;
}

int ld_server_wait(ld_server* s, int64_t ticket, double timeout_s, ld_estimate_result* out,
                   ld_request_times* times) {
    if (s == nullptr || out == nullptr) return fail(LD_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(LD_EINVAL, "unknown ticket");
    auto done = [&] {
        auto i = s->tickets.find(ticket);
        return i == s->tickets.end() || i->second.state == DONE;
    };
    if (timeout_s < 0)
        s->cv_done.wait(lk, done);
    else if (timeout_s > 0)
        s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
    it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(LD_EINVAL, "ticket was collected by another caller");
    if (it->second.state != DONE) return LD_PENDING;
    *out = it->second.res;
    if (times) *times = it->second.times;
    const int status = it->second.status;
    s->tickets.erase(it);
    return status;
}

int ld_server_stats_get(ld_server* s, ld_server_stats* out) {
    if (s == nullptr || out == nullptr) return fail(LD_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->queued = (int64_t)s->queue.size();
    out->running = (int64_t)s->running.size();
    return LD_OK;
}

}  // extern "C"
