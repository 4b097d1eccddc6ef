// serve.hip -- the served form: views arrive one by one, as a scanning
// microscope produces them, and are tracked in batches formed on the fly.
//
// A worker thread owns n_pipes contexts, each with its own stream and
// device buffers. Whenever a pipeline is free and views are waiting, it
// takes the waiting views in arrival order, as many as fit the pipeline's
// share of the HBM budget (and max_batch_views), and enqueues them as one
// batch. With two or more pipelines a batch is admitted while another is
// still on the device, so their kernels overlap. Results are exact integer
// decisions, so a view's tracks do not depend on which batch it joined.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "emt.h"
#include "emt_host.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0, view_id = 0;
    std::vector<int32_t> xyz;
    uint32_t n = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int status = EMT_OK;
    uint32_t batch_views = 0;
    std::vector<emt_track> tracks;
    std::vector<uint32_t> grains;
    emt_view_stats stats{};
};

struct Pipe {
    emt_ctx *ctx = nullptr;
    std::vector<Request *> batch;
    std::vector<emt_view_in> ins;
    std::vector<emt_view_out> outs;
    bool busy = false;
};

constexpr uint32_t kMaxPipes = 8;
constexpr auto kDevicePoll = std::chrono::microseconds(20);

}  // namespace

struct emt_server {
    emt_config cfg{};
    std::vector<Pipe> pipes;
    uint32_t max_batch_views = 0;
    unsigned long long max_batch_grains = 0;  // 0: no limit
    size_t pipe_budget = 0;

    std::mutex mu;
    std::condition_variable cv_work;  // the worker waits for arrivals
    std::condition_variable cv_done;  // pollers wait for completions
    std::deque<Request *> queue;      // submitted, not yet admitted
    std::deque<Request *> done;       // finished, not yet polled
    std::vector<Request *> handed;    // returned by the last poll
    uint64_t next_ticket = 1;
    bool stop = false;
    int fatal = EMT_OK;
    std::thread worker;
    Clock::time_point t0;

    emt_server_stats st{};
    uint32_t n_busy = 0;
    double t_mark = 0;  // last change of n_busy
};

namespace {

double now_ms(const emt_server *S) {
    return std::chrono::duration<double, std::milli>(Clock::now() - S->t0).count();
}

// Busy-time integrals; called with the lock held whenever n_busy changes.
void account(emt_server *S, int delta) {
    const double t = now_ms(S);
    if (S->n_busy >= 1) S->st.busy_ms += t - S->t_mark;
    if (S->n_busy >= 2) S->st.overlap_ms += t - S->t_mark;
    S->t_mark = t;
    S->n_busy = (uint32_t)((int)S->n_busy + delta);
}

// Take waiting views for a free pipeline: arrival order, while the batch
// fits the pipeline's HBM share, its view limit and its grain limit (a view
// larger than the grain limit goes alone). A view that alone exceeds the
// HBM share fails.
void form_batch(emt_server *S, Pipe &p, std::vector<Request *> &rejected) {
    p.batch.clear();
    unsigned long long n_total = 0;
    uint32_t max_n = 0;
    while (!S->queue.empty() && p.batch.size() < S->max_batch_views) {
        Request *r = S->queue.front();
        const unsigned long long nt = n_total + r->n;
        if (S->max_batch_grains && !p.batch.empty() && nt > S->max_batch_grains) break;
        const uint32_t mn = std::max(max_n, r->n);
        const size_t need = emt::batch_bytes(p.ctx, nt, (uint32_t)p.batch.size() + 1, mn);
        if (need > S->pipe_budget) {
            if (p.batch.empty()) {
                S->queue.pop_front();
                r->status = EMT_ENOMEM;
                rejected.push_back(r);
                continue;
            }
            break;
        }
        S->queue.pop_front();
        p.batch.push_back(r);
        n_total = nt;
        max_n = mn;
    }
}

void finish_batch(emt_server *S, Pipe &p, int rc) {
    for (size_t v = 0; v < p.batch.size(); ++v) {
        Request *r = p.batch[v];
        r->status = rc;
        r->batch_views = (uint32_t)p.batch.size();
        if (rc != EMT_OK) continue;
        const emt_view_out &o = p.outs[v];
        r->tracks.assign(o.tracks, o.tracks + o.n_tracks);
        r->grains.assign(o.grains, o.grains + o.n_track_grains);
        r->stats = o.stats;
    }
}

void worker_main(emt_server *S) {
    (void)hipSetDevice(S->cfg.device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool progress = false;
        // completions
        for (Pipe &p : S->pipes) {
            if (!p.busy) continue;
            lk.unlock();
            const bool ready = emt::views_ready(p.ctx);
            int rc = EMT_OK;
            if (ready) {
                rc = emt::finish_views(p.ctx, p.outs.data());
                finish_batch(S, p, rc);
                (void)hipGetLastError();
            }
            lk.lock();
            if (!ready) continue;
            const double t = now_ms(S);
            for (Request *r : p.batch) {
                r->t_done = t;
                S->done.push_back(r);
            }
            S->st.completed += p.batch.size();
            p.batch.clear();
            p.busy = false;
            account(S, -1);
            if (rc == EMT_EDEVICE) S->fatal = rc;
            progress = true;
            S->cv_done.notify_all();
        }
        // admissions
        for (Pipe &p : S->pipes) {
            if (p.busy || S->queue.empty() || S->stop || S->fatal) continue;
            std::vector<Request *> rejected;
            form_batch(S, p, rejected);
            const double t = now_ms(S);
            for (Request *r : rejected) {
                r->t_admit = r->t_done = t;
                S->done.push_back(r);
                S->st.completed++;
            }
            if (!rejected.empty()) S->cv_done.notify_all();
            if (p.batch.empty()) continue;
            for (Request *r : p.batch) r->t_admit = t;
            lk.unlock();
            const uint32_t nv = (uint32_t)p.batch.size();
            p.ins.resize(nv);
            p.outs.assign(nv, emt_view_out{});
            for (uint32_t v = 0; v < nv; ++v) {
                p.ins[v].xyz = p.batch[v]->n ? p.batch[v]->xyz.data() : nullptr;
                p.ins[v].n_grains = p.batch[v]->n;
                p.ins[v].reserved = 0;
                p.ins[v].view_id = p.batch[v]->view_id;
            }
            const int rc = emt::begin_views(p.ctx, p.ins.data(), nv);
            if (rc != EMT_OK) finish_batch(S, p, rc);
            (void)hipGetLastError();
            lk.lock();
            S->st.batches++;
            S->st.max_batch_views_seen = std::max(S->st.max_batch_views_seen, nv);
            if (rc == EMT_OK) {
                p.busy = true;
                account(S, +1);
            } else {
                const double td = now_ms(S);
                for (Request *r : p.batch) {
                    r->t_done = td;
                    S->done.push_back(r);
                }
                S->st.completed += nv;
                p.batch.clear();
                if (rc == EMT_EDEVICE) S->fatal = rc;
                S->cv_done.notify_all();
            }
            progress = true;
        }
        bool any_busy = false;
        for (const Pipe &p : S->pipes) any_busy = any_busy || p.busy;
        if (!any_busy && (S->stop || S->fatal)) break;
        if (progress) continue;
        if (any_busy)
            S->cv_work.wait_for(lk, kDevicePoll);
        else
            S->cv_work.wait(lk, [S] { return S->stop || !S->queue.empty(); });
    }
    // views never admitted (destroy or a device error) end with an error
    const double t = now_ms(S);
    while (!S->queue.empty()) {
        Request *r = S->queue.front();
        S->queue.pop_front();
        r->status = S->fatal ? S->fatal : EMT_EINVAL;
        r->t_done = t;
        S->done.push_back(r);
    }
    S->cv_done.notify_all();
}

void free_server(emt_server *S) {
    for (Pipe &p : S->pipes)
        if (p.ctx) emt_destroy(p.ctx);
    for (Request *r : S->queue) delete r;
    for (Request *r : S->done) delete r;
    for (Request *r : S->handed) delete r;
    delete S;
}

}  // namespace

extern "C" {

int emt_server_create(const emt_config *cfg, uint32_t n_pipes, uint32_t max_batch_views,
                      emt_server **out) {
    emt_server_limits lim{};
    lim.n_pipes = n_pipes;
    lim.max_batch_views = max_batch_views;
    lim.max_batch_grains = 0;
    return emt_server_create2(cfg, &lim, out);
}

int emt_server_create2(const emt_config *cfg, const emt_server_limits *lim, emt_server **out) {
    if (!out) return EMT_EINVAL;
    *out = nullptr;
    if (!cfg || !lim) return EMT_EINVAL;
    const uint32_t n_pipes = lim->n_pipes, max_batch_views = lim->max_batch_views;
    if (n_pipes < 1 || n_pipes > kMaxPipes || max_batch_views < 1) return EMT_EINVAL;
    if (cfg->flags & EMT_F_DEVICE_PTRS) return EMT_EINVAL;  // submissions are host copies
    int rc = emt_validate(cfg, nullptr, 0);
    if (rc) return rc;
    if (hipSetDevice(cfg->device) != hipSuccess) {
        (void)hipGetLastError();
        return EMT_EDEVICE;
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        return EMT_EDEVICE;
    }
    emt_server *S = new (std::nothrow) emt_server();
    if (!S) return EMT_ENOMEM;
    S->cfg = *cfg;
    S->max_batch_views = max_batch_views;
    S->max_batch_grains = lim->max_batch_grains;
    const size_t budget = cfg->hbm_budget ? (size_t)cfg->hbm_budget : (size_t)(0.8 * (double)free_b);
    S->pipe_budget = budget / n_pipes;
    S->pipes.resize(n_pipes);
    emt_config pc = *cfg;
    pc.hbm_budget = S->pipe_budget;
    pc.stream = nullptr;  // every pipeline on a stream of its own
    for (Pipe &p : S->pipes) {
        if ((rc = emt_create(&pc, &p.ctx)) != EMT_OK) {
            free_server(S);
            return rc;
        }
    }
    S->st.n_pipes = n_pipes;
    S->t0 = Clock::now();
    try {
        S->worker = std::thread(worker_main, S);
    } catch (...) {
        free_server(S);
        return EMT_ENOMEM;
    }
    *out = S;
    return EMT_OK;
}

int emt_server_submit(emt_server *S, const emt_view_in *view, uint64_t *ticket) {
    if (!S || !view) return EMT_EINVAL;
    int rc = emt_validate(&S->cfg, view, 1);
    if (rc) return rc;
    Request *r = new (std::nothrow) Request();
    if (!r) return EMT_ENOMEM;
    try {
        r->xyz.assign(view->xyz, view->xyz + 3 * (size_t)view->n_grains);
    } catch (...) {
        delete r;
        return EMT_ENOMEM;
    }
    r->n = view->n_grains;
    r->view_id = view->view_id;
    uint64_t my_ticket;
    {
        std::lock_guard<std::mutex> g(S->mu);
        if (S->fatal || S->stop) {
            delete r;
            return S->fatal ? S->fatal : EMT_EINVAL;
        }
        // the request belongs to the worker once queued: keep what is
        // reported from it before the lock is released
        my_ticket = r->ticket = S->next_ticket++;
        r->t_submit = now_ms(S);
        S->queue.push_back(r);
        S->st.submitted++;
    }
    S->cv_work.notify_one();
    if (ticket) *ticket = my_ticket;
    return EMT_OK;
}

int emt_server_poll(emt_server *S, emt_served *out, uint32_t max_out, uint32_t *n_out,
                    int32_t wait_ms) {
    if (!S || !n_out || (max_out > 0 && !out)) return EMT_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    for (Request *r : S->handed) delete r;
    S->handed.clear();
    auto ready = [S] { return !S->done.empty() || S->fatal != EMT_OK; };
    if (wait_ms < 0)
        S->cv_done.wait(lk, ready);
    else if (wait_ms > 0)
        S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
    uint32_t n = 0;
    while (n < max_out && !S->done.empty()) {
        Request *r = S->done.front();
        S->done.pop_front();
        S->handed.push_back(r);
        emt_served &o = out[n++];
        o.ticket = r->ticket;
        o.view_id = r->view_id;
        o.status = r->status;
        o.n_tracks = (uint32_t)r->tracks.size();
        o.n_track_grains = (uint32_t)r->grains.size();
        o.batch_views = r->batch_views;
        o.tracks = r->tracks.empty() ? nullptr : r->tracks.data();
        o.grains = r->grains.empty() ? nullptr : r->grains.data();
        o.stats = r->stats;
        o.t_submit_ms = r->t_submit;
        o.t_admit_ms = r->t_admit;
        o.t_done_ms = r->t_done;
    }
    *n_out = n;
    return S->fatal;
}

int emt_server_get_stats(emt_server *S, emt_server_stats *stats) {
    if (!S || !stats) return EMT_EINVAL;
    std::lock_guard<std::mutex> g(S->mu);
    account(S, 0);
    *stats = S->st;
    stats->elapsed_ms = now_ms(S);
    return EMT_OK;
}

void emt_server_destroy(emt_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    free_server(S);
    (void)hipGetLastError();
}

}  // extern "C"
