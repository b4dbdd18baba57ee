// Serving: continuous batching of independent solve requests on one device.
//
// Worker threads (one per slot) take requests first-in first-out from a
// queue; a request is admitted when the footprint estimates of the requests
// running stay within the device-memory budget, or when nothing else runs.
// Each worker runs setup, plane waves and the solve of its request through
// the public entry points on its own default stream (the library is built
// with per-thread default streams), so requests overlap on the device.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>

#include "problem.h"

using namespace sie;

namespace {

struct Job {
    uint64_t ticket = 0;
    sie_problem *p = nullptr;
    std::vector<double> khat;
    std::vector<sie_c128> e0;
    sie_precision prec = SIE_FP32;
    sie_solver_opts opts{};
    bool has_opts = false;
    sie_job_info info{};
    std::string error;
};

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// Device bytes of one problem, estimated from its description: near-field
// CSR of every medium (FP64 L, K and direct L, FP32 L and K, column index;
// rows times an estimate of the RWG functions within the near region),
// grid buffers and spectra, and the Krylov bases of the solve (outer
// dimension `restart`, nested max(restart, min(inner_max_iter, 300))).
size_t sie::estimate_footprint(const sie_problem *p, int restart, int inner_max_iter) {
    int64_t T = 0;
    for (const auto &o : p->objs) T += (int64_t)o.tri.size() / 3;
    const double E = 1.5 * (double)T;
    auto grid_bytes = [&](int n, int R, double rows) {
        const int nn = n > 0 ? n : 64;
        const int Rr = R > 0 ? R : 5;
        // RWG functions in the (2R+1)^2 surface cells around a row: about 40
        // per cell on the structured and geodesic meshes of the workloads
        const double cols = std::min(E, 40.0 * (2 * Rr + 1) * (2 * Rr + 1));
        const double near = rows * cols * (3 * 16 + 2 * 8 + 4);
        double m = 1;
        while (m < 2 * nn - 1) m *= 2;
        const double fft = 3.0 * m * m * m * 16.0;        // buffers + spectra (octants, both precisions)
        return near + fft;
    };
    // near-field fill transients of one medium at a time (freed before the
    // next): pair blocks of a chunk (at most 30M pairs x 27 complex128) and
    // the precorrection tables of its rows (at most 4 GB)
    auto fill_bytes = [&](int R, double tris) {
        const int Rr = R > 0 ? R : 5;
        const double pairs = tris * std::min(tris, 27.0 * (2 * Rr + 1) * (2 * Rr + 1));
        const double tab = tris * std::pow(2.0 * Rr + 3.0, 3) * 10.0 * 16.0;
        return std::min(pairs, 30e6) * 27.0 * 16.0 + std::min(tab, 4e9);
    };
    double b = grid_bytes(p->ext_req.n, p->ext_req.R, E);
    double transient = fill_bytes(p->ext_req.R, (double)T);
    for (size_t i = 0; i < p->obj_req.size(); ++i) {
        const double rows = p->objs.empty() ? 0.0 : 1.5 * (double)p->objs[i].tri.size() / 3.0;
        b += grid_bytes(p->obj_req[i].n, p->obj_req[i].R, rows);
        if (!p->objs.empty()) transient = std::max(transient, fill_bytes(p->obj_req[i].R, (double)p->objs[i].tri.size() / 3.0));
    }
    b += transient;
    if (p->aug_mode == 1) {
        // augmented EFIE: the exterior A0 near values, the pulse integrals per
        // near pair, the charge unknowns in the outer basis, the Schur factors
        const double cols = std::min(E, 40.0 * 121.0);
        b += E * cols * 16.0 + (double)T * std::min((double)T, 27.0 * 121.0) * 16.0;
        b += (double)T * (2.0 * restart + 1.0) * 16.0 + (double)T * 200.0 * 16.0;
    }
    const int mi = std::max(restart, std::min(inner_max_iter, 300));
    b += E * ((2.0 * restart + 1.0) + (2.0 * mi + 1.0)) * (16.0 + 8.0);   // outer and nested bases, FP64 + FP32
    b += E * 64.0 * 16.0;                                     // vectors of the solve
    return (size_t)b;
}

struct sie_server {
    sie_ctx *ctx = nullptr;
    size_t budget = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;       // queue / admission changes
    std::condition_variable done_cv;  // a request finished
    std::deque<Job *> queue;
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    uint64_t next = 1;
    size_t in_use = 0;
    int running = 0;
    bool stop = false;
    std::vector<std::thread> workers;

    void work() {
        (void)hipSetDevice(ctx->device);
        mark_worker_thread();
        while (true) {
            Job *j = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] {
                    if (stop) return true;
                    if (queue.empty()) return false;
                    const size_t fp = queue.front()->info.footprint;
                    return running == 0 || in_use + fp <= budget;
                });
                if (stop && queue.empty()) return;
                if (queue.empty()) continue;
                const size_t fp = queue.front()->info.footprint;
                if (!(running == 0 || in_use + fp <= budget)) continue;
                j = queue.front();
                queue.pop_front();
                in_use += fp;
                ++running;
                j->info.running = 1;
                j->info.t_start_s = now_s(t0);
            }
            sie_status st = SIE_OK;
            sie_report rep{};
            if (!j->p->is_setup) st = sie_problem_setup(j->p);
            if (st == SIE_OK)
                st = sie_set_planewaves(j->p, (int32_t)(j->khat.size() / 3), j->khat.data(), j->e0.data());
            if (st == SIE_OK) st = sie_solve(j->p, j->prec, j->has_opts ? &j->opts : nullptr, &rep);
            const std::string err = st == SIE_OK ? std::string() : std::string(sie_last_error());
            {
                std::lock_guard<std::mutex> lk(mu);
                in_use -= j->info.footprint;
                --running;
                j->info.running = 0;
                j->info.done = 1;
                j->info.status = st;
                j->info.report = rep;
                j->info.t_end_s = now_s(t0);
                j->error = err;
                std::snprintf(j->info.message, sizeof(j->info.message), "%s", err.c_str());
            }
            cv.notify_all();
            done_cv.notify_all();
        }
    }
};

template <typename F>
static sie_status sguard(sie_ctx *ctx, F &&f) {
    std::string msg;
    sie_status st = SIE_OK;
    try {
        set_last_error("");
        f();
        return SIE_OK;
    } catch (const Error &e) {
        msg = e.what(); st = e.code;
    } catch (const std::bad_alloc &) {
        msg = "host allocation failed"; st = SIE_ENOMEM;
    } catch (const std::exception &e) {
        msg = e.what(); st = SIE_EINVAL;
    }
    set_last_error(msg);
    if (ctx) ctx_set_error(ctx, msg);
    return st;
}

extern "C" {

sie_status sie_problem_footprint(const sie_problem *p, size_t *device_bytes) {
    return sguard(p ? p->ctx : nullptr, [&] {
        SIE_CHECK(p && device_bytes, SIE_EINVAL, "NULL argument");
        SIE_CHECK(!p->objs.empty(), SIE_ESTATE, "no objects");
        *device_bytes = estimate_footprint(p, 100, 800);
    });
}

sie_status sie_server_create(sie_ctx *ctx, size_t hbm_budget_bytes, int32_t max_slots, sie_server **out) {
    return sguard(ctx, [&] {
        SIE_CHECK(ctx && out, SIE_EINVAL, "NULL argument");
        SIE_CHECK(max_slots >= 1 && max_slots <= 64, SIE_EINVAL, "max_slots must be 1..64");
        SIE_HIP(hipSetDevice(ctx->device));
        size_t budget = hbm_budget_bytes;
        if (budget == 0) {
            size_t fr = 0, tot = 0;
            SIE_HIP(hipMemGetInfo(&fr, &tot));
            int dev = 0;
            SIE_HIP(hipGetDevice(&dev));
            budget = (size_t)(0.8 * (double)(fr + pool_cached_bytes(dev)));   // cached blocks are free to reuse
        }
        auto *s = new sie_server;
        s->ctx = ctx;
        s->budget = budget;
        s->t0 = std::chrono::steady_clock::now();
        for (int i = 0; i < max_slots; ++i) s->workers.emplace_back([s] { s->work(); });
        *out = s;
    });
}

sie_status sie_server_submit(sie_server *s, sie_problem *p, int32_t nrhs, const double *khat, const sie_c128 *e0,
                             sie_precision prec, const sie_solver_opts *opts, uint64_t *ticket) {
    return sguard(s ? s->ctx : nullptr, [&] {
        SIE_CHECK(s && p && khat && e0 && ticket, SIE_EINVAL, "NULL argument");
        SIE_CHECK(nrhs >= 1, SIE_EINVAL, "need at least one plane wave");
        SIE_CHECK(prec == SIE_FP64 || prec == SIE_FP32, SIE_EINVAL, "unknown precision");
        SIE_CHECK(!p->objs.empty(), SIE_ESTATE, "no objects");
        auto j = std::make_unique<Job>();
        j->p = p;
        j->khat.assign(khat, khat + 3 * (size_t)nrhs);
        j->e0.assign(e0, e0 + 3 * (size_t)nrhs);
        j->prec = prec;
        if (opts) { j->opts = *opts; j->has_opts = true; }
        j->info.footprint = estimate_footprint(p, opts && opts->restart > 0 ? opts->restart : 100,
                                               opts && opts->inner_max_iter > 0 ? opts->inner_max_iter : 800);
        j->info.status = SIE_OK;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            SIE_CHECK(!s->stop, SIE_ESTATE, "server is shutting down");
            j->ticket = s->next++;
            j->info.t_submit_s = now_s(s->t0);
            *ticket = j->ticket;
            s->queue.push_back(j.get());
            s->jobs[j->ticket] = std::move(j);
        }
        s->cv.notify_all();
    });
}

sie_status sie_server_poll(sie_server *s, uint64_t ticket, sie_job_info *info) {
    return sguard(s ? s->ctx : nullptr, [&] {
        SIE_CHECK(s && info, SIE_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->jobs.find(ticket);
        SIE_CHECK(it != s->jobs.end(), SIE_EINVAL, "unknown ticket");
        *info = it->second->info;
    });
}

sie_status sie_server_take(sie_server *s, uint64_t ticket, sie_problem **out) {
    return sguard(s ? s->ctx : nullptr, [&] {
        SIE_CHECK(s && out, SIE_EINVAL, "NULL argument");
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->jobs.find(ticket);
        SIE_CHECK(it != s->jobs.end(), SIE_EINVAL, "unknown ticket");
        Job *j = it->second.get();
        s->done_cv.wait(lk, [&] { return j->info.done != 0; });
        *out = j->p;
        s->jobs.erase(it);
    });
}

void sie_server_destroy(sie_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        // requests not started yet are dropped (their problems destroyed below)
        s->queue.clear();
        s->stop = true;
    }
    s->cv.notify_all();
    for (auto &t : s->workers) t.join();
    for (auto &kv : s->jobs) sie_problem_destroy(kv.second->p);
    delete s;
}

}  // extern "C"
