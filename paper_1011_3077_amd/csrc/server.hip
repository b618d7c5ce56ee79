// Served form of the split step (include/sdc.h, sdc_server_*): a request
// queue, HBM-budget admission and continuous batching on one worker thread.
//
// The worker owns a handle with its own stream.  Each loop it admits waiting
// requests (arrival order, while the admitted workspaces fit the budget and
// fewer than max_active run), gives each its own device workspace, runs one
// tick of the incremental driver over every admitted request (one
// repeated-squaring iteration each; the finishing stage for those whose
// squaring ended), then completes the finished ones and frees their memory.
// Independent requests are the independent subproblems of Sec. 4.3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.hpp"
#include "engine_util.hpp"
#include "sdc.h"

using Clock = std::chrono::steady_clock;

namespace {

struct Request {
    long long ticket = 0;
    bool fallback = false;  // redone in FP64 after failed FP32 attempts
    sdc::SplitJob job;
    Clock::time_point t_submit;
    size_t bytes = 0;
    char* ws = nullptr;
    sdc::JobRun* run = nullptr;
};

struct Result {
    bool done = false;
    int status = 0;
    sdc_info_t info{};
};

double nominal_flops(const sdc::SplitJob& j) {
    const double m3 = (double)j.n * j.n * j.n;
    if (j.pencil) return (40.0 / 3.0 * (j.info.iters_right + j.info.iters_left) + 32.0) * m3;
    return (40.0 / 3.0 * j.info.iters_right + 16.0) * m3;
}

}  // namespace

struct sdc_server_s {
    int device = 0;
    size_t budget = 0;
    int max_active = 64;
    sdc::Handle h;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::vector<Request*> active;
    std::unordered_map<long long, Result> results;
    long long next_ticket = 1;
    bool stop = false;
    // statistics (under mu)
    std::vector<double> lat_ms;
    long long submitted = 0, completed = 0, failed = 0, ticks = 0;
    int peak_active = 0;
    size_t used = 0, peak_bytes = 0;
    double flops = 0;
    bool any_submit = false;
    Clock::time_point t_first, t_last;

    void complete(Request* r, int status) {
        const double ms = std::chrono::duration<double, std::milli>(Clock::now() - r->t_submit).count();
        Result& res = results[r->ticket];
        res.done = true;
        res.status = status;
        res.info = r->job.info;
        res.info.ms = ms;
        res.info.fp64_fallback = r->fallback ? 1 : 0;
        lat_ms.push_back(ms);
        ++completed;
        if (status < 0) ++failed;
        else flops += nominal_flops(r->job);
        t_last = Clock::now();
    }

    void release(Request* r) {
        if (r->run) sdc::job_run_destroy(r->run);
        if (r->ws) (void)hipFree(r->ws);
        delete r;
    }

    void loop();
};

void sdc_server_s::loop() {
    (void)hipSetDevice(device);
    std::vector<char> done;
    for (;;) {
        std::vector<Request*> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                while (!pending.empty() && (int)(active.size() + admitted.size()) < max_active) {
                    Request* r = pending.front();
                    if (r->bytes > budget) {  // can never fit
                        pending.pop_front();
                        complete(r, SDC_ERR_NOMEM);
                        release(r);
                        cv_done.notify_all();
                        continue;
                    }
                    if (used + r->bytes > budget) break;  // wait for memory
                    pending.pop_front();
                    used += r->bytes;
                    peak_bytes = std::max(peak_bytes, used);
                    admitted.push_back(r);
                }
                if (!active.empty() || !admitted.empty()) break;
                if (stop && pending.empty()) return;
                cv_work.wait(lk);
            }
        }
        // workspaces of the newly admitted requests (outside the lock)
        for (Request* r : admitted) {
            int st = SDC_OK;
            if (hipMalloc(reinterpret_cast<void**>(&r->ws), r->bytes) != hipSuccess) {
                r->ws = nullptr;
                st = SDC_ERR_NOMEM;
            } else {
                r->run = sdc::job_run_create(h, &r->job, r->ws, r->bytes);
                if (!r->run) st = SDC_ERR_NOMEM;
            }
            if (st != SDC_OK) {
                (void)hipGetLastError();
                std::lock_guard<std::mutex> lk(mu);
                used -= r->bytes;
                complete(r, st);
                release(r);
                cv_done.notify_all();
                continue;
            }
            std::lock_guard<std::mutex> lk(mu);
            active.push_back(r);
        }
        if (active.empty()) continue;
        std::vector<sdc::JobRun*> runs;
        for (Request* r : active) runs.push_back(r->run);
        const int rc = sdc::job_runs_tick(h, runs, done);
        std::lock_guard<std::mutex> lk(mu);
        ++ticks;
        peak_active = std::max(peak_active, (int)active.size());
        std::vector<Request*> keep;
        for (size_t i = 0; i < active.size(); ++i) {
            Request* r = active[i];
            if (rc >= 0 && done[i] && r->job.opts.prec == SDC_FP32_REFINE &&
                sdc::fp32_needs_fallback(r->job.status)) {
                // every FP32 attempt failed: requeue first in line, in FP64
                used -= r->bytes;
                sdc::job_run_destroy(r->run);
                r->run = nullptr;
                (void)hipFree(r->ws);
                r->ws = nullptr;
                r->fallback = true;
                r->job.opts.prec = SDC_FP64;
                r->job.status = 0;
                r->job.info = sdc_info_t{};
                r->job.info.n = r->job.n;
                r->bytes = sdc::job_run_bytes(r->job);
                pending.push_front(r);
            } else if (rc < 0 || done[i]) {
                used -= r->bytes;
                complete(r, rc < 0 ? rc : r->job.status);
                release(r);
            } else {
                keep.push_back(r);
            }
        }
        if (rc < 0) (void)hipDeviceSynchronize();
        active.swap(keep);
        cv_done.notify_all();
    }
}

extern "C" {

sdc_status_t sdc_server_create(sdc_server_t* server, int device, size_t budget, int max_active) {
    if (!server) return SDC_ERR_INVALID;
    *server = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SDC_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return SDC_ERR_DEVICE;
    sdc_server_s* s = new (std::nothrow) sdc_server_s;
    if (!s) return SDC_ERR_NOMEM;
    s->device = device;
    s->max_active = max_active > 0 ? max_active : 64;
    if (budget == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            delete s;
            return SDC_ERR_DEVICE;
        }
        budget = free_b / 10 * 8;
    }
    s->budget = budget;
    s->h.device = device;
    if (hipStreamCreate(&s->h.stream) != hipSuccess) {
        delete s;
        return SDC_ERR_DEVICE;
    }
    s->worker = std::thread([s] { s->loop(); });
    *server = s;
    return SDC_OK;
}

sdc_status_t sdc_server_submit(sdc_server_t s, const sdc_request_t* q, long long* ticket) {
    if (!s || !q || !ticket) return SDC_ERR_INVALID;
    const int n = q->n;
    const bool pencil = q->kind == SDC_REQ_PENCIL;
    if ((q->kind != SDC_REQ_SYM && !pencil) || n < 1 || n > sdc::kMaxN || !q->A || q->lda < n || !q->Q ||
        q->ldq < n || !q->Ahat || q->ldah < n || !sdc::region_ok(q->region) || !sdc::prec_ok(q->opts, pencil, q->region.kind))
        return SDC_ERR_INVALID;
    if (pencil && (!q->B || q->ldb < n || !q->QL || q->ldql < n || !q->Bhat || q->ldbh < n)) return SDC_ERR_INVALID;
    Request* r = new (std::nothrow) Request;
    if (!r) return SDC_ERR_NOMEM;
    sdc::SplitJob& j = r->job;
    j.n = n; j.pencil = pencil; j.A = q->A; j.lda = q->lda; j.region = q->region; j.opts = q->opts;
    j.Q = q->Q; j.ldq = q->ldq; j.Ahat = q->Ahat; j.ldah = q->ldah;
    if (pencil) {
        j.B = q->B; j.ldb = q->ldb; j.QL = q->QL; j.ldql = q->ldql; j.Bhat = q->Bhat; j.ldbh = q->ldbh;
    }
    j.info.n = n;
    r->bytes = sdc::job_run_bytes(j);
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            return SDC_ERR_INVALID;
        }
        r->ticket = s->next_ticket++;
        s->results[r->ticket] = Result{};
        s->pending.push_back(r);
        ++s->submitted;
        if (!s->any_submit) {
            s->any_submit = true;
            s->t_first = r->t_submit;
        }
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return SDC_OK;
}

static sdc_status_t take_result(sdc_server_s* s, long long ticket, int* status, sdc_info_t* info) {
    auto it = s->results.find(ticket);
    if (status) *status = it->second.status;
    if (info) *info = it->second.info;
    s->results.erase(it);
    s->cv_done.notify_all();  // another waiter on this ticket now sees it released
    return SDC_OK;
}

sdc_status_t sdc_server_poll(sdc_server_t s, long long ticket, int* done, int* status, sdc_info_t* info) {
    if (!s || !done) return SDC_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return SDC_ERR_INVALID;
    *done = it->second.done ? 1 : 0;
    if (!*done) return SDC_OK;
    return take_result(s, ticket, status, info);
}

sdc_status_t sdc_server_wait(sdc_server_t s, long long ticket, int* status, sdc_info_t* info) {
    if (!s) return SDC_ERR_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return SDC_ERR_INVALID;
    // a second waiter on the same ticket wakes when the first takes the
    // result and then reports the ticket as released
    s->cv_done.wait(lk, [&] {
        auto jt = s->results.find(ticket);
        return jt == s->results.end() || jt->second.done;
    });
    if (s->results.find(ticket) == s->results.end()) return SDC_ERR_INVALID;
    return take_result(s, ticket, status, info);
}

sdc_status_t sdc_server_stats(sdc_server_t s, sdc_server_stats_t* out) {
    if (!s || !out) return SDC_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    sdc_server_stats_t r{};
    r.submitted = s->submitted;
    r.completed = s->completed;
    r.failed = s->failed;
    r.active = (int)s->active.size();
    r.pending = (int)s->pending.size();
    r.peak_active = s->peak_active;
    r.ticks = s->ticks;
    r.peak_bytes = s->peak_bytes;
    r.budget_bytes = s->budget;
    r.nominal_flops = s->flops;
    if (!s->lat_ms.empty()) {
        std::vector<double> v = s->lat_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            const size_t i = (size_t)std::min<double>(v.size() - 1, std::ceil(q * v.size()) - 1);
            return v[i];
        };
        r.p50_ms = pct(0.50);
        r.p99_ms = pct(0.99);
        r.max_ms = v.back();
        double sum = 0;
        for (double x : v) sum += x;
        r.mean_ms = sum / v.size();
        r.wall_ms = std::chrono::duration<double, std::milli>(s->t_last - s->t_first).count();
    }
    *out = r;
    return SDC_OK;
}

sdc_status_t sdc_server_destroy(sdc_server_t s) {
    if (!s) return SDC_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->device);
    sdc::Handle& h = s->h;
    if (h.stream) (void)hipStreamSynchronize(h.stream);
    if (h.ws) (void)hipFree(h.ws);
    if (h.desc_d) (void)hipFree(h.desc_d);
    if (h.desc_h) (void)hipHostFree(h.desc_h);
    if (h.host) (void)hipHostFree(h.host);
    if (h.ws2) (void)hipFree(h.ws2);
    if (h.dnorm) (void)hipFree(h.dnorm);
    if (h.dstage) (void)hipFree(h.dstage);
    if (h.ev_sync) (void)hipEventDestroy(h.ev_sync);
    if (h.ev_desc) (void)hipEventDestroy(h.ev_desc);
    sdc::release_streams(h);
    if (h.stream) (void)hipStreamDestroy(h.stream);
    delete s;
    return SDC_OK;
}

}  // extern "C"
