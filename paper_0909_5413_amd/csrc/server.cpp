// server.cpp -- a request loop over many interpolation problems on one GPU.
//
// Requests (points, values, sigma, cutoff, overlap, solve options) are queued
// on submission and admitted in arrival order whenever fewer than max_active
// are on the device and their predicted device footprint fits the remaining
// budget (a request larger than the whole budget is admitted alone).  Each
// admitted request runs on a worker thread, on that worker's own HIP stream
// (default priority, created once per worker): setup, preconditioner, solve,
// copy-out, release.  Device buffers come from the library's block cache, so
// a request neither maps fresh memory nor waits for the device on release.  Requests that
// arrive while others run are admitted as slots and memory free up, and their
// kernels overlap on the device with the running ones.  Every request runs
// exactly the same launches as a lone rbf_solve_device call, so its weights
// do not depend on the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <string>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/rbf.h"
#include "rbf_internal.hpp"

namespace {

using clk = std::chrono::steady_clock;

struct Request {
    long long id = 0;
    std::vector<double> pts, vals;
    long long n = 0;
    double sigma = 0, cutoff = 0;
    int overlap = 1;
    rbf_solve_opts opts{};
    size_t predicted = 0;
    clk::time_point t_submit, t_admit, t_done;
    std::vector<double> lambda;
    rbf_status status = RBF_OK;
    rbf_solve_info info{};
    std::string message;
    bool done = false;
};

// Device bytes a request will hold, from its points alone: cells of side
// `cutoff` over the points' bounding box give the mean block size n_omega;
// Z (n * n_omega values), the neighbour lists (about a third of the block is
// within the cutoff, 16-bit entries, padded), the Krylov basis and vectors,
// the sorted copies, and the setup scratch of one batch, plus 10%.
size_t predict_bytes(const double* pts, long long n, double cutoff, int overlap,
                     const rbf_solve_opts& o) {
    double x0 = pts[0], x1 = pts[0], y0 = pts[1], y1 = pts[1];
    for (long long i = 1; i < n; ++i) {
        x0 = std::min(x0, pts[2 * i]);
        x1 = std::max(x1, pts[2 * i]);
        y0 = std::min(y0, pts[2 * i + 1]);
        y1 = std::max(y1, pts[2 * i + 1]);
    }
    const double ncx = std::floor((x1 - x0) / cutoff) + 1, ncy = std::floor((y1 - y0) / cutoff) + 1;
    const double ncells = ncx * ncy;
    const double per_cell = (double)n / ncells;
    const double k = 2.0 * overlap + 1.0;
    const double n_omega = std::min((double)n, k * k * per_cell * 1.15);
    const double s = o.precision == RBF_MIXED ? 4.0 : 8.0;
    const double m = o.restart > 0 ? o.restart : 30;
    double bytes = (double)n * n_omega * s;                   // Z
    bytes += (double)n * std::min((double)n, 9.0 * per_cell) * 0.4 * 2.0 * 1.3;   // lists
    bytes += (double)n * 8.0 * (m + 1 + 10);                  // Krylov basis and vectors
    bytes += (double)n * 64.0;                                // sorted copies, permutations
    const double b = std::ceil(n_omega * 1.2 / 32.0);
    const double slots = std::min(ncells, 8192.0);
    bytes += std::min(slots * 512.0 * b * (b + 1.0) * s, 12.0 * 1073741824.0);   // setup scratch
    return (size_t)(1.1 * bytes);
}

}  // namespace

struct rbf_server {
    rbf_server_opts opts{};
    int device = 0;
    size_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Request*> queue, ready;
    std::map<long long, std::unique_ptr<Request>> reqs;
    int active = 0;
    size_t used = 0;
    long long next_id = 0, finished = 0;
    bool stopping = false;
    std::thread dispatcher;
    std::vector<std::thread> workers;

    void dispatch_loop() {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_sched.wait(lk, [&] {
                if (stopping && queue.empty()) return true;
                if (queue.empty() || active >= opts.max_active) return false;
                return active == 0 || used + queue.front()->predicted <= budget;
            });
            if (queue.empty()) return;   // stopping
            Request* r = queue.front();
            queue.pop_front();
            ++active;
            used += r->predicted;
            r->t_admit = clk::now();
            ready.push_back(r);
            cv_sched.notify_all();
        }
    }

    void run(Request* r, hipStream_t st) {
        (void)hipSetDevice(device);
        rbf_problem* h = nullptr;
        void *b_pts = nullptr, *b_vals = nullptr, *b_lam = nullptr;
        size_t g_pts = 0, g_vals = 0, g_lam = 0;
        rbf_status s = st ? RBF_OK : RBF_EDEVICE;
        std::string msg;
        auto hip = [&](hipError_t e) {
            if (e != hipSuccess && s == RBF_OK) {
                s = e == hipErrorOutOfMemory ? RBF_ENOMEM : RBF_EDEVICE;
                msg = std::string("request staging: ") + hipGetErrorString(e);
            }
            return s == RBF_OK;
        };
        const size_t nb = sizeof(double) * (size_t)r->n;
        if (s == RBF_OK && hip(rbf::cached_alloc(device, 2 * nb, &b_pts, &g_pts)) &&
            hip(rbf::cached_alloc(device, nb, &b_vals, &g_vals)) &&
            hip(rbf::cached_alloc(device, nb, &b_lam, &g_lam)) &&
            hip(hipMemcpyAsync(b_pts, r->pts.data(), 2 * nb, hipMemcpyHostToDevice, st)) &&
            hip(hipMemcpyAsync(b_vals, r->vals.data(), nb, hipMemcpyHostToDevice, st))) {
            s = rbf_setup_device(static_cast<double*>(b_pts), static_cast<double*>(b_vals), r->n,
                                 r->sigma, r->cutoff, r->overlap, st, &h);
            if (s != RBF_OK) msg = std::string("setup: ") + rbf_last_error();
        }
        double* d_lam = static_cast<double*>(b_lam);
        if (s == RBF_OK) {
            rbf::set_setup_lanes(h, 1);
            s = rbf_precond_setup(h, r->opts.precision, st);
            if (s != RBF_OK) msg = std::string("preconditioner: ") + rbf_last_error();
        }
        rbf_solve_info info{};
        if (s == RBF_OK) {
            rbf_solve_opts o = r->opts;
            o.stream = st;
            s = rbf_solve_device(h, &o, nullptr, d_lam, &info);
            if (s != RBF_OK) msg = std::string("solve: ") + rbf_last_error();
        }
        if (s == RBF_OK || s == RBF_ENOCONV) {
            r->lambda.resize(r->n);
            const rbf_status s2 = s;
            if (hip(hipMemcpyAsync(r->lambda.data(), d_lam, nb, hipMemcpyDeviceToHost, st)) &&
                hip(hipStreamSynchronize(st)))
                s = s2;
        }
        info.history = nullptr;
        info.history_len = 0;
        rbf_destroy(h);
        if (b_pts) rbf::cached_free(device, b_pts, g_pts, st);
        if (b_vals) rbf::cached_free(device, b_vals, g_vals, st);
        if (b_lam) rbf::cached_free(device, b_lam, g_lam, st);
        std::lock_guard<std::mutex> lk(mu);
        r->status = s;
        r->message = s == RBF_OK ? std::string() : msg;
        r->info = info;
        r->t_done = clk::now();
        r->done = true;
        r->pts.clear();
        r->pts.shrink_to_fit();
        r->vals.clear();
        r->vals.shrink_to_fit();
        --active;
        used -= r->predicted;
        ++finished;
        cv_sched.notify_all();
        cv_done.notify_all();
    }

    void worker_loop() {
        (void)hipSetDevice(device);
        hipStream_t st = nullptr;
        if (hipStreamCreate(&st) != hipSuccess) st = nullptr;
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_sched.wait(lk, [&] { return !ready.empty() || (stopping && queue.empty() && ready.empty()); });
            if (ready.empty()) break;
            Request* r = ready.front();
            ready.pop_front();
            lk.unlock();
            run(r, st);
            lk.lock();
        }
        lk.unlock();
        if (st) (void)hipStreamDestroy(st);
    }
};

extern "C" {

void rbf_server_default_opts(rbf_server_opts* o) {
    if (!o) return;
    o->max_active = 8;
    o->max_device_bytes = 0;
}

rbf_status rbf_server_create(const rbf_server_opts* opts, rbf_server** out) {
    if (!out) return RBF_EINVAL;
    *out = nullptr;
    rbf_server_opts o;
    rbf_server_default_opts(&o);
    if (opts) o = *opts;
    if (o.max_active < 1 || o.max_active > 64) return RBF_EINVAL;
    rbf_server* s = new (std::nothrow) rbf_server();
    if (!s) return RBF_ENOMEM;
    s->opts = o;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return RBF_EDEVICE;
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        delete s;
        return RBF_EDEVICE;
    }
    s->budget = o.max_device_bytes ? o.max_device_bytes : (size_t)(0.9 * (double)free_b);
    s->dispatcher = std::thread([s] { s->dispatch_loop(); });
    for (int i = 0; i < o.max_active; ++i) s->workers.emplace_back([s] { s->worker_loop(); });
    *out = s;
    return RBF_OK;
}

rbf_status rbf_server_submit(rbf_server* s, const double* points, const double* values,
                             long long n, double sigma, double cutoff, int overlap,
                             const rbf_solve_opts* opts, long long* id) {
    if (!s || !points || !values || !id || n < 1) return RBF_EINVAL;
    auto r = std::make_unique<Request>();
    r->pts.assign(points, points + 2 * n);
    r->vals.assign(values, values + n);
    r->n = n;
    r->sigma = sigma;
    r->cutoff = cutoff;
    r->overlap = overlap;
    if (opts)
        r->opts = *opts;
    else
        rbf_default_opts(&r->opts);
    if (!(cutoff > 0) || overlap < 0) return RBF_EINVAL;
    r->predicted = predict_bytes(points, n, cutoff, overlap, r->opts);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return RBF_ESTATE;
    r->id = s->next_id++;
    r->t_submit = clk::now();
    *id = r->id;
    s->queue.push_back(r.get());
    s->reqs[r->id] = std::move(r);
    s->cv_sched.notify_all();
    return RBF_OK;
}

rbf_status rbf_server_wait(rbf_server* s, long long id, double* lambda_out,
                           rbf_request_result* result) {
    if (!s) return RBF_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return RBF_EINVAL;
    Request* r = it->second.get();
    s->cv_done.wait(lk, [&] { return r->done; });
    if (lambda_out && !r->lambda.empty())
        std::copy(r->lambda.begin(), r->lambda.end(), lambda_out);
    if (result) {
        using sec = std::chrono::duration<double>;
        result->status = r->status;
        result->info = r->info;
        result->t_queue = sec(r->t_admit - r->t_submit).count();
        result->t_run = sec(r->t_done - r->t_admit).count();
        result->latency = sec(r->t_done - r->t_submit).count();
        result->predicted_bytes = r->predicted;
        std::snprintf(result->message, sizeof result->message, "%s", r->message.c_str());
    }
    const rbf_status st = r->status;
    s->reqs.erase(it);
    return st;
}

rbf_status rbf_server_stats(rbf_server* s, long long* submitted, long long* finished,
                            int* active, int* queued, size_t* bytes_charged) {
    if (!s) return RBF_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (submitted) *submitted = s->next_id;
    if (finished) *finished = s->finished;
    if (active) *active = s->active;
    if (queued) *queued = (int)s->queue.size();
    if (bytes_charged) *bytes_charged = s->used;
    return RBF_OK;
}

void rbf_server_destroy(rbf_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cv_sched.notify_all();
    }
    if (s->dispatcher.joinable()) s->dispatcher.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->cv_sched.notify_all();
    }
    for (auto& t : s->workers)
        if (t.joinable()) t.join();
    delete s;
}

}  // extern "C"
