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

// A prepared request on its way to the packed engine: its handle (set up and
// factored) and its staging buffers.
struct Prepared {
    Request* r = nullptr;
    rbf_problem* h = nullptr;
    void *b_pts = nullptr, *b_vals = nullptr, *b_lam = nullptr;
    size_t g_pts = 0, g_vals = 0, g_lam = 0;
};

struct rbf_server {
    rbf_server_opts opts{};
    int device = 0;
    size_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_engine;
    std::deque<Request*> queue, ready;
    std::deque<Prepared> prepared;    // packed: set up, waiting to join the engine
    std::map<long long, std::unique_ptr<Request>> reqs;
    int active = 0;
    size_t used = 0;
    long long next_id = 0, finished = 0;
    bool stopping = false;
    int workers_left = 0;
    std::thread dispatcher;
    std::vector<std::thread> workers, engines;
    std::vector<int> engine_load;      // solves each engine is running

    // a request's end: its result recorded, its slot and budget freed
    void complete(Request* r, rbf_status s, const std::string& msg, const rbf_solve_info& info) {
        std::lock_guard<std::mutex> lk(mu);
        r->status = s;
        r->message = s == RBF_OK ? std::string() : msg;
        r->info = info;
        r->info.history = nullptr;
        r->info.history_len = 0;
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

    // The packed engine's thread: prepared requests join at step boundaries,
    // every active solve advances one step per engine step, ended ones are
    // copied out and released.
    // Several engines (each a thread and a stream) share the prepared requests,
    // each taking new ones only while it runs no more than any other: while one
    // engine's host reads its step's results and updates its recurrences, the
    // others' steps keep the device busy.
    void engine_loop(int id) {
        (void)hipSetDevice(device);
        hipStream_t st = nullptr;
        if (hipStreamCreate(&st) != hipSuccess) st = nullptr;
        rbf::Engine* eng = st ? rbf::engine_create(st, opts.max_active, opts.graphs != 0) : nullptr;
        std::map<void*, Prepared> running;
        std::vector<rbf::EngineDone> done;
        for (;;) {
            std::deque<Prepared> joining;
            {
                std::unique_lock<std::mutex> lk(mu);
                auto least = [&] {
                    for (int l : engine_load)
                        if (l < engine_load[id]) return false;
                    return true;
                };
                cv_engine.wait(lk, [&] {
                    return (!prepared.empty() && least()) || !running.empty() ||
                           (stopping && workers_left == 0);
                });
                if (prepared.empty() && running.empty()) break;
                while (!prepared.empty() && least()) {
                    joining.push_back(prepared.front());
                    prepared.pop_front();
                    ++engine_load[id];
                }
            }
            for (Prepared& pr : joining) {
                rbf_solve_opts o = pr.r->opts;
                o.stream = st;
                rbf_status s = eng ? rbf::engine_add(eng, pr.h, o, static_cast<double*>(pr.b_lam), pr.r)
                                   : RBF_EDEVICE;
                if (s == RBF_OK) {
                    running[pr.r] = pr;
                } else {   // cannot be packed (no lists, or no engine): solve it alone here
                    rbf_solve_info info{};
                    s = rbf_solve_device(pr.h, &o, nullptr, static_cast<double*>(pr.b_lam), &info);
                    const std::string msg = s == RBF_OK ? std::string() : std::string("solve: ") + rbf_last_error();
                    finish(pr, st, s, msg, info);
                    unload(id);
                }
            }
            if (running.empty()) continue;
            done.clear();
            const rbf_status es = rbf::engine_step(eng, &done);
            if (es != RBF_OK) {   // a device error: every running request fails
                const std::string msg = std::string("engine: ") + rbf_last_error();
                for (auto& kv : running) {
                    finish(kv.second, st, es, msg, rbf_solve_info{});
                    unload(id);
                }
                running.clear();
                rbf::engine_destroy(eng);
                eng = rbf::engine_create(st, opts.max_active, false);
                continue;
            }
            for (const rbf::EngineDone& d : done) {
                auto it = running.find(d.tag);
                if (it == running.end()) continue;
                rbf_solve_info info{};
                rbf::engine_info(it->second.h, &info);
                finish(it->second, st, d.status,
                       d.status == RBF_OK ? std::string() : std::string("solve: ") + d.message, info);
                running.erase(it);
                unload(id);
            }
        }
        if (eng) rbf::engine_destroy(eng);
        if (st) (void)hipStreamDestroy(st);
    }

    void unload(int id) {
        std::lock_guard<std::mutex> lk(mu);
        --engine_load[id];
        cv_engine.notify_all();
    }

    // copy out, release, complete (weights also on RBF_ENOCONV)
    void finish(Prepared& pr, hipStream_t st, rbf_status s, const std::string& msg,
                const rbf_solve_info& info) {
        Request* r = pr.r;
        const size_t nb = sizeof(double) * (size_t)r->n;
        rbf_status out = s;
        std::string m = msg;
        if (s == RBF_OK || s == RBF_ENOCONV) {
            r->lambda.resize(r->n);
            hipError_t e = hipMemcpyAsync(r->lambda.data(), pr.b_lam, nb, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                out = RBF_EDEVICE;
                m = std::string("copy-out: ") + hipGetErrorString(e);
            }
        }
        rbf_destroy(pr.h);
        if (pr.b_pts) rbf::cached_free(device, pr.b_pts, pr.g_pts, st);
        if (pr.b_vals) rbf::cached_free(device, pr.b_vals, pr.g_vals, st);
        if (pr.b_lam) rbf::cached_free(device, pr.b_lam, pr.g_lam, st);
        complete(r, out, m, info);
    }

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
        if (s == RBF_OK && opts.packed &&
            (opts.pack_max_points == 0 || r->n <= opts.pack_max_points)) {   // an engine takes it
            std::lock_guard<std::mutex> lk(mu);
            prepared.push_back(Prepared{r, h, b_pts, b_vals, b_lam, g_pts, g_vals, g_lam});
            cv_engine.notify_all();
            return;
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
        rbf_destroy(h);
        if (b_pts) rbf::cached_free(device, b_pts, g_pts, st);
        if (b_vals) rbf::cached_free(device, b_vals, g_vals, st);
        if (b_lam) rbf::cached_free(device, b_lam, g_lam, st);
        complete(r, s, msg, info);
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
        --workers_left;
        cv_engine.notify_all();
        lk.unlock();
        if (st) (void)hipStreamDestroy(st);
    }
};

extern "C" {

void rbf_server_default_opts(rbf_server_opts* o) {
    if (!o) return;
    o->max_active = 8;
    o->max_device_bytes = 0;
    o->packed = 2;
    o->graphs = 1;
    o->pack_max_points = 65536;
}

rbf_status rbf_server_create(const rbf_server_opts* opts, rbf_server** out) {
    if (!out) return RBF_EINVAL;
    *out = nullptr;
    rbf_server_opts o;
    rbf_server_default_opts(&o);
    if (opts) o = *opts;
    if (o.max_active < 1 || o.max_active > 64 || o.packed < 0 || o.packed > 8 ||
        o.pack_max_points < 0)
        return rbf::set_error(RBF_EINVAL, "server options: max_active in 1..64, packed in 0..8, "
                                          "pack_max_points >= 0");
    rbf_server* s = new (std::nothrow) rbf_server();
    if (!s) return rbf::set_error(RBF_ENOMEM, "server allocation");
    s->opts = o;
    hipError_t e = hipGetDevice(&s->device);
    size_t free_b = 0, total_b = 0;
    if (e == hipSuccess) e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) {
        delete s;
        return rbf::set_error(RBF_EDEVICE, "server device query: %s", hipGetErrorString(e));
    }
    s->budget = o.max_device_bytes ? o.max_device_bytes : (size_t)(0.9 * (double)free_b);
    s->workers_left = o.max_active;
    s->dispatcher = std::thread([s] { s->dispatch_loop(); });
    for (int i = 0; i < o.max_active; ++i) s->workers.emplace_back([s] { s->worker_loop(); });
    if (o.packed > 0) {
        s->engine_load.assign(o.packed, 0);
        for (int i = 0; i < o.packed; ++i) s->engines.emplace_back([s, i] { s->engine_loop(i); });
    }
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
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->cv_engine.notify_all();
    }
    for (auto& t : s->engines)
        if (t.joinable()) t.join();
    delete s;
}

}  // extern "C"
