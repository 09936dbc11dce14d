// capi.cpp -- host driver and C ABI (include/rbf.h).
//
// Runs the whole method on one GPU: binning, RASM setup, right-preconditioned
// GMRES(m) (Section 2.2) in FP64 or as FP32 inner solves inside an FP64
// residual-correction loop, and evaluation of the interpolant (eq. rbf1).
// Every step is a kernel from binning.hip / matvec.hip / precond.hip /
// krylov.hip; the host only sizes buffers, launches, and runs the m x m
// Hessenberg least-squares recurrence (Givens rotations), which is O(m) work
// per Arnoldi step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rbf.h"
#include "rbf_internal.hpp"

using rbf::Grid;

static constexpr double kPi = 3.14159265358979323846;
static constexpr long double kLn2L = 0.693147180559945309417232121458176568L;

namespace {

thread_local std::string g_last_error;

rbf_status fail(rbf_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? RBF_ENOMEM : RBF_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                \
    } while (0)

#define RBF_TRY(expr)                    \
    do {                                 \
        rbf_status s_ = (expr);          \
        if (s_ != RBF_OK) return s_;     \
    } while (0)

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double sec() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

// device buffer owned by a problem
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Device blocks released by problems, kept for reuse by later allocations of
// about the same size.  A fresh multi-GB hipMalloc maps new pages and hipFree
// waits for the whole device, which together cost more than a solve when
// problems of varying sizes follow one another (the serving loop).  A block is
// taken back only once the work that used it has finished: the releasing call
// waits for its own stream first (at that point nearly always idle already),
// so that nothing in the cache refers to a stream that may be destroyed later.
// Idle blocks are returned to the runtime when an allocation fails, when they
// exceed a quarter of the device memory, or on rbf_block_cache.
class BlockCache {
public:
    static BlockCache& get() {
        static BlockCache* c = new BlockCache;  // outlives every static destructor
        return *c;
    }
    // Sizes are rounded so that blocks of one size class are interchangeable.
    static size_t round(size_t b) {
        if (b <= 256) return 256;
        if (b < (1u << 20)) {
            size_t r = 256;
            while (r < b) r <<= 1;
            return r;
        }
        const size_t g = 2u << 20;
        return (b + g - 1) / g * g;
    }
    // A block of at least `want` (rounded) and at most `limit` bytes; *got is
    // its size.  An idle block may be up to 1/8 larger than asked for, or up to
    // 1/2 larger for blocks of 64 MiB and more: requests of a serving stream
    // differ in size, and a miss on a large block (a fresh hipMalloc, ~15 ms,
    // and sooner or later a hipFree that waits for the device) costs far more
    // than the memory a larger idle block leaves unused while it is held.
    hipError_t alloc(int dev, size_t want, size_t limit, void** out, size_t* got) {
        const size_t r = round(want);
        const size_t hi = std::min(limit, r >= (64u << 20) ? r + r / 2 : r + r / 8);
        Blk b{};
        bool found = false;
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (auto it = idle_.lower_bound(r); it != idle_.end() && it->first <= hi; ++it)
                if (it->second.dev == dev) {
                    b = it->second;
                    idle_.erase(it);
                    idle_bytes_[dev] -= b.bytes;
                    found = true;
                    break;
                }
        }
        if (found) {
            *out = b.p;
            *got = b.bytes;
            return hipSuccess;
        }
        if (r > limit) return hipErrorOutOfMemory;
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, r);
        if (e == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            trim(dev);
            e = hipMalloc(&p, r);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        *out = p;
        *got = r;
        return hipSuccess;
    }
    // Takes back a block; pending: work enqueued on `st` before this call may
    // still use it (waited for here).
    void put(int dev, void* p, size_t bytes, hipStream_t st, bool pending) {
        if (pending && hipStreamSynchronize(st) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipDeviceSynchronize();
        }
        Blk b{p, bytes, dev};
        std::vector<Blk> evict;
        {
            std::lock_guard<std::mutex> lk(mu_);
            idle_.emplace(bytes, b);
            idle_bytes_[dev] += bytes;
            const size_t cap = cap_locked(dev);
            // evict the largest idle blocks of the device beyond the cap
            for (auto it = idle_.end(); idle_bytes_[dev] > cap && it != idle_.begin();) {
                --it;
                if (it->second.dev != dev) continue;
                idle_bytes_[dev] -= it->second.bytes;
                evict.push_back(it->second);
                it = idle_.erase(it);
            }
        }
        for (Blk& e : evict) (void)hipFree(e.p);
    }
    // Returns the idle blocks of device dev (all devices if dev < 0) to the
    // runtime; the number of bytes freed.
    size_t trim(int dev) {
        std::vector<Blk> evict;
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (auto it = idle_.begin(); it != idle_.end();) {
                if (dev < 0 || it->second.dev == dev) {
                    idle_bytes_[it->second.dev] -= it->second.bytes;
                    evict.push_back(it->second);
                    it = idle_.erase(it);
                } else {
                    ++it;
                }
            }
        }
        size_t freed = 0;
        for (Blk& e : evict) {
            (void)hipFree(e.p);
            freed += e.bytes;
        }
        return freed;
    }
    size_t idle_bytes(int dev) {
        std::lock_guard<std::mutex> lk(mu_);
        size_t t = 0;
        for (auto& kv : idle_bytes_)
            if (dev < 0 || kv.first == dev) t += kv.second;
        return t;
    }

private:
    struct Blk {
        void* p;
        size_t bytes;
        int dev;
    };
    size_t cap_locked(int dev) {
        auto it = cap_.find(dev);
        if (it != cap_.end()) return it->second;
        size_t fr = 0, tot = 0;
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(dev);
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) tot = 0;
        (void)hipSetDevice(cur);
        const size_t cap = tot / 4;
        cap_[dev] = cap;
        return cap;
    }
    std::mutex mu_;
    std::multimap<size_t, Blk> idle_;
    std::map<int, size_t> idle_bytes_;
    std::map<int, size_t> cap_;
};

}  // namespace

struct rbf_problem {
    int device = 0;
    long long n = 0;
    double sigma = 0, cutoff = 0;
    int overlap = 1;
    Grid g{};
    long long ncells = 0;
    size_t bytes = 0;
    size_t budget = 0;                 // 0 = unlimited
    std::vector<DevBuf> bufs;

    // sorted data
    double *xs = nullptr, *ys = nullptr, *fs = nullptr;
    float *xr = nullptr, *yr = nullptr;
    int *perm = nullptr, *cell_of = nullptr, *cell_start = nullptr;
    bool have_values = false;
    double t_init = 0;                 // seconds of the handle's set-up
    double sc32 = 0;                   // FP32 coordinate scale
    long long interactions = -1;
    double* etab = nullptr;            // e^{-n/128}, n < ntab (device), or NULL
    double* t32 = nullptr;             // 2^(j/32), j < 32 (device)
    int ntab = 0;
    float* w32 = nullptr;              // FP32 weights workspace of the FP32 matvec

    // preconditioner: its subdomains are the cells (with `overlap` layers), or
    // after rbf_set_geometry boxes of side B with overlapping squares of side D
    std::vector<int> cs_host;          // cell_start on host
    long long nsub = 0;                // subdomains
    std::vector<int> n_omega, n_c;     // per subdomain
    double xmax = 0, ymax = 0;         // largest coordinates (the box grid's extent)
    bool geo = false;
    rbf::BoxGeometry bg{};
    int* mem = nullptr;                // box members (sorted-order indices), own last
    long long* moff = nullptr;         // per box, offset into mem (nsub + 1)
    int* nown = nullptr;               // per box, own points
    // box truncation of the product (truncation side T > 0 in the geometry):
    // per box the sorted-order indices of the points of its square
    bool boxT = false;
    double halfT = 0;
    int* tsrc = nullptr;
    long long* tsoff = nullptr;
    std::vector<long long> zoff_host;
    long long* zoff = nullptr;
    int np_max = 0, nc_max = 0;
    double* Z64 = nullptr;
    float* Z32 = nullptr;
    double t_pcsetup64 = 0, t_pcsetup32 = 0;
    int shifted_blocks32 = 0;

    // solve workspace
    int ws_m = 0;
    double *V = nullptr, *w = nullptr, *z = nullptr, *r = nullptr, *x = nullptr, *d = nullptr;
    double* rhs = nullptr;
    double *partial = nullptr, *hdev = nullptr;
    int* flag = nullptr;
    double* lam = nullptr;             // last solution, sorted order
    bool solved = false;
    rbf::NeighborLists nl{};           // matvec neighbour lists (nunits == 0: none)
    bool profiling = false;            // event timing of the setup launches
    int setup_lanes = 2;               // batches of the factorisations in flight (1 or 2)
    // Arnoldi step: the Gram-Schmidt part of step j (two classical passes, the
    // norm, the normalisation and the read-back of the H column into pinned
    // host memory) as one captured graph per j (with rbf_set_graphs), built
    // when step j comes round the second time and kept while the workspace
    // stands; events time the step's phases.
    hipStream_t gstream = nullptr;     // capture stream (default priority)
    std::vector<hipGraphExec_t> gs_exec;
    std::vector<int> gs_uses;          // launches of step j's work so far
    bool use_graphs = false;           // rbf_set_graphs
    bool graphs_off = false;           // capture failed once: launch eagerly
    double* hh = nullptr;              // pinned host, 3 * 64 + 1 doubles
    hipEvent_t pev[4] = {};
    bool ktimes_valid[2] = {false, false};
    double kms[2][RBF_K_SETUP_KINDS] = {};
    int kcount[2][RBF_K_SETUP_KINDS] = {};
    std::vector<double> history;
    rbf_solve_info last_info{};        // of the last solve the packed engine ran

    rbf_status alloc(void** out, size_t bytes_) {
        const size_t want = BlockCache::round(bytes_);
        if (budget && this->bytes + want > budget)
            return fail(RBF_ENOMEM, "device memory budget of %zu bytes exceeded (%zu + %zu)",
                        budget, this->bytes, want);
        const size_t limit = budget ? budget - this->bytes : (size_t)-1;
        void* p = nullptr;
        size_t got = 0;
        hipError_t e = BlockCache::get().alloc(device, bytes_, limit, &p, &got);
        if (e != hipSuccess)
            return fail(RBF_ENOMEM, "device allocation of %zu bytes: %s", want,
                        hipGetErrorString(e));
        bufs.push_back({p, got});
        this->bytes += got;
        *out = p;
        return RBF_OK;
    }
    template <typename T>
    rbf_status alloc_n(T** out, long long count) {
        return alloc(reinterpret_cast<void**>(out), sizeof(T) * (size_t)(count > 0 ? count : 1));
    }
    // Gives a buffer back; work enqueued on st before this call may still use it.
    void release(void* q, hipStream_t st) {
        for (size_t i = 0; i < bufs.size(); ++i)
            if (bufs[i].p == q) {
                BlockCache::get().put(device, q, bufs[i].bytes, st, true);
                bytes -= bufs[i].bytes;
                bufs.erase(bufs.begin() + i);
                return;
            }
    }
    // Records the completion of the work a call enqueued on st, so that
    // destruction waits for it and no longer.
    void mark(hipStream_t st) const {
        if (!done && hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) {
            done = nullptr;
            (void)hipStreamSynchronize(st);
            return;
        }
        if (hipEventRecord(done, st) != hipSuccess) (void)hipStreamSynchronize(st);
    }
    mutable hipEvent_t done = nullptr;
    void drop_graphs() {
        for (hipGraphExec_t& e : gs_exec)
            if (e) (void)hipGraphExecDestroy(e);
        gs_exec.clear();
        gs_uses.clear();
    }
    ~rbf_problem() {
        if (done) {
            (void)hipEventSynchronize(done);
            (void)hipEventDestroy(done);
        }
        drop_graphs();
        if (gstream) (void)hipStreamDestroy(gstream);
        if (hh) (void)hipHostFree(hh);
        for (hipEvent_t& e : pev)
            if (e) (void)hipEventDestroy(e);
        for (auto& b : bufs) BlockCache::get().put(device, b.p, b.bytes, nullptr, false);
    }

    rbf::MatvecArgs mv_args() const {
        rbf::MatvecArgs a;
        a.sx = xs;
        a.sy = ys;
        a.scell = cell_start;
        a.tx = xs;
        a.ty = ys;
        a.tcell = cell_start;
        a.g = g;
        a.rc2 = cutoff * cutoff;
        a.mk = -1.0 / (2.0 * sigma * sigma);
        a.beta = (double)(-16.0L / ((long double)sigma * (long double)sigma * kLn2L));
        a.norm = 1.0 / (2.0 * kPi * sigma * sigma);
        a.etab = etab;
        a.ntab = ntab;
        a.t32 = t32;
        return a;
    }
    rbf::Matvec32Args mv32_args() const {
        rbf::Matvec32Args a;
        a.sx = xr;
        a.sy = yr;
        a.scell = cell_start;
        a.g = g;
        a.Ls = (float)(g.L * sc32);
        a.rc2s = (float)(cutoff * cutoff * sc32 * sc32);
        a.norm = 1.0 / (2.0 * kPi * sigma * sigma);
        return a;
    }
    rbf::BoxTrunc bt_args() const {
        rbf::BoxTrunc b;
        b.bg = bg;
        b.halfT = halfT;
        // exp(-d2 / (2 sigma^2)) >= e^-690: the table-driven exponential's range
        b.d2max = 1380.0 * sigma * sigma;
        b.nbox = nsub;
        b.src = tsrc;
        b.soff = tsoff;
        b.mem = mem;
        b.moff = moff;
        b.nown = nown;
        return b;
    }
    rbf::PrecondArgs pc_args() const {
        rbf::PrecondArgs a;
        a.xs = xs;
        a.ys = ys;
        a.cell_start = cell_start;
        a.g = g;
        a.overlap = overlap;
        a.mk = -1.0 / (2.0 * sigma * sigma);
        a.norm = 1.0 / (2.0 * kPi * sigma * sigma);
        a.zoff = zoff;
        a.np_max = np_max;
        a.nc_max = nc_max;
        a.ncells = nsub;
        a.xy = nullptr;
        a.mem = geo ? mem : nullptr;
        a.moff = geo ? moff : nullptr;
        a.nown = geo ? nown : nullptr;
        return a;
    }
};

namespace rbf {
rbf_status set_error(rbf_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

void set_setup_lanes(rbf_problem* p, int lanes) {
    if (p) p->setup_lanes = lanes > 1 ? 2 : 1;
}

hipError_t cached_alloc(int dev, size_t bytes, void** out, size_t* got) {
    return BlockCache::get().alloc(dev, bytes, (size_t)-1, out, got);
}
void cached_free(int dev, void* p, size_t bytes, hipStream_t st) {
    BlockCache::get().put(dev, p, bytes, st, true);
}
}  // namespace rbf

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Marks, when a call returns (also on errors), the end of the work it
// enqueued on its stream.
struct MarkOnExit {
    const rbf_problem* p;
    hipStream_t st;
    ~MarkOnExit() {
        if (p) p->mark(st);
    }
};

bool finite(double v) { return std::isfinite(v); }

rbf_status check_args(long long n, double sigma, double cutoff, int overlap) {
    if (n < 1) return fail(RBF_EINVAL, "n must be >= 1 (got %lld)", n);
    if (n > 2000000000LL) return fail(RBF_ELIMIT, "n = %lld exceeds 2e9", n);
    if (!(sigma > 0) || !finite(sigma)) return fail(RBF_EINVAL, "sigma must be finite and > 0");
    if (!(cutoff > 0) || !finite(cutoff)) return fail(RBF_EINVAL, "cutoff must be finite and > 0");
    if (overlap < 0) return fail(RBF_EINVAL, "overlap must be >= 0");
    if (overlap > 16) return fail(RBF_ELIMIT, "overlap must be <= 16");
    return RBF_OK;
}

// The setup pipeline on device arrays d_pts (n x 2) and d_vals (n or NULL).
// Neighbour lists of the matvec (skipped when some 3x3 block of cells holds
// more sources than a list-driven launch can stage; the candidate kernels then
// serve every matvec).  Groups run along cell rows: a group takes consecutive
// cells of one row while it spans at most kGroupCells columns, stages at most
// kGroupSpan sources and holds at most kGroupMaxUnits units of 64 targets; a
// cell with more targets than that is split over several groups.
rbf_status build_lists(rbf_problem* p, hipStream_t st) {
    const rbf::Grid& g = p->g;
    const int* cs = p->cs_host.data();
    const int ncx = g.ncx, ncy = g.ncy;
    auto span = [&](int cy, int cxa, int cxb) {
        const int xlo = std::max(cxa - 1, 0), xhi = std::min(cxb + 1, ncx - 1);
        long long s = 0;
        for (int ny = std::max(cy - 1, 0); ny <= std::min(cy + 1, ncy - 1); ++ny)
            s += cs[(long long)ny * ncx + xhi + 1] - cs[(long long)ny * ncx + xlo];
        return s;
    };
    const int max_targets = 64 * rbf::kGroupMaxUnits;
    std::vector<rbf::ListGroup> groups;
    int nu = 0, max_nb = 0, gmax = 0;
    auto emit = [&](int cy, int cxa, int cxb, int t0, int t1) {
        rbf::ListGroup gr{};
        gr.u0 = nu;
        gr.nu = (t1 - t0 + 63) / 64;
        gr.cy = cy;
        gr.cxa = cxa;
        gr.cxb = cxb;
        gr.t0 = t0;
        gr.t1 = t1;
        groups.push_back(gr);
        nu += gr.nu;
        gmax = std::max(gmax, gr.nu);
        max_nb = std::max(max_nb, (int)span(cy, cxa, cxb));
    };
    for (int cy = 0; cy < ncy; ++cy) {
        const int* row = cs + (long long)cy * ncx;
        int cx = 0;
        while (cx < ncx) {
            if (row[cx + 1] == row[cx]) {   // no targets: starts no group
                ++cx;
                continue;
            }
            if (span(cy, cx, cx) > rbf::kListMaxNb) return RBF_OK;
            int cxb = cx;
            while (cxb + 1 < ncx && cxb + 2 - cx <= rbf::kGroupCells &&
                   span(cy, cx, cxb + 1) <= rbf::kGroupSpan &&
                   row[cxb + 2] - row[cx] <= max_targets)
                ++cxb;
            if (row[cxb + 1] - row[cx] <= max_targets) {
                emit(cy, cx, cxb, row[cx], row[cxb + 1]);
            } else {   // one cell with more targets than a group holds
                for (int t = row[cx]; t < row[cx + 1]; t += max_targets)
                    emit(cy, cx, cx, t, std::min(t + max_targets, row[cx + 1]));
            }
            cx = cxb + 1;
        }
    }
    if (nu == 0) return RBF_OK;
    rbf::ListGroup* group = nullptr;
    int* len = nullptr;
    long long* off = nullptr;
    unsigned short* idx = nullptr;
    RBF_TRY(p->alloc_n(&group, groups.size()));
    RBF_TRY(p->alloc_n(&len, nu));
    RBF_TRY(p->alloc_n(&off, nu + 1));
    HIP_TRY(hipMemcpyAsync(group, groups.data(), sizeof(rbf::ListGroup) * groups.size(),
                           hipMemcpyHostToDevice, st));
    rbf::NeighborLists nl{};
    nl.group = group;
    nl.off = off;
    nl.len = len;
    nl.nunits = nu;
    nl.ngroups = (int)groups.size();
    nl.gunits = gmax;
    nl.max_nb = max_nb;
    const rbf::MatvecArgs a = p->mv_args();
    HIP_TRY(rbf::launch_list_count(a, nl, len, st));
    std::vector<int> hl(nu);
    HIP_TRY(hipMemcpyAsync(hl.data(), len, sizeof(int) * nu, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<long long> ho(nu + 1);
    ho[0] = 0;
    for (int u = 0; u < nu; ++u) ho[u + 1] = ho[u] + 64LL * hl[u];
    RBF_TRY(p->alloc_n(&idx, ho[nu]));
    HIP_TRY(hipMemcpyAsync(off, ho.data(), sizeof(long long) * (nu + 1), hipMemcpyHostToDevice, st));
    HIP_TRY(rbf::launch_list_fill(a, nl, idx, st));
    HIP_TRY(hipStreamSynchronize(st));
    nl.idx = idx;
    p->nl = nl;
    return RBF_OK;
}

rbf_status setup_impl(rbf_problem* p, const double* d_pts, const double* d_vals, hipStream_t st) {
    const long long n = p->n;
    double* work;
    double* mm;
    int* bad;
    RBF_TRY(p->alloc_n(&work, 4 * rbf::kReduceBlocks + 4));
    mm = work + 4 * rbf::kReduceBlocks;
    RBF_TRY(p->alloc_n(&bad, 4));
    HIP_TRY(hipMemsetAsync(bad, 0, 4 * sizeof(int), st));
    HIP_TRY(rbf::launch_minmax(d_pts, d_vals, n, work, mm, bad, st));
    double h_mm[4];
    int h_bad = 0;
    HIP_TRY(hipMemcpyAsync(h_mm, mm, sizeof h_mm, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&h_bad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h_bad) return fail(RBF_EINVAL, "points or values contain NaN or Inf");
    Grid& g = p->g;
    g.x0 = h_mm[0];
    g.y0 = h_mm[1];
    p->xmax = h_mm[2];
    p->ymax = h_mm[3];
    g.L = p->cutoff;
    g.invL = 1.0 / p->cutoff;
    double fx = std::floor((h_mm[2] - h_mm[0]) * g.invL);
    double fy = std::floor((h_mm[3] - h_mm[1]) * g.invL);
    if (!(fx < 1e9) || !(fy < 1e9) || (fx + 1) * (fy + 1) > 1e9)
        return fail(RBF_EINVAL, "cell grid too large: %.0f x %.0f cells (cutoff too small)",
                    fx + 1, fy + 1);
    g.ncx = (int)fx + 1;
    g.ncy = (int)fy + 1;
    p->ncells = g.ncells();
    const long long nc = p->ncells;

    int *counts, *slot, *tmp, *scan_work;
    RBF_TRY(p->alloc_n(&p->cell_of, n));
    RBF_TRY(p->alloc_n(&p->perm, n));
    RBF_TRY(p->alloc_n(&p->cell_start, nc + 1));
    RBF_TRY(p->alloc_n(&counts, nc));
    RBF_TRY(p->alloc_n(&slot, n));
    RBF_TRY(p->alloc_n(&tmp, n));
    RBF_TRY(p->alloc_n(&scan_work, rbf::scan_work_ints(nc)));
    HIP_TRY(hipMemsetAsync(counts, 0, sizeof(int) * nc, st));
    HIP_TRY(rbf::launch_cell_count(d_pts, n, g, p->cell_of, slot, counts, st));
    HIP_TRY(rbf::launch_exclusive_scan(counts, p->cell_start, nc, scan_work, st));
    HIP_TRY(rbf::launch_scatter(p->cell_of, slot, p->cell_start, n, tmp, st));
    HIP_TRY(rbf::launch_sort_cells(tmp, p->cell_start, nc, p->perm, RBF_MAX_CELL_POINTS, bad + 1,
                                   st));
    RBF_TRY(p->alloc_n(&p->xs, n));
    RBF_TRY(p->alloc_n(&p->ys, n));
    RBF_TRY(p->alloc_n(&p->fs, n));
    RBF_TRY(p->alloc_n(&p->xr, n));
    RBF_TRY(p->alloc_n(&p->yr, n));
    // FP32 coordinates: scaled so that |dx_s|^2 = |dx|^2 log2(e) / (2 sigma^2)
    p->sc32 = std::sqrt(1.4426950408889634 / 2.0) / p->sigma;
    HIP_TRY(rbf::launch_gather(d_pts, d_vals, p->perm, p->cell_of, n, g, p->sc32, p->xs, p->ys,
                               p->fs, p->xr, p->yr, st));
    HIP_TRY(rbf::launch_dup_check(p->xs, p->ys, p->cell_start, nc, bad + 2, st));
    int h_flags[4];
    HIP_TRY(hipMemcpyAsync(h_flags, bad, sizeof h_flags, hipMemcpyDeviceToHost, st));
    p->cs_host.resize(nc + 1);
    HIP_TRY(hipMemcpyAsync(p->cs_host.data(), p->cell_start, sizeof(int) * (nc + 1),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h_flags[1])
        return fail(RBF_ELIMIT, "%d cells hold more than %d points", h_flags[1],
                    RBF_MAX_CELL_POINTS);
    if (h_flags[2]) return fail(RBF_EDUPLICATE, "two points are bit-identical");
    p->have_values = d_vals != nullptr;
    p->release(counts, st);
    p->release(slot, st);
    p->release(tmp, st);
    p->release(scan_work, st);
    p->release(work, st);
    // keep `bad` as a flag word for later use
    p->flag = bad;

    // per-cell block sizes (host): members of the (2*ov+1)^2 block, own points
    const int ov = p->overlap;
    p->nsub = nc;
    p->n_omega.assign(nc, 0);
    p->n_c.assign(nc, 0);
    int maxo = 0;
    for (long long c = 0; c < nc; ++c) {
        int cx = (int)(c % g.ncx), cy = (int)(c / g.ncx);
        int xlo = std::max(cx - ov, 0), xhi = std::min(cx + ov, g.ncx - 1);
        long long tot = 0;
        for (int dy = -ov; dy <= ov; ++dy) {
            int ny = cy + dy;
            if (ny < 0 || ny >= g.ncy) continue;
            tot += p->cs_host[(long long)ny * g.ncx + xhi + 1] - p->cs_host[(long long)ny * g.ncx + xlo];
        }
        int own = p->cs_host[c + 1] - p->cs_host[c];
        p->n_c[c] = own;
        p->n_omega[c] = (int)std::min<long long>(tot, 1 << 30);
        if (own > 0) maxo = std::max(maxo, p->n_omega[c]);
        p->nc_max = std::max(p->nc_max, own);
    }
    p->np_max = (maxo + 63) / 64 * 64;   // the factorisation advances 64 columns at a time

    // table e^{-n/128} covering the matvec's exponents down to -cutoff^2/(2 sigma^2)
    const double xmin = p->cutoff * p->cutoff / (2.0 * p->sigma * p->sigma);
    const double nt = std::floor(128.0 * xmin * (1.0 + 1e-12)) + 2.0;
    if (nt <= rbf::kExpTableMax) {
        p->ntab = (int)nt;
        std::vector<double> tab(p->ntab);
        for (int k = 0; k < p->ntab; ++k) tab[k] = (double)std::exp(-(long double)k / 128.0L);
        RBF_TRY(p->alloc_n(&p->etab, p->ntab));
        HIP_TRY(hipMemcpyAsync(p->etab, tab.data(), sizeof(double) * p->ntab, hipMemcpyHostToDevice,
                               st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    {
        double tab[32];
        for (int j = 0; j < 32; ++j) tab[j] = (double)std::exp2((long double)j / 32.0L);
        RBF_TRY(p->alloc_n(&p->t32, 32));
        HIP_TRY(hipMemcpyAsync(p->t32, tab, sizeof tab, hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    RBF_TRY(p->alloc_n(&p->w32, n));
    return build_lists(p, st);
}

rbf_status create(const double* pts, const double* vals, bool on_device, long long n,
                  double sigma, double cutoff, int overlap, hipStream_t st, rbf_problem** out) {
    if (!out) return fail(RBF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!pts) return fail(RBF_EINVAL, "points is NULL");
    RBF_TRY(check_args(n, sigma, cutoff, overlap));
    rbf_problem* p = new (std::nothrow) rbf_problem();
    if (!p) return fail(RBF_ENOMEM, "host allocation failed");
    HIP_TRY(hipGetDevice(&p->device));
    p->n = n;
    p->sigma = sigma;
    p->cutoff = cutoff;
    p->overlap = overlap;
    rbf_status s;
    Timer t_init;
    if (on_device) {
        s = setup_impl(p, pts, vals, st);
    } else {
        double *dp = nullptr, *dv = nullptr;
        s = p->alloc_n(&dp, 2 * n);
        if (s == RBF_OK && vals) s = p->alloc_n(&dv, n);
        if (s == RBF_OK) {
            hipError_t e = hipMemcpyAsync(dp, pts, sizeof(double) * 2 * n, hipMemcpyHostToDevice, st);
            if (e == hipSuccess && vals)
                e = hipMemcpyAsync(dv, vals, sizeof(double) * n, hipMemcpyHostToDevice, st);
            if (e != hipSuccess) s = fail(RBF_EDEVICE, "copy to device: %s", hipGetErrorString(e));
        }
        if (s == RBF_OK) s = setup_impl(p, dp, dv, st);
        if (dp) p->release(dp, st);
        if (dv) p->release(dv, st);
    }
    if (s != RBF_OK) {
        p->mark(st);
        delete p;
        return s;
    }
    p->mark(st);
    p->t_init = t_init.sec();   // setup_impl ends with a wait for its stream
    *out = p;
    return RBF_OK;
}

template <typename T>
rbf_status precond_setup_impl(rbf_problem* p, hipStream_t st) {
    const bool is64 = sizeof(T) == 8;
    if (is64 ? p->Z64 != nullptr : p->Z32 != nullptr) return RBF_OK;
    Timer tm;
    const long long nc = p->nsub;
    if (p->np_max > RBF_MAX_BLOCK)
        return fail(RBF_ELIMIT, "a local block has %d points, above the limit %d", p->np_max,
                    RBF_MAX_BLOCK);
    if (p->zoff_host.empty()) {
        p->zoff_host.resize(nc);
        long long tot = 0;
        for (long long c = 0; c < nc; ++c) {
            p->zoff_host[c] = tot;
            tot += (long long)p->n_c[c] * p->n_omega[c];
        }
        p->zoff_host.push_back(tot);
        RBF_TRY(p->alloc_n(&p->zoff, nc + 1));
        HIP_TRY(hipMemcpyAsync(p->zoff, p->zoff_host.data(), sizeof(long long) * (nc + 1),
                               hipMemcpyHostToDevice, st));
    }
    const long long ztot = p->zoff_host[nc];
    T* Z;
    RBF_TRY(p->alloc_n(&Z, ztot));
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    const long long slot_elems = rbf::slot_elems64(p->np_max);
    // cells per batch: one scratch matrix per cell of a batch that the
    // lockstep launches advance together
    long long nslots = std::min<long long>(nc, 8192);
    const long long max_scratch = 12LL << 30;
    while (nslots > cus && nslots * slot_elems * (long long)sizeof(T) > max_scratch) nslots /= 2;
    if (nslots > 8) nslots &= ~7LL;
    if (nslots < 1) nslots = 1;
    const long long pad = (nslots + 7) / 8 * 8;
    // Two lanes (two batches in flight on two streams) when there are two
    // batches or more and their buffers fit; one when profiling, so that the
    // per-kernel event times are those of kernels that run alone.
    const long long nbatch = (nc + nslots - 1) / nslots;
    int nlanes = (nbatch >= 2 && !p->profiling && p->setup_lanes > 1) ? 2 : 1;
    rbf::SetupLane<T> lane[2] = {};
    int* status = nullptr;
    hipStream_t st2 = nullptr;
    auto alloc_lane = [&](rbf::SetupLane<T>& L) -> rbf_status {
        RBF_TRY(p->alloc_n(&L.scratch, nslots * slot_elems));
        RBF_TRY(p->alloc_n(&L.xy, pad * p->np_max));
        RBF_TRY(p->alloc_n(&L.meta, pad));
        RBF_TRY(p->alloc_n(&L.lvl, pad));
        RBF_TRY(p->alloc_n(&L.lt, 2 * pad * 2048));
        return RBF_OK;
    };
    auto release_lane = [&](rbf::SetupLane<T>& L) {
        if (L.scratch) p->release(L.scratch, st);
        if (L.xy) p->release(L.xy, st);
        if (L.meta) p->release(L.meta, st);
        if (L.lvl) p->release(L.lvl, st);
        if (L.lt) p->release(L.lt, st);
        L = rbf::SetupLane<T>{};
    };
    auto release_all = [&]() {
        release_lane(lane[0]);
        release_lane(lane[1]);
        if (status) p->release(status, st);
    };
    rbf_status s = p->alloc_n(&status, nc);
    if (s == RBF_OK) s = alloc_lane(lane[0]);
    if (s != RBF_OK) {
        p->release(Z, st);
        release_all();
        return s;
    }
    lane[0].st = st;
    if (nlanes == 2) {
        // the second lane is optional: without memory or a stream, one lane
        if (alloc_lane(lane[1]) != RBF_OK ||
            hipStreamCreateWithFlags(&st2, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            release_lane(lane[1]);
            st2 = nullptr;
            nlanes = 1;
        }
        lane[1].st = st2;
    }
    rbf::PrecondArgs a = p->pc_args();
    rbf::SetupProfile prof;
    rbf::SetupProfile* pp = p->profiling ? &prof : nullptr;
    hipError_t e;
    if (is64)
        e = rbf::launch_precond_setup64(a, reinterpret_cast<double*>(Z), (int)nslots,
                                        reinterpret_cast<const rbf::SetupLane<double>*>(lane),
                                        nlanes, status, st, pp);
    else
        e = rbf::launch_precond_setup32(a, reinterpret_cast<float*>(Z), (int)nslots,
                                        reinterpret_cast<const rbf::SetupLane<float>*>(lane),
                                        nlanes, status, st, pp);
    std::vector<int> hs(nc);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hs.data(), status, sizeof(int) * nc, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (pp) {
        const int pi = is64 ? 0 : 1;
        for (int k = 0; k < RBF_K_SETUP_KINDS; ++k) {
            p->kms[pi][k] = 0.0;
            p->kcount[pi][k] = 0;
        }
        for (auto& r : prof.recs) {
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
            p->kms[pi][r.kind] += ms;
            p->kcount[pi][r.kind] += 1;
            (void)hipEventDestroy(r.start);
            (void)hipEventDestroy(r.stop);
        }
        p->ktimes_valid[pi] = e == hipSuccess;
    }
    if (st2) {   // normally already joined into st; after an error perhaps not
        (void)hipStreamSynchronize(st2);
        (void)hipGetLastError();
    }
    release_all();
    if (st2) (void)hipStreamDestroy(st2);
    if (e != hipSuccess) {
        p->release(Z, st);
        return fail(RBF_EDEVICE, "preconditioner setup: %s", hipGetErrorString(e));
    }
    int bad = 0, shifted = 0;
    long long first_bad = -1;
    for (long long c = 0; c < nc; ++c) {
        if (hs[c] > 0) {
            if (first_bad < 0) first_bad = c;
            ++bad;
        } else if (hs[c] < 0) {
            ++shifted;
        }
    }
    if (bad) {
        p->release(Z, st);
        return fail(RBF_ENOTPD, "%d local blocks are not positive definite (first: cell %lld, pivot %d)",
                    bad, first_bad, hs[first_bad]);
    }
    if (is64) {
        p->Z64 = reinterpret_cast<double*>(Z);
        p->t_pcsetup64 = tm.sec();
    } else {
        p->Z32 = reinterpret_cast<float*>(Z);
        p->t_pcsetup32 = tm.sec();
        p->shifted_blocks32 = shifted;
    }
    return RBF_OK;
}

// the FP32 local factors serve both the mixed form and the FP64 method with
// FP32 local inverses
rbf_status precond_setup(rbf_problem* p, rbf_precision prec, hipStream_t st) {
    if (prec == RBF_FP64) return precond_setup_impl<double>(p, st);
    if (prec == RBF_MIXED || prec == RBF_FP64_PC32) return precond_setup_impl<float>(p, st);
    return fail(RBF_EINVAL, "unknown precision %d", (int)prec);
}

// the matvec's precision under a solve's precision: FP32 only in the mixed form
inline rbf_precision operator_precision(rbf_precision prec) {
    return prec == RBF_MIXED ? RBF_MIXED : RBF_FP64;
}

rbf_status matvec(rbf_problem* p, rbf_precision prec, const double* w, double* y, hipStream_t st) {
    const bool lists = p->nl.nunits > 0;
    prec = operator_precision(prec);
    if (p->boxT) {
        if (prec != RBF_FP64)
            return fail(RBF_EINVAL, "the box-truncated product runs in FP64 only");
        HIP_TRY(rbf::launch_matvec64_box(p->mv_args(), p->bt_args(), w, y, st));
        return RBF_OK;
    }
    if (prec == RBF_FP64) {
        if (lists)
            HIP_TRY(rbf::launch_matvec64_lists(p->mv_args(), p->nl, w, y, st));
        else
            HIP_TRY(rbf::launch_matvec64(p->mv_args(), w, y, nullptr, st));
    } else {
        if (lists)
            HIP_TRY(rbf::launch_matvec32_lists(p->mv32_args(), p->nl, w, y, st));
        else
            HIP_TRY(rbf::launch_matvec32(p->mv32_args(), w, p->w32, y, p->n, st));
    }
    return RBF_OK;
}

rbf_status rasm(rbf_problem* p, rbf_precision prec, const double* v, double* z, hipStream_t st) {
    RBF_TRY(precond_setup(p, prec, st));
    if (prec == RBF_FP64) {
        HIP_TRY(rbf::launch_rasm_apply64(p->pc_args(), p->Z64, v, z, st));
    } else if (prec == RBF_MIXED) {
        HIP_TRY(rbf::launch_rasm_apply32(p->pc_args(), p->Z32, v, z, st));
    } else {
        HIP_TRY(rbf::launch_rasm_apply32x64(p->pc_args(), p->Z32, v, z, st));
    }
    return RBF_OK;
}

rbf_status ensure_workspace(rbf_problem* p, int m, hipStream_t st) {
    if (!p->hh) {
        if (hipHostMalloc(reinterpret_cast<void**>(&p->hh), sizeof(double) * (3 * 64 + 1)) !=
            hipSuccess) {
            p->hh = nullptr;
            return fail(RBF_ENOMEM, "pinned host buffer of the Arnoldi step");
        }
        for (hipEvent_t& e : p->pev) HIP_TRY(hipEventCreate(&e));
    }
    if (p->ws_m >= m) return RBF_OK;
    p->drop_graphs();   // they refer to the old basis
    if (p->V) {
        p->release(p->V, st);
        p->V = nullptr;
    }
    const long long n = p->n;
    RBF_TRY(p->alloc_n(&p->V, (long long)(m + 1) * n));
    if (!p->w) {
        RBF_TRY(p->alloc_n(&p->w, n));
        RBF_TRY(p->alloc_n(&p->z, n));
        RBF_TRY(p->alloc_n(&p->r, n));
        RBF_TRY(p->alloc_n(&p->x, n));
        RBF_TRY(p->alloc_n(&p->d, n));
        RBF_TRY(p->alloc_n(&p->rhs, n));
        RBF_TRY(p->alloc_n(&p->partial, 64LL * rbf::kDotBlocks));
        RBF_TRY(p->alloc_n(&p->hdev, 4 * 64));
    }
    p->ws_m = m;
    return RBF_OK;
}

struct PhaseTimes {
    double matmult = 0, matsolve = 0, vecmdot = 0, other = 0;
    int mv64 = 0, mv32 = 0, pc = 0;
};

// ||v||^2 on device -> host
rbf_status norm2(rbf_problem* p, const double* v, double* out_host, hipStream_t st) {
    HIP_TRY(rbf::launch_multidot(v, 0, 1, v, p->n, p->partial, p->hdev + 192, st));
    HIP_TRY(hipMemcpyAsync(out_host, p->hdev + 192, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return RBF_OK;
}

// One or more GMRES(m) cycles, right-preconditioned, on A x = b with x on
// device (updated in place).  prec selects the operator and preconditioner
// arithmetic.  Returns when the residual estimate is <= tol_abs, after
// max_cycles cycles, or after the iteration budget.  Each cycle starts from the
// residual b - A x with the same operator (r0, if given, is that residual for
// the first cycle).
struct CycleResult {
    int iters = 0, cycles = 0;
    double est = 0;             // last residual estimate (absolute)
    bool breakdown = false;
};

// Step j of the Arnoldi process after the product w = A M^-1 v_j: classical
// Gram-Schmidt applied twice (h1, h2), ||w||^2, v_{j+1} = w / ||w||, and the
// device H column (h1, h2, ||w||^2) copied into p->hh.
hipError_t enqueue_gram_schmidt(rbf_problem* p, int j, hipStream_t st) {
    const long long n = p->n;
    double* V = p->V;
    double* h1 = p->hdev;
    double* h2 = p->hdev + 64;
    double* hn2 = p->hdev + 128;
    hipError_t e;
    if ((e = rbf::launch_multidot(V, n, j + 1, p->w, n, p->partial, h1, st)) != hipSuccess) return e;
    if ((e = rbf::launch_multi_axpy(V, n, j + 1, h1, p->w, n, -1.0, st)) != hipSuccess) return e;
    if ((e = rbf::launch_multidot(V, n, j + 1, p->w, n, p->partial, h2, st)) != hipSuccess) return e;
    if ((e = rbf::launch_multi_axpy(V, n, j + 1, h2, p->w, n, -1.0, st)) != hipSuccess) return e;
    if ((e = rbf::launch_multidot(p->w, 0, 1, p->w, n, p->partial, hn2, st)) != hipSuccess) return e;
    if ((e = rbf::launch_scale_by_inv(p->w, hn2, V + (long long)(j + 1) * n, n, st)) != hipSuccess)
        return e;
    return hipMemcpyAsync(p->hh, p->hdev, sizeof(double) * (2 * 64 + 1), hipMemcpyDeviceToHost, st);
}

// The same work as one graph launch, captured on the problem's own stream when
// step j comes round the second time (a restart, the next outer step of the
// mixed form, the next solve on the handle), so that a capture is only paid
// for where it is replayed; falls back to single launches if capture fails.
rbf_status gram_schmidt(rbf_problem* p, int j, hipStream_t st) {
    if ((int)p->gs_exec.size() <= j) {
        p->gs_exec.resize(j + 1, nullptr);
        p->gs_uses.resize(j + 1, 0);
    }
    if (p->use_graphs && !p->graphs_off && p->gs_uses[j]++ > 0) {
        if (!p->gs_exec[j]) {
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            bool ok = p->gstream || hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking) == hipSuccess;
            if (ok) ok = hipStreamBeginCapture(p->gstream, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                const hipError_t le = enqueue_gram_schmidt(p, j, p->gstream);
                const hipError_t ce = hipStreamEndCapture(p->gstream, &graph);
                ok = le == hipSuccess && ce == hipSuccess && graph != nullptr;
            }
            if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            if (ok) {
                p->gs_exec[j] = exec;
            } else {
                if (exec) (void)hipGraphExecDestroy(exec);
                p->graphs_off = true;
            }
        }
        if (!p->graphs_off) {
            HIP_TRY(hipGraphLaunch(p->gs_exec[j], st));
            return RBF_OK;
        }
    }
    HIP_TRY(enqueue_gram_schmidt(p, j, st));
    return RBF_OK;
}

float event_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    return hipEventElapsedTime(&ms, a, b) == hipSuccess ? ms : 0.f;
}

rbf_status gmres_cycles(rbf_problem* p, rbf_precision prec, const double* b, double* x, int m,
                        double tol_abs, int max_cycles, int iter_budget, hipStream_t st,
                        CycleResult* res, PhaseTimes* pt, const double* r0) {
    const long long n = p->n;
    double* V = p->V;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gv(m + 1), yv(m);
    for (int cyc = 0; cyc < max_cycles && res->iters < iter_budget; ++cyc) {
        // r = b - A x  into V_0
        bool timed = false;
        if (r0 && cyc == 0) {   // residual of the starting x already known
            HIP_TRY(hipMemcpyAsync(V, r0, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        } else {
            HIP_TRY(hipEventRecord(p->pev[0], st));
            RBF_TRY(matvec(p, prec, x, p->w, st));
            HIP_TRY(hipEventRecord(p->pev[1], st));
            timed = true;
            HIP_TRY(rbf::launch_sub(b, p->w, V, n, st));
            (operator_precision(prec) == RBF_FP64 ? pt->mv64 : pt->mv32) += 1;
        }
        double beta2;
        RBF_TRY(norm2(p, V, &beta2, st));   // waits for the stream
        if (timed) pt->matmult += 1e-3 * event_ms(p->pev[0], p->pev[1]);
        double beta = std::sqrt(beta2);
        if (!std::isfinite(beta)) return fail(RBF_ENAN, "non-finite residual");
        res->est = beta;
        if (beta <= tol_abs || beta == 0.0) return RBF_OK;
        HIP_TRY(rbf::launch_scale_by_inv(V, p->hdev + 192, V, n, st));
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = beta;
        int k = 0;
        bool stop = false;
        for (int j = 0; j < m && !stop; ++j) {
            double* vj = V + (long long)j * n;
            // the step's launches are enqueued back to back; the one wait is
            // for the H column, and events time the phases
            HIP_TRY(hipEventRecord(p->pev[0], st));
            RBF_TRY(rasm(p, prec, vj, p->z, st));
            HIP_TRY(hipEventRecord(p->pev[1], st));
            pt->pc += 1;
            RBF_TRY(matvec(p, prec, p->z, p->w, st));
            HIP_TRY(hipEventRecord(p->pev[2], st));
            (operator_precision(prec) == RBF_FP64 ? pt->mv64 : pt->mv32) += 1;
            RBF_TRY(gram_schmidt(p, j, st));
            HIP_TRY(hipEventRecord(p->pev[3], st));
            HIP_TRY(hipEventSynchronize(p->pev[3]));
            pt->matsolve += 1e-3 * event_ms(p->pev[0], p->pev[1]);
            pt->matmult += 1e-3 * event_ms(p->pev[1], p->pev[2]);
            pt->vecmdot += 1e-3 * event_ms(p->pev[2], p->pev[3]);
            const double* hh = p->hh;
            Timer t4;
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hh[i] + hh[64 + i];
            double hn = std::sqrt(hh[128]);
            H[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
            double rho = std::hypot(a, bb);
            if (!std::isfinite(rho)) return fail(RBF_ENAN, "non-finite Hessenberg entry");
            cs[j] = rho > 0 ? a / rho : 1.0;
            sn[j] = rho > 0 ? bb / rho : 0.0;
            H[(size_t)j * m + j] = rho;
            H[(size_t)(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            ++res->iters;
            k = j + 1;
            res->est = std::fabs(gv[j + 1]);
            if (hn == 0.0) {
                res->breakdown = true;
                stop = true;
            }
            if (res->est <= tol_abs || res->iters >= iter_budget) stop = true;
            pt->other += t4.sec();
        }
        // y = H^{-1} g, u = V y, x += M^{-1} u
        Timer t5;
        for (int i = k - 1; i >= 0; --i) {
            double s = gv[i];
            for (int jj = i + 1; jj < k; ++jj) s -= H[(size_t)i * m + jj] * yv[jj];
            yv[i] = s / H[(size_t)i * m + i];
        }
        HIP_TRY(hipMemcpyAsync(p->hdev, yv.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
        HIP_TRY(rbf::launch_fill(p->w, 0.0, n, st));
        HIP_TRY(rbf::launch_multi_axpy(V, n, k, p->hdev, p->w, n, 1.0, st));
        pt->vecmdot += t5.sec();
        Timer t6;
        RBF_TRY(rasm(p, prec, p->w, p->z, st));
        pt->pc += 1;
        HIP_TRY(rbf::launch_axpy(1.0, p->z, x, n, st));
        HIP_TRY(hipStreamSynchronize(st));
        pt->matsolve += t6.sec();
        ++res->cycles;
        if (res->est <= tol_abs || res->breakdown) return RBF_OK;
    }
    return RBF_OK;
}

rbf_status count_interactions(rbf_problem* p, int* d_nnb_sorted, hipStream_t st);

// The stagnation stop of the FP64 solves: the cycle-start true residuals in
// history (the last one the current), k > 0 cycles back.
bool stalled(const std::vector<double>& history, int k) {
    const size_t n = history.size();
    return k > 0 && n > (size_t)k && history[n - 1] > 0.5 * history[n - 1 - (size_t)k];
}

rbf_status true_rel_residual(rbf_problem* p, const double* b, const double* x, double bnorm,
                             double* rel, hipStream_t st, PhaseTimes* pt) {
    HIP_TRY(hipEventRecord(p->pev[0], st));
    RBF_TRY(matvec(p, RBF_FP64, x, p->w, st));
    HIP_TRY(hipEventRecord(p->pev[1], st));
    pt->mv64 += 1;
    HIP_TRY(rbf::launch_sub(b, p->w, p->r, p->n, st));
    double r2;
    RBF_TRY(norm2(p, p->r, &r2, st));   // waits for the stream
    *rel = std::sqrt(r2) / bnorm;
    pt->matmult += 1e-3 * event_ms(p->pev[0], p->pev[1]);
    return RBF_OK;
}

rbf_status solve_impl(rbf_problem* p, const rbf_solve_opts* o, const double* d_lambda0,
                      bool lambda0_on_device, const double* h_lambda0, rbf_solve_info* info) {
    rbf_solve_opts opts;
    rbf_default_opts(&opts);
    if (o) opts = *o;
    hipStream_t st = as_stream(opts.stream);
    if (opts.restart < 1 || opts.restart > 63) return fail(RBF_EINVAL, "restart must be in [1, 63]");
    if (!(opts.rtol >= 0)) return fail(RBF_EINVAL, "rtol must be >= 0");
    if (opts.max_iters < 0) return fail(RBF_EINVAL, "max_iters must be >= 0");
    if (opts.stall_cycles < 0) return fail(RBF_EINVAL, "stall_cycles must be >= 0");
    if (opts.precision != RBF_FP64 && opts.precision != RBF_MIXED &&
        opts.precision != RBF_FP64_PC32)
        return fail(RBF_EINVAL, "unknown precision");
    if (p->boxT && opts.precision == RBF_MIXED)
        return fail(RBF_EINVAL, "the box-truncated product runs in FP64 only: solve with "
                                "RBF_FP64 or RBF_FP64_PC32");
    if (!p->have_values) return fail(RBF_ESTATE, "no right-hand side: pass values or call rbf_set_values");
    p->budget = opts.max_device_bytes;
    if (p->budget && p->bytes > p->budget)
        return fail(RBF_ENOMEM, "the problem already holds %zu device bytes, above the budget %zu",
                    p->bytes, p->budget);
    Timer total;
    PhaseTimes pt;
    double t_pc = 0;
    {
        Timer t;
        RBF_TRY(precond_setup(p, opts.precision, st));
        HIP_TRY(hipStreamSynchronize(st));
        t_pc = t.sec();
    }
    const int m = opts.restart;
    RBF_TRY(ensure_workspace(p, m, st));

    const long long n = p->n;
    // initial guess (sorted order)
    if (d_lambda0 || h_lambda0) {
        if (lambda0_on_device) {
            HIP_TRY(rbf::launch_permute(d_lambda0, p->perm, n, p->x, st));
        } else {
            HIP_TRY(hipMemcpyAsync(p->r, h_lambda0, sizeof(double) * n, hipMemcpyHostToDevice, st));
            HIP_TRY(rbf::launch_permute(p->r, p->perm, n, p->x, st));
        }
    } else {
        HIP_TRY(rbf::launch_fill(p->x, 0.0, n, st));
    }
    double bnorm2;
    RBF_TRY(norm2(p, p->fs, &bnorm2, st));
    const double bnorm = std::sqrt(bnorm2);
    p->history.clear();
    rbf_status status = RBF_OK;
    double rel = 0;
    int iters = 0, cycles = 0, outer = 0;
    if (bnorm == 0.0) {
        HIP_TRY(rbf::launch_fill(p->x, 0.0, n, st));
        rel = 0;
    } else if (opts.precision != RBF_MIXED) {   // FP64, with FP64 or FP32 local inverses
        for (;;) {
            RBF_TRY(true_rel_residual(p, p->fs, p->x, bnorm, &rel, st, &pt));
            p->history.push_back(rel);
            if (!std::isfinite(rel)) {
                status = fail(RBF_ENAN, "non-finite residual");
                break;
            }
            if (rel <= opts.rtol) break;
            if (iters >= opts.max_iters) {
                status = fail(RBF_ENOCONV, "no convergence in %d iterations (rel. residual %.3e)",
                              iters, rel);
                break;
            }
            if (stalled(p->history, opts.stall_cycles)) {
                status = fail(RBF_ENOCONV, "stalled: residual %.3e after %d iterations, above "
                                           "half its value %d cycles earlier",
                              rel, iters, opts.stall_cycles);
                break;
            }
            CycleResult cr;
            RBF_TRY(gmres_cycles(p, opts.precision, p->fs, p->x, m, opts.rtol * bnorm, 1,
                                 opts.max_iters - iters, st, &cr, &pt, p->r));
            iters += cr.iters;
            cycles += cr.cycles;
            if (cr.breakdown) {
                RBF_TRY(true_rel_residual(p, p->fs, p->x, bnorm, &rel, st, &pt));
                p->history.push_back(rel);
                if (rel > opts.rtol)
                    status = fail(RBF_EBREAKDOWN, "Arnoldi breakdown at residual %.3e", rel);
                break;
            }
        }
    } else {
        // mixed: FP64 residual, FP32 inner GMRES on A d = r, FP64 update.  An
        // outer step that does not lower the FP64 residual (the FP32 product's
        // error times a large correction outweighs what the inner solve
        // removed: kappa(A) u32 near or above 1) is undone, and the refinement
        // stops there with the previous iterate.
        double prev = 0.0;
        for (;;) {
            RBF_TRY(true_rel_residual(p, p->fs, p->x, bnorm, &rel, st, &pt));
            p->history.push_back(rel);
            if (outer > 0 && !(rel < prev)) {
                HIP_TRY(hipMemcpyAsync(p->x, p->rhs, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
                const double worse = rel;
                rel = prev;
                status = fail(RBF_ENOCONV,
                              "refinement stalled after %d outer steps: residual %.3e, the next "
                              "step gave %.3e",
                              outer - 1, rel, worse);
                break;
            }
            if (!std::isfinite(rel)) {
                status = fail(RBF_ENAN, "non-finite residual");
                break;
            }
            if (rel <= opts.rtol) break;
            if (outer >= opts.max_outer || iters >= opts.max_iters) {
                status = fail(RBF_ENOCONV, "no convergence in %d outer steps (rel. residual %.3e)",
                              outer, rel);
                break;
            }
            double rnorm = rel * bnorm;
            HIP_TRY(rbf::launch_fill(p->d, 0.0, n, st));
            CycleResult cr;
            // the residual is overwritten by later true-residual checks: keep a copy
            HIP_TRY(hipMemcpyAsync(p->rhs, p->r, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            RBF_TRY(gmres_cycles(p, RBF_MIXED, p->rhs, p->d, m,
                                 std::max(opts.inner_rtol * rnorm, 0.5 * opts.rtol * bnorm), 1,
                                 opts.max_iters - iters, st, &cr, &pt, p->rhs));
            // the inner solve is done with its right-hand side: keep the
            // iterate there in case this step has to be undone
            HIP_TRY(hipMemcpyAsync(p->rhs, p->x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            HIP_TRY(rbf::launch_axpy(1.0, p->d, p->x, n, st));
            prev = rel;
            iters += cr.iters;
            cycles += cr.cycles;
            ++outer;
        }
    }
    // keep the solution for evaluate
    if (!p->lam) RBF_TRY(p->alloc_n(&p->lam, n));
    HIP_TRY(hipMemcpyAsync(p->lam, p->x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    p->solved = (status == RBF_OK);
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->iterations = iters;
        info->outer_iterations = outer;
        info->restarts = cycles;
        info->rel_residual = rel;
        info->t_init = p->t_init;
        info->t_pcsetup = t_pc;
        info->t_matmult = pt.matmult;
        info->t_matsolve = pt.matsolve;
        info->t_vecmdot = pt.vecmdot;
        double acc = t_pc + pt.matmult + pt.matsolve + pt.vecmdot;
        info->t_other = std::max(0.0, total.sec() - acc);
        info->interactions_per_matvec = p->interactions;
        info->matvecs64 = pt.mv64;
        info->matvecs32 = pt.mv32;
        info->precond_applies = pt.pc;
        info->device_bytes = p->bytes;
        info->history_len = (int)p->history.size();
        info->history = p->history.data();
        info->shifted_blocks = opts.precision != RBF_FP64 ? p->shifted_blocks32 : 0;
    }
    return status;
}

rbf_status count_interactions(rbf_problem* p, int* d_nnb_sorted, hipStream_t st) {
    double* y;
    RBF_TRY(p->alloc_n(&y, p->n));
    long long* tot;
    RBF_TRY(p->alloc_n(&tot, 1));
    HIP_TRY(hipMemcpyAsync(y, p->fs, sizeof(double) * p->n, hipMemcpyDeviceToDevice, st));
    if (p->boxT)
        HIP_TRY(rbf::launch_evaluate_box(p->mv_args(), p->bt_args(), p->xs, p->ys, p->n, p->fs, y,
                                         d_nnb_sorted, st));
    else
        HIP_TRY(rbf::launch_matvec64(p->mv_args(), p->fs, y, d_nnb_sorted, st));
    HIP_TRY(rbf::launch_sum_counts(d_nnb_sorted, p->n, tot, st));
    long long h = 0;
    HIP_TRY(hipMemcpyAsync(&h, tot, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    p->interactions = h;
    p->release(y, st);
    p->release(tot, st);
    return RBF_OK;
}

rbf_status evaluate_impl(const rbf_problem* cp, const double* d_t, long long m, double* d_out,
                         hipStream_t st, int* d_counts = nullptr) {
    rbf_problem* p = const_cast<rbf_problem*>(cp);
    if (!d_counts && (!p->solved || !p->lam))
        return fail(RBF_ESTATE, "evaluate needs a successful solve first");
    if (m == 0) return RBF_OK;
    if (m < 0 || !d_t || !d_out) return fail(RBF_EINVAL, "bad targets");
    const long long nc = p->ncells;
    double* work;
    int *flag, *cell_of, *slot, *counts, *tcs, *tperm, *scan_work;
    double *tx, *ty, *yo;
    float *fx, *fy;
    RBF_TRY(p->alloc_n(&work, 4 * rbf::kReduceBlocks + 4));
    RBF_TRY(p->alloc_n(&flag, 4));
    HIP_TRY(hipMemsetAsync(flag, 0, 4 * sizeof(int), st));
    HIP_TRY(rbf::launch_minmax(d_t, nullptr, m, work, work + 4 * rbf::kReduceBlocks, flag, st));
    RBF_TRY(p->alloc_n(&cell_of, m));
    RBF_TRY(p->alloc_n(&slot, m));
    RBF_TRY(p->alloc_n(&counts, nc));
    RBF_TRY(p->alloc_n(&tcs, nc + 1));
    RBF_TRY(p->alloc_n(&tperm, m));
    RBF_TRY(p->alloc_n(&scan_work, rbf::scan_work_ints(nc)));
    RBF_TRY(p->alloc_n(&tx, m));
    RBF_TRY(p->alloc_n(&ty, m));
    RBF_TRY(p->alloc_n(&yo, m));
    RBF_TRY(p->alloc_n(&fx, m));
    RBF_TRY(p->alloc_n(&fy, m));
    HIP_TRY(hipMemsetAsync(counts, 0, sizeof(int) * nc, st));
    HIP_TRY(rbf::launch_cell_count(d_t, m, p->g, cell_of, slot, counts, st));
    HIP_TRY(rbf::launch_exclusive_scan(counts, tcs, nc, scan_work, st));
    HIP_TRY(rbf::launch_scatter(cell_of, slot, tcs, m, tperm, st));
    HIP_TRY(rbf::launch_gather(d_t, nullptr, tperm, cell_of, m, p->g, p->sc32, tx, ty, nullptr, fx,
                               fy, st));
    rbf::MatvecArgs a = p->mv_args();
    a.tx = tx;
    a.ty = ty;
    a.tcell = tcs;
    if (d_counts) {   // the targets' in-cutoff counts: the product of the data f
        int* cnt_sorted;
        RBF_TRY(p->alloc_n(&cnt_sorted, m));
        if (p->boxT)
            HIP_TRY(rbf::launch_evaluate_box(a, p->bt_args(), tx, ty, m, p->fs, yo, cnt_sorted, st));
        else
            HIP_TRY(rbf::launch_matvec64(a, p->fs, yo, cnt_sorted, st));
        HIP_TRY(rbf::launch_unpermute_int(cnt_sorted, tperm, m, d_counts, st));
        HIP_TRY(hipStreamSynchronize(st));
        p->release(cnt_sorted, st);
    } else {
        if (p->boxT)
            HIP_TRY(rbf::launch_evaluate_box(a, p->bt_args(), tx, ty, m, p->lam, yo, nullptr, st));
        else
            HIP_TRY(rbf::launch_matvec64(a, p->lam, yo, nullptr, st));
        HIP_TRY(rbf::launch_unpermute(yo, tperm, m, d_out, st));
    }
    int hflag = 0;
    HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (void* q : {(void*)work, (void*)flag, (void*)cell_of, (void*)slot, (void*)counts, (void*)tcs,
                    (void*)tperm, (void*)scan_work, (void*)tx, (void*)ty, (void*)yo, (void*)fx,
                    (void*)fy})
        p->release(q, st);
    if (hflag) return fail(RBF_EINVAL, "targets contain NaN or Inf");
    return RBF_OK;
}

}  // namespace

// ---- the packed solve engine -------------------------------------------------
// Advances the GMRES(m) solves of several prepared problems together: one
// engine step runs, for every active problem, one Arnoldi step, or the start
// (x = 0, ||f||) or the end of a cycle with its true residual, and every
// kernel of the step is launched once for all problems through device job
// tables.  Each problem runs exactly the operations of solve_impl, in the same
// order and with the same per-problem block decompositions, so its weights are
// bit-identical to a lone solve; the host keeps each problem's Givens
// recurrence.  A step is a fixed sequence of phases and every problem holds one
// job slot per phase (marked idle when its state needs no work there), so the
// step's launches depend only on the set of active problems: with graphs on,
// they are captured once per set as a HIP graph whose first node copies the
// step's job tables from pinned host memory, and replayed every step.
namespace rbf {

namespace {

enum : int {   // vector phases of a step, in launch order
    kVPrep = 0,    // x = 0 | V_0 = r / ||r|| | w = V y
    kVUpd,         // x += z
    kVSub,         // r = f - w
    kVAxpy1,       // w -= V h1
    kVAxpy2,       // w -= V h2
    kVScale,       // V_{j+1} = w / ||w||
    kVPhases
};

struct EngResult {   // per problem, written by the step's reductions
    double h1[64], h2[64], n2;
};

struct EngProb {
    rbf_problem* p = nullptr;
    rbf_solve_opts o{};
    double* lam_out = nullptr;
    void* tag = nullptr;
    bool mixed = false;
    int m = 30;
    enum St { kInit, kResid, kArnoldi, kUpdate } st = kInit;
    bool start_cycle = false;
    int j = 0, k = 0;
    std::vector<double> H, cs, sn, gv, yv;
    double bnorm = 0, rel = 0, tol_abs = 0, est = 0;
    double prev = 0;     // mixed: the residual before the current outer step
    bool undo = false;   // mixed: the current outer step changed x (its old x is in p->rhs)
    int iters = 0, cycles = 0, outer = 0, mv64 = 0, mv32 = 0, pc = 0;
    bool breakdown = false;
    int slot = -1;   // its result slot, kept while it is active
    // block counts of its jobs
    int nb_vec = 0, nb_dot = 0, ngroups = 0, nsub = 0;
};

}  // namespace

class Engine {
public:
    hipStream_t st = nullptr;
    int cap = 0;
    bool use_graphs = false;
    std::vector<EngProb> act;         // active problems, in join order
    std::vector<EngProb> joining;     // added since the last step
    // tables: pinned host staging and its device copy, laid out for the current set
    char* h_tab = nullptr;
    char* d_tab = nullptr;
    size_t tab_bytes = 0, tab_cap = 0;
    EngResult* d_res = nullptr;       // cap results, one slot per active problem
    EngResult* h_res = nullptr;       // pinned
    std::vector<int> free_slots;
    double* d_coef = nullptr;         // cap x 64 update coefficients (inside the tables)
    struct Layout {
        size_t vec[kVPhases], bvec[kVPhases], dot[3], bdot[3], bred[3], mv, bmv, rasm, brasm, coef;
        int nvec[kVPhases], ndot[3], nred[3], nmv, nrasm, mv_threads;
    } L{};
    bool layout_valid = false;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t ev_done = nullptr;

    ~Engine() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (ev_done) (void)hipEventDestroy(ev_done);
        if (h_tab) (void)hipHostFree(h_tab);
        if (d_tab) (void)hipFree(d_tab);
        if (d_res) (void)hipFree(d_res);
        if (h_res) (void)hipHostFree(h_res);
    }

    template <typename J>
    J* host(size_t off) { return reinterpret_cast<J*>(h_tab + off); }
    template <typename J>
    J* dev(size_t off) { return reinterpret_cast<J*>(d_tab + off); }

    // offsets of every table for the active set, and their block offsets
    hipError_t plan() {
        const int na = (int)act.size();
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t o = off;
            off += (bytes + 255) / 256 * 256;
            return o;
        };
        for (int v = 0; v < kVPhases; ++v) {
            L.vec[v] = take(sizeof(VecJob) * na);
            L.bvec[v] = take(sizeof(int) * (na + 1));
        }
        for (int d = 0; d < 3; ++d) {
            L.dot[d] = take(sizeof(DotJob) * na);
            L.bdot[d] = take(sizeof(int) * (na + 1));
            L.bred[d] = take(sizeof(int) * (na + 1));
        }
        L.mv = take(sizeof(MatvecJob) * na);
        L.bmv = take(sizeof(int) * (na + 1));
        L.rasm = take(sizeof(RasmJob) * na);
        L.brasm = take(sizeof(int) * (na + 1));
        L.coef = take(sizeof(double) * 64 * na);
        tab_bytes = off;
        if (tab_bytes > tab_cap) {
            if (h_tab) (void)hipHostFree(h_tab);
            if (d_tab) (void)hipFree(d_tab);
            h_tab = nullptr;
            d_tab = nullptr;
            tab_cap = 0;
            hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&h_tab), tab_bytes);
            if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d_tab), tab_bytes);
            if (e != hipSuccess) return e;
            tab_cap = tab_bytes;
        }
        // block offsets: fixed per problem, whatever its state
        auto offsets = [&](size_t o, auto count) {
            int* b = host<int>(o);
            b[0] = 0;
            for (int q = 0; q < na; ++q) b[q + 1] = b[q] + count(act[q]);
            return b[na];
        };
        for (int v = 0; v < kVPhases; ++v) L.nvec[v] = offsets(L.bvec[v], [](const EngProb& q) { return q.nb_vec; });
        for (int d = 0; d < 3; ++d) {
            L.ndot[d] = offsets(L.bdot[d], [](const EngProb& q) { return q.nb_dot; });
            L.nred[d] = offsets(L.bred[d], [](const EngProb& q) { return q.m + 1; });
        }
        L.nmv = offsets(L.bmv, [](const EngProb& q) { return q.ngroups; });
        L.nrasm = offsets(L.brasm, [](const EngProb& q) { return q.nsub; });
        L.mv_threads = 64;
        for (const EngProb& q : act) L.mv_threads = std::max(L.mv_threads, 64 * q.p->nl.gunits);
        d_coef = dev<double>(L.coef);
        layout_valid = true;
        return hipSuccess;
    }

    // the launches of one step, on stream s (captured or not)
    hipError_t enqueue(hipStream_t s) {
        const int na = (int)act.size();
        hipError_t e = hipMemcpyAsync(d_tab, h_tab, tab_bytes, hipMemcpyHostToDevice, s);
        auto vec = [&](int v) {
            if (e == hipSuccess)
                e = launch_vec_packed(dev<VecJob>(L.vec[v]), dev<int>(L.bvec[v]), na, L.nvec[v], s);
        };
        auto dot = [&](int d) {
            if (e == hipSuccess)
                e = launch_multidot_packed(dev<DotJob>(L.dot[d]), dev<int>(L.bdot[d]), na, L.ndot[d], s);
            if (e == hipSuccess)
                e = launch_reduce_packed(dev<DotJob>(L.dot[d]), dev<int>(L.bred[d]), na, L.nred[d], s);
        };
        vec(kVPrep);
        if (e == hipSuccess)
            e = launch_rasm_packed(dev<RasmJob>(L.rasm), dev<int>(L.brasm), na, L.nrasm, s);
        vec(kVUpd);
        if (e == hipSuccess)
            e = launch_matvec_lists_packed(dev<MatvecJob>(L.mv), dev<int>(L.bmv), na, L.nmv,
                                           L.mv_threads, s);
        vec(kVSub);
        dot(0);
        vec(kVAxpy1);
        dot(1);
        vec(kVAxpy2);
        dot(2);
        vec(kVScale);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h_res, d_res, sizeof(EngResult) * cap, hipMemcpyDeviceToHost, s);
        return e;
    }

    // the step's jobs of problem q (slot i) from its state
    void fill(int i, EngProb& q) {
        rbf_problem* p = q.p;
        const long long n = p->n;
        const int prec = (q.mixed && q.st == EngProb::kArnoldi) ? 1 : 0;   // the operator's precision
        // the preconditioner's: FP64 Z; FP32 Z with FP32 sums; FP32 Z with FP64 sums
        const int rprec = q.mixed ? 1 : (q.o.precision == RBF_FP64_PC32 ? 2 : 0);
        for (int v = 0; v < kVPhases; ++v) {
            VecJob& J = host<VecJob>(L.vec[v])[i];
            J = VecJob{};
            J.op = VecJob::kNop;
            J.n = n;
        }
        for (int d = 0; d < 3; ++d) {
            DotJob& D = host<DotJob>(L.dot[d])[i];
            D = DotJob{};
            D.nb = q.nb_dot;
            D.n = n;
            D.partial = p->partial;
        }
        MatvecJob& M = host<MatvecJob>(L.mv)[i];
        M = MatvecJob{};
        M.a = p->mv_args();
        M.a32 = p->mv32_args();
        M.nl = p->nl;
        M.skip = 1;
        RasmJob& Rj = host<RasmJob>(L.rasm)[i];
        Rj = RasmJob{};
        Rj.a = p->pc_args();
        Rj.Z = rprec ? static_cast<const void*>(p->Z32) : static_cast<const void*>(p->Z64);
        Rj.prec = rprec;
        Rj.skip = 1;
        EngResult* res = d_res + q.slot;
        double* res_n2 = &res->n2;
        auto dotjob = [&](int d, const double* V, long long ldv, int nv, const double* w, double* out) {
            DotJob& D = host<DotJob>(L.dot[d])[i];
            D.V = V;
            D.ldv = ldv;
            D.nv = nv;
            D.w = w;
            D.out = out;
        };
        auto resid = [&]() {   // w = A x, r = f - w, <r, r>
            M.skip = 0;
            M.prec = 0;
            M.w = p->x;
            M.y = p->w;
            VecJob& S = host<VecJob>(L.vec[kVSub])[i];
            S.op = VecJob::kSub;
            S.a = p->fs;
            S.b = p->w;
            S.y = p->r;
            dotjob(0, p->r, 0, 1, p->r, res_n2);
        };
        switch (q.st) {
            case EngProb::kInit: {
                VecJob& F = host<VecJob>(L.vec[kVPrep])[i];
                F.op = VecJob::kFill;
                F.y = p->x;
                dotjob(0, p->fs, 0, 1, p->fs, res_n2);
                break;
            }
            case EngProb::kResid:
                resid();
                break;
            case EngProb::kArnoldi: {
                double* V = p->V;
                double* vj = V + (long long)q.j * n;
                if (q.start_cycle) {
                    VecJob& P0 = host<VecJob>(L.vec[kVPrep])[i];
                    P0.op = VecJob::kScaleByInv;
                    P0.a = p->r;
                    P0.den = res_n2;
                    P0.y = V;
                }
                Rj.skip = 0;
                Rj.v = vj;
                Rj.z = p->z;
                M.skip = 0;
                M.prec = prec;
                M.w = p->z;
                M.y = p->w;
                dotjob(0, V, n, q.j + 1, p->w, res->h1);
                VecJob& A1 = host<VecJob>(L.vec[kVAxpy1])[i];
                A1.op = VecJob::kMultiAxpy;
                A1.a = V;
                A1.ld = n;
                A1.nv = q.j + 1;
                A1.coef = res->h1;
                A1.y = p->w;
                A1.sign = -1.0;
                dotjob(1, V, n, q.j + 1, p->w, res->h2);
                VecJob& A2 = host<VecJob>(L.vec[kVAxpy2])[i];
                A2 = A1;
                A2.coef = res->h2;
                dotjob(2, p->w, 0, 1, p->w, res_n2);
                VecJob& Sc = host<VecJob>(L.vec[kVScale])[i];
                Sc.op = VecJob::kScaleByInv;
                Sc.a = p->w;
                Sc.den = res_n2;
                Sc.y = V + (long long)(q.j + 1) * n;
                break;
            }
            case EngProb::kUpdate: {
                double* coef = host<double>(L.coef) + 64 * i;
                for (int t = 0; t < q.k; ++t) coef[t] = q.yv[t];
                VecJob& P0 = host<VecJob>(L.vec[kVPrep])[i];
                P0.op = VecJob::kMultiAxpy;
                P0.a = p->V;
                P0.ld = n;
                P0.nv = q.k;
                P0.coef = d_coef + 64 * i;
                P0.y = p->w;
                P0.sign = 1.0;
                P0.overwrite = 1;
                Rj.skip = 0;
                Rj.v = p->w;
                Rj.z = p->z;
                VecJob& U = host<VecJob>(L.vec[kVUpd])[i];
                U.op = q.mixed ? VecJob::kAxpyKeep : VecJob::kAxpy;   // mixed: keep the old x
                U.a = p->z;
                U.y = p->x;
                U.keep = p->rhs;
                if (q.mixed) q.undo = true;
                resid();
                break;
            }
        }
    }

    // the true residual's decision (solve_impl's loop head); false: the problem ended
    bool decide(EngProb& q, std::vector<EngineDone>* done, double n2) {
        rbf_problem* p = q.p;
        q.rel = std::sqrt(n2) / q.bnorm;
        p->history.push_back(q.rel);
        rbf_status s = RBF_OK;
        std::string msg;
        if (q.mixed && q.outer > 0 && !(q.rel < q.prev)) {   // as the lone solve: undo, stop
            if (q.undo &&
                hipMemcpyAsync(p->x, p->rhs, sizeof(double) * p->n, hipMemcpyDeviceToDevice, st) !=
                    hipSuccess) {
                finish(q, done, RBF_EDEVICE, "copy failed");
                return false;
            }
            const double worse = q.rel;
            q.rel = q.prev;
            char buf[160];
            snprintf(buf, sizeof buf,
                     "refinement stalled after %d outer steps: residual %.3e, the next step gave %.3e",
                     q.outer - 1, q.rel, worse);
            finish(q, done, RBF_ENOCONV, buf);
            return false;
        }
        if (!std::isfinite(q.rel)) {
            s = RBF_ENAN;
            msg = "non-finite residual";
        } else if (q.rel <= q.o.rtol) {
            s = RBF_OK;
        } else if (!q.mixed && q.iters >= q.o.max_iters) {
            s = RBF_ENOCONV;
        } else if (!q.mixed && stalled(p->history, q.o.stall_cycles)) {
            char buf[160];
            snprintf(buf, sizeof buf,
                     "stalled: residual %.3e after %d iterations, above half its value %d cycles "
                     "earlier",
                     q.rel, q.iters, q.o.stall_cycles);
            finish(q, done, RBF_ENOCONV, buf);
            return false;
        } else if (q.mixed && (q.outer >= q.o.max_outer || q.iters >= q.o.max_iters)) {
            s = RBF_ENOCONV;
        } else {
            // a new cycle: beta = ||r|| (the lone solve's norm of its copy of r)
            const double beta = std::sqrt(n2);
            q.tol_abs = q.mixed ? std::max(q.o.inner_rtol * (q.rel * q.bnorm), 0.5 * q.o.rtol * q.bnorm)
                                : q.o.rtol * q.bnorm;
            if (!std::isfinite(beta)) {
                finish(q, done, RBF_ENAN, "non-finite residual");
                return false;
            }
            q.prev = q.rel;
            if (beta <= q.tol_abs) {   // nothing to do in this cycle
                if (q.mixed) {
                    ++q.outer;
                    q.undo = false;
                    q.st = EngProb::kResid;
                    return true;
                }
                finish(q, done, RBF_ENOCONV, "residual estimate below tolerance, true residual above");
                return false;
            }
            q.est = beta;
            std::fill(q.H.begin(), q.H.end(), 0.0);
            std::fill(q.gv.begin(), q.gv.end(), 0.0);
            q.gv[0] = beta;
            q.j = 0;
            q.k = 0;
            q.breakdown = false;
            q.start_cycle = true;
            q.st = EngProb::kArnoldi;
            return true;
        }
        if (s == RBF_ENOCONV) {
            char buf[160];
            snprintf(buf, sizeof buf, q.mixed ? "no convergence in %d outer steps (rel. residual %.3e)"
                                              : "no convergence in %d iterations (rel. residual %.3e)",
                     q.mixed ? q.outer : q.iters, q.rel);
            msg = buf;
        }
        finish(q, done, s, msg);
        return false;
    }

    void finish(EngProb& q, std::vector<EngineDone>* done, rbf_status s, const std::string& msg) {
        rbf_problem* p = q.p;
        hipError_t e = launch_unpermute(p->x, p->perm, p->n, q.lam_out, st);
        if (e == hipSuccess && !p->lam) {
            if (p->alloc_n(&p->lam, p->n) != RBF_OK) e = hipErrorOutOfMemory;
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->lam, p->x, sizeof(double) * p->n, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess && s == RBF_OK) s = RBF_EDEVICE;
        p->solved = s == RBF_OK;
        // the information a lone solve reports (phase times are not per problem here)
        p->last_info = rbf_solve_info{};
        rbf_solve_info& info = p->last_info;
        info.iterations = q.iters;
        info.outer_iterations = q.outer;
        info.restarts = q.cycles;
        info.rel_residual = q.rel;
        info.t_init = p->t_init;
        info.t_pcsetup = q.o.precision == RBF_FP64 ? p->t_pcsetup64 : p->t_pcsetup32;
        info.interactions_per_matvec = p->interactions;
        info.matvecs64 = q.mv64;
        info.matvecs32 = q.mv32;
        info.precond_applies = q.pc;
        info.device_bytes = p->bytes;
        info.shifted_blocks = q.o.precision == RBF_FP64 ? 0 : p->shifted_blocks32;
        p->mark(st);
        done->push_back(EngineDone{q.tag, s, e != hipSuccess ? hipGetErrorString(e) : msg});
        free_slots.push_back(q.slot);
        q.p = nullptr;   // ended
    }

    // after the step: read each problem's results and advance its state
    void advance(std::vector<EngineDone>* done) {
        for (size_t i = 0; i < act.size(); ++i) {
            EngProb& q = act[i];
            const EngResult& r = h_res[q.slot];
            switch (q.st) {
                case EngProb::kInit: {
                    q.bnorm = std::sqrt(r.n2);
                    q.p->history.clear();
                    if (q.bnorm == 0.0) {
                        q.rel = 0.0;
                        finish(q, done, RBF_OK, "");
                    } else {
                        q.st = EngProb::kResid;
                    }
                    break;
                }
                case EngProb::kResid:
                    q.mv64 += 1;
                    decide(q, done, r.n2);
                    break;
                case EngProb::kArnoldi: {
                    q.start_cycle = false;
                    q.pc += 1;
                    (q.mixed ? q.mv32 : q.mv64) += 1;
                    const int m = q.m, j = q.j;
                    std::vector<double>& H = q.H;
                    for (int t = 0; t <= j; ++t) H[(size_t)t * m + j] = r.h1[t] + r.h2[t];
                    const double hn = std::sqrt(r.n2);
                    H[(size_t)(j + 1) * m + j] = hn;
                    for (int t = 0; t < j; ++t) {
                        const double a = H[(size_t)t * m + j], bb = H[(size_t)(t + 1) * m + j];
                        H[(size_t)t * m + j] = q.cs[t] * a + q.sn[t] * bb;
                        H[(size_t)(t + 1) * m + j] = -q.sn[t] * a + q.cs[t] * bb;
                    }
                    const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
                    const double rho = std::hypot(a, bb);
                    if (!std::isfinite(rho)) {
                        finish(q, done, RBF_ENAN, "non-finite Hessenberg entry");
                        break;
                    }
                    q.cs[j] = rho > 0 ? a / rho : 1.0;
                    q.sn[j] = rho > 0 ? bb / rho : 0.0;
                    H[(size_t)j * m + j] = rho;
                    H[(size_t)(j + 1) * m + j] = 0.0;
                    q.gv[j + 1] = -q.sn[j] * q.gv[j];
                    q.gv[j] = q.cs[j] * q.gv[j];
                    ++q.iters;
                    q.k = j + 1;
                    q.est = std::fabs(q.gv[j + 1]);
                    bool stop = false;
                    if (hn == 0.0) {
                        q.breakdown = true;
                        stop = true;
                    }
                    if (q.est <= q.tol_abs || q.iters >= q.o.max_iters) stop = true;
                    if (stop || j + 1 == m) {
                        // y = H^{-1} g for the cycle's end, next step
                        for (int t = q.k - 1; t >= 0; --t) {
                            double sacc = q.gv[t];
                            for (int jj = t + 1; jj < q.k; ++jj) sacc -= H[(size_t)t * m + jj] * q.yv[jj];
                            q.yv[t] = sacc / H[(size_t)t * m + t];
                        }
                        q.st = EngProb::kUpdate;
                    } else {
                        q.j = j + 1;
                    }
                    break;
                }
                case EngProb::kUpdate: {
                    q.pc += 1;
                    q.mv64 += 1;
                    ++q.cycles;
                    if (q.mixed) {
                        ++q.outer;
                        decide(q, done, r.n2);
                    } else if (q.breakdown) {
                        q.rel = std::sqrt(r.n2) / q.bnorm;
                        q.p->history.push_back(q.rel);
                        if (q.rel > q.o.rtol) {
                            char buf[96];
                            snprintf(buf, sizeof buf, "Arnoldi breakdown at residual %.3e", q.rel);
                            finish(q, done, RBF_EBREAKDOWN, buf);
                        } else {
                            finish(q, done, RBF_OK, "");
                        }
                    } else {
                        decide(q, done, r.n2);
                    }
                    break;
                }
            }
        }
        // drop the problems that ended
        std::vector<EngProb> keep;
        for (EngProb& q : act)
            if (q.p) keep.push_back(std::move(q));
        if (keep.size() != act.size()) layout_valid = false;
        act.swap(keep);
    }

    rbf_status step(std::vector<EngineDone>* done) {
        if (!joining.empty()) {
            for (EngProb& q : joining) act.push_back(std::move(q));
            joining.clear();
            layout_valid = false;
        }
        if (act.empty()) return RBF_OK;
        if (!layout_valid) {
            if (gexec) {
                (void)hipGraphExecDestroy(gexec);
                gexec = nullptr;
            }
            HIP_TRY(plan());
        }
        for (size_t i = 0; i < act.size(); ++i) fill((int)i, act[i]);
        if (use_graphs && !gexec) {
            hipGraph_t g = nullptr;
            hipStream_t cs = nullptr;
            bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
            if (ok) ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                const hipError_t le = enqueue(cs);
                const hipError_t ce = hipStreamEndCapture(cs, &g);
                ok = le == hipSuccess && ce == hipSuccess && g != nullptr;
            }
            if (ok) ok = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
            if (cs) (void)hipStreamDestroy(cs);
            (void)hipGetLastError();
            if (!ok) {
                if (gexec) (void)hipGraphExecDestroy(gexec);
                gexec = nullptr;
                use_graphs = false;   // launch one by one from now on
            }
        }
        if (gexec)
            HIP_TRY(hipGraphLaunch(gexec, st));
        else
            HIP_TRY(enqueue(st));
        HIP_TRY(hipEventRecord(ev_done, st));
        HIP_TRY(hipEventSynchronize(ev_done));
        advance(done);
        return RBF_OK;
    }
};

Engine* engine_create(hipStream_t st, int capacity, bool graphs) {
    Engine* e = new (std::nothrow) Engine();
    if (!e) return nullptr;
    e->st = st;
    e->cap = std::max(1, std::min(capacity, 64));
    e->use_graphs = graphs;
    for (int k = e->cap - 1; k >= 0; --k) e->free_slots.push_back(k);
    if (hipMalloc(reinterpret_cast<void**>(&e->d_res), sizeof(EngResult) * e->cap) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&e->h_res), sizeof(EngResult) * e->cap) != hipSuccess ||
        hipEventCreateWithFlags(&e->ev_done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        delete e;
        return nullptr;
    }
    return e;
}

void engine_destroy(Engine* e) { delete e; }

int engine_active(const Engine* e) { return (int)(e->act.size() + e->joining.size()); }

rbf_status engine_add(Engine* e, rbf_problem* p, const rbf_solve_opts& o, double* d_lam_out,
                      void* tag) {
    if (engine_active(e) >= e->cap) return fail(RBF_ELIMIT, "the engine is full");
    if (p->nl.nunits == 0) return fail(RBF_ELIMIT, "the problem has no neighbour lists");
    if (p->boxT) return fail(RBF_ELIMIT, "box-truncated products are not packed");
    if (o.restart < 1 || o.restart > 63) return fail(RBF_EINVAL, "restart must be in [1, 63]");
    if (o.stall_cycles < 0) return fail(RBF_EINVAL, "stall_cycles must be >= 0");
    if (!p->have_values) return fail(RBF_ESTATE, "no right-hand side");
    if (o.precision != RBF_FP64 && o.precision != RBF_MIXED && o.precision != RBF_FP64_PC32)
        return fail(RBF_EINVAL, "unknown precision");
    const bool mixed = o.precision == RBF_MIXED;
    if (o.precision == RBF_FP64 ? !p->Z64 : !p->Z32)
        return fail(RBF_ESTATE, "the preconditioner is not built");
    RBF_TRY(ensure_workspace(p, o.restart, e->st));
    EngProb q;
    q.p = p;
    q.o = o;
    q.lam_out = d_lam_out;
    q.tag = tag;
    q.mixed = mixed;
    q.m = o.restart;
    q.H.assign((size_t)(q.m + 1) * q.m, 0.0);
    q.cs.assign(q.m, 0.0);
    q.sn.assign(q.m, 0.0);
    q.gv.assign(q.m + 1, 0.0);
    q.yv.assign(q.m, 0.0);
    q.nb_vec = vec_blocks(p->n);
    q.nb_dot = dot_blocks(p->n);
    q.ngroups = p->nl.ngroups;
    q.nsub = (int)p->nsub;
    q.slot = e->free_slots.back();
    e->free_slots.pop_back();
    p->history.clear();
    e->joining.push_back(std::move(q));
    return RBF_OK;
}

rbf_status engine_step(Engine* e, std::vector<EngineDone>* done) {
    try {
        return e->step(done);
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in the packed engine");
    }
}

void engine_info(const rbf_problem* p, rbf_solve_info* info) {
    if (info) *info = p->last_info;
}

}  // namespace rbf

extern "C" {

void rbf_default_opts(rbf_solve_opts* o) {
    if (!o) return;
    o->restart = 30;
    o->max_iters = 10000;
    o->rtol = 1e-10;
    o->precision = RBF_FP64;
    o->inner_rtol = 1e-4;
    o->max_outer = 60;
    o->max_device_bytes = 0;
    o->stream = nullptr;
    o->stall_cycles = 0;
}

rbf_status rbf_setup(const double* points, const double* values, long long n, double sigma,
                     double cutoff, int overlap, rbf_problem** out) {
    try {
        return create(points, values, false, n, sigma, cutoff, overlap, nullptr, out);
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_setup");
    }
}

rbf_status rbf_setup_device(const double* d_points, const double* d_values, long long n,
                            double sigma, double cutoff, int overlap, void* stream,
                            rbf_problem** out) {
    try {
        return create(d_points, d_values, true, n, sigma, cutoff, overlap, as_stream(stream), out);
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_setup_device");
    }
}

rbf_status rbf_set_values(rbf_problem* p, const double* values, int on_device, void* stream) {
    if (!p || !values) return fail(RBF_EINVAL, "NULL argument");
    hipStream_t st = as_stream(stream);
    MarkOnExit mk{p, st};
    double* src = const_cast<double*>(values);
    double* tmp = nullptr;
    if (!on_device) {
        RBF_TRY(p->alloc_n(&tmp, p->n));
        HIP_TRY(hipMemcpyAsync(tmp, values, sizeof(double) * p->n, hipMemcpyHostToDevice, st));
        src = tmp;
    }
    int* flag = p->flag;
    HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), st));
    HIP_TRY(rbf::launch_check_finite(src, p->n, flag, st));
    HIP_TRY(rbf::launch_permute(src, p->perm, p->n, p->fs, st));
    int h = 0;
    HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (tmp) p->release(tmp, st);
    if (h) return fail(RBF_EINVAL, "values contain NaN or Inf");
    p->have_values = true;
    p->solved = false;
    return RBF_OK;
}

rbf_status rbf_precond_setup(rbf_problem* p, rbf_precision precision, void* stream) {
    if (!p) return fail(RBF_EINVAL, "NULL problem");
    try {
        MarkOnExit mk{p, as_stream(stream)};
        return precond_setup(p, precision, as_stream(stream));
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_precond_setup");
    }
}

rbf_status rbf_solve(rbf_problem* p, const rbf_solve_opts* opts, const double* lambda0,
                     double* lambda_out, rbf_solve_info* info) {
    if (!p || !lambda_out) return fail(RBF_EINVAL, "NULL argument");
    try {
        MarkOnExit mk{p, as_stream(opts ? opts->stream : nullptr)};
        rbf_status s = solve_impl(p, opts, nullptr, false, lambda0, info);
        if (s != RBF_OK && s != RBF_ENOCONV && s != RBF_EBREAKDOWN) return s;
        hipStream_t st = as_stream(opts ? opts->stream : nullptr);
        std::string keep = g_last_error;
        HIP_TRY(rbf::launch_unpermute(p->x, p->perm, p->n, p->r, st));
        HIP_TRY(hipMemcpyAsync(lambda_out, p->r, sizeof(double) * p->n, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        g_last_error = keep;
        return s;
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_solve");
    }
}

rbf_status rbf_solve_device(rbf_problem* p, const rbf_solve_opts* opts, const double* d_lambda0,
                            double* d_lambda_out, rbf_solve_info* info) {
    if (!p || !d_lambda_out) return fail(RBF_EINVAL, "NULL argument");
    try {
        MarkOnExit mk{p, as_stream(opts ? opts->stream : nullptr)};
        rbf_status s = solve_impl(p, opts, d_lambda0, true, nullptr, info);
        if (s != RBF_OK && s != RBF_ENOCONV && s != RBF_EBREAKDOWN) return s;
        hipStream_t st = as_stream(opts ? opts->stream : nullptr);
        std::string keep = g_last_error;
        HIP_TRY(rbf::launch_unpermute(p->x, p->perm, p->n, d_lambda_out, st));
        g_last_error = keep;
        return s;
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_solve_device");
    }
}

rbf_status rbf_evaluate(const rbf_problem* p, const double* targets, long long m, double* out) {
    if (!p) return fail(RBF_EINVAL, "NULL problem");
    if (m < 0 || (m > 0 && (!targets || !out))) return fail(RBF_EINVAL, "bad targets");
    if (m == 0) return p->solved ? RBF_OK : fail(RBF_ESTATE, "evaluate needs a successful solve first");
    try {
        rbf_problem* q = const_cast<rbf_problem*>(p);
        double *dt, *dout;
        RBF_TRY(q->alloc_n(&dt, 2 * m));
        RBF_TRY(q->alloc_n(&dout, m));
        HIP_TRY(hipMemcpy(dt, targets, sizeof(double) * 2 * m, hipMemcpyHostToDevice));
        rbf_status s = evaluate_impl(p, dt, m, dout, nullptr);
        if (s == RBF_OK) {
            hipError_t e = hipMemcpy(out, dout, sizeof(double) * m, hipMemcpyDeviceToHost);
            if (e != hipSuccess) s = fail(RBF_EDEVICE, "copy out: %s", hipGetErrorString(e));
        }
        q->release(dt, nullptr);
        q->release(dout, nullptr);
        return s;
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_evaluate");
    }
}

rbf_status rbf_evaluate_device(const rbf_problem* p, const double* d_targets, long long m,
                               double* d_out, void* stream) {
    if (!p) return fail(RBF_EINVAL, "NULL problem");
    try {
        MarkOnExit mk{p, as_stream(stream)};
        return evaluate_impl(p, d_targets, m, d_out, as_stream(stream));
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_evaluate_device");
    }
}

namespace {

// cell coordinate of v along one axis: the binning's rule (floor((v - v0) / L)
// by the stored reciprocal, clamped), the arithmetic of every kernel
int axis_cell(double v, double v0, double invL, int n) {
    double t = std::floor((v - v0) * invL);
    if (!(t >= 0.0)) t = 0.0;
    if (t > (double)(n - 1)) t = (double)(n - 1);
    return (int)t;
}

// Lattice indices 0 .. n-1 of one axis (coordinate v0 + i hv) grouped by cell
// (the rule is monotone in i for hv > 0), each run cut into chunks of at most
// kLatticeChunk.
void lattice_chunks(double v0, double hv, long long n, double g0, double invL, int nc,
                    std::vector<rbf::LatticeChunk>* out) {
    long long i = 0;
    while (i < n) {
        const int c = axis_cell(v0 + (double)i * hv, g0, invL, nc);
        long long e = i + 1;
        while (e < n && axis_cell(v0 + (double)e * hv, g0, invL, nc) == c) ++e;
        for (long long t = i; t < e; t += rbf::kLatticeChunk)
            out->push_back({t, c, (int)std::min<long long>(rbf::kLatticeChunk, e - t)});
        i = e;
    }
}

// RBF_OK with nothing to do for an empty lattice (*empty set), else the
// argument checks of both lattice entry points
rbf_status check_lattice(const rbf_problem* p, double x0, double y0, double hx, double hy,
                         long long nx, long long ny, const double* out, bool* empty) {
    *empty = true;
    if (!p->solved || !p->lam) return fail(RBF_ESTATE, "evaluate needs a successful solve first");
    if (nx < 0 || ny < 0) return fail(RBF_EINVAL, "negative lattice size");
    if (nx == 0 || ny == 0) return RBF_OK;
    if (!out) return fail(RBF_EINVAL, "NULL output");
    if (!(hx > 0) || !(hy > 0) || !std::isfinite(x0) || !std::isfinite(y0) ||
        !std::isfinite(x0 + (double)(nx - 1) * hx) || !std::isfinite(y0 + (double)(ny - 1) * hy))
        return fail(RBF_EINVAL, "lattice: need finite origin and spacings > 0 with finite extent");
    if (nx > (1LL << 31) || ny > (1LL << 31) || nx * ny > (1LL << 40))
        return fail(RBF_ELIMIT, "lattice of %lld x %lld targets", nx, ny);
    *empty = false;
    return RBF_OK;
}

rbf_status evaluate_lattice_impl(const rbf_problem* cp, double x0, double y0, double hx, double hy,
                                 long long nx, long long ny, double* d_out, hipStream_t st) {
    rbf_problem* p = const_cast<rbf_problem*>(cp);
    rbf::LatticeArgs L{};
    L.x0 = x0;
    L.y0 = y0;
    L.hx = hx;
    L.hy = hy;
    L.nx = nx;
    if (p->boxT) {   // the box truncation takes target arrays
        const long long m = nx * ny;
        double *tx, *ty;
        RBF_TRY(p->alloc_n(&tx, m));
        RBF_TRY(p->alloc_n(&ty, m));
        HIP_TRY(rbf::launch_lattice_points(L, ny, tx, ty, st));
        HIP_TRY(rbf::launch_evaluate_box(p->mv_args(), p->bt_args(), tx, ty, m, p->lam, d_out,
                                         nullptr, st));
        p->release(tx, st);
        p->release(ty, st);
        return RBF_OK;
    }
    std::vector<rbf::LatticeChunk> col, row;
    lattice_chunks(x0, hx, nx, p->g.x0, p->g.invL, p->g.ncx, &col);
    lattice_chunks(y0, hy, ny, p->g.y0, p->g.invL, p->g.ncy, &row);
    // one 64-thread workgroup per chunk pair, at most 2^32 - 1 threads per launch
    if ((long long)col.size() * (long long)row.size() > (1LL << 26) - 1)
        return fail(RBF_ELIMIT, "lattice needs %zu x %zu chunks of 8 x 8 targets (at most 2^26)",
                    col.size(), row.size());
    rbf::LatticeChunk *dcol, *drow;
    RBF_TRY(p->alloc_n(&dcol, (long long)col.size()));
    RBF_TRY(p->alloc_n(&drow, (long long)row.size()));
    HIP_TRY(hipMemcpyAsync(dcol, col.data(), sizeof(rbf::LatticeChunk) * col.size(),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(drow, row.data(), sizeof(rbf::LatticeChunk) * row.size(),
                           hipMemcpyHostToDevice, st));
    L.col = dcol;
    L.row = drow;
    L.ncol = (int)col.size();
    L.nrow = (int)row.size();
    HIP_TRY(rbf::launch_evaluate_lattice(p->mv_args(), L, p->lam, d_out, st));
    // the chunk tables are host vectors: wait for the copies before they go
    HIP_TRY(hipStreamSynchronize(st));
    p->release(dcol, st);
    p->release(drow, st);
    return RBF_OK;
}

}  // namespace

rbf_status rbf_evaluate_lattice(const rbf_problem* p, double x0, double y0, double hx, double hy,
                                long long nx, long long ny, double* out) {
    if (!p) return fail(RBF_EINVAL, "NULL problem");
    bool empty;
    RBF_TRY(check_lattice(p, x0, y0, hx, hy, nx, ny, out, &empty));
    if (empty) return RBF_OK;
    try {
        MarkOnExit mk{p, nullptr};
        rbf_problem* q = const_cast<rbf_problem*>(p);
        double* dout;
        RBF_TRY(q->alloc_n(&dout, nx * ny));
        rbf_status s = evaluate_lattice_impl(p, x0, y0, hx, hy, nx, ny, dout, nullptr);
        if (s == RBF_OK) {
            hipError_t e = hipMemcpy(out, dout, sizeof(double) * nx * ny, hipMemcpyDeviceToHost);
            if (e != hipSuccess) s = fail(RBF_EDEVICE, "copy out: %s", hipGetErrorString(e));
        }
        q->release(dout, nullptr);
        return s;
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_evaluate_lattice");
    }
}

rbf_status rbf_evaluate_lattice_device(const rbf_problem* p, double x0, double y0, double hx,
                                       double hy, long long nx, long long ny, double* d_out,
                                       void* stream) {
    if (!p) return fail(RBF_EINVAL, "NULL problem");
    bool empty;
    RBF_TRY(check_lattice(p, x0, y0, hx, hy, nx, ny, d_out, &empty));
    if (empty) return RBF_OK;
    try {
        MarkOnExit mk{p, as_stream(stream)};
        return evaluate_lattice_impl(p, x0, y0, hx, hy, nx, ny, d_out, as_stream(stream));
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_evaluate_lattice_device");
    }
}

rbf_status rbf_target_counts_device(const rbf_problem* p, const double* d_targets, long long m,
                                    int* d_counts, void* stream) {
    if (!p) return fail(RBF_EINVAL, "NULL problem");
    if (m < 0 || (m > 0 && (!d_targets || !d_counts))) return fail(RBF_EINVAL, "bad targets");
    if (m == 0) return RBF_OK;
    try {
        MarkOnExit mk{p, as_stream(stream)};
        double* scratch_out;
        rbf_problem* q = const_cast<rbf_problem*>(p);
        RBF_TRY(q->alloc_n(&scratch_out, m));
        rbf_status s = evaluate_impl(p, d_targets, m, scratch_out, as_stream(stream), d_counts);
        q->release(scratch_out, as_stream(stream));
        return s;
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_target_counts_device");
    }
}

void rbf_destroy(rbf_problem* p) { delete p; }

rbf_status rbf_block_cache(int device, int trim, size_t* idle_bytes) {
    try {
        BlockCache& c = BlockCache::get();
        if (idle_bytes) *idle_bytes = c.idle_bytes(device);
        if (trim) (void)c.trim(device);
        return RBF_OK;
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_block_cache");
    }
}

rbf_status rbf_grid(const rbf_problem* p, double* out4, long long* ncxy) {
    if (!p || !out4 || !ncxy) return fail(RBF_EINVAL, "NULL argument");
    out4[0] = p->g.x0;
    out4[1] = p->g.y0;
    out4[2] = p->g.L;
    out4[3] = p->g.invL;
    ncxy[0] = p->g.ncx;
    ncxy[1] = p->g.ncy;
    return RBF_OK;
}

rbf_status rbf_binning(const rbf_problem* p, int* cell_of, int* perm, int* cell_start) {
    if (!p) return fail(RBF_EINVAL, "NULL problem");
    if (cell_of) HIP_TRY(hipMemcpy(cell_of, p->cell_of, sizeof(int) * p->n, hipMemcpyDeviceToHost));
    if (perm) HIP_TRY(hipMemcpy(perm, p->perm, sizeof(int) * p->n, hipMemcpyDeviceToHost));
    if (cell_start)
        HIP_TRY(hipMemcpy(cell_start, p->cell_start, sizeof(int) * (p->ncells + 1),
                          hipMemcpyDeviceToHost));
    return RBF_OK;
}

rbf_status rbf_neighbor_counts(rbf_problem* p, int* nnb, long long* total) {
    if (!p) return fail(RBF_EINVAL, "NULL problem");
    try {
        int *d_sorted, *d_orig;
        RBF_TRY(p->alloc_n(&d_sorted, p->n));
        RBF_TRY(p->alloc_n(&d_orig, p->n));
        RBF_TRY(count_interactions(p, d_sorted, nullptr));
        HIP_TRY(rbf::launch_unpermute_int(d_sorted, p->perm, p->n, d_orig, nullptr));
        if (nnb) HIP_TRY(hipMemcpy(nnb, d_orig, sizeof(int) * p->n, hipMemcpyDeviceToHost));
        HIP_TRY(hipDeviceSynchronize());
        p->release(d_sorted, nullptr);
        p->release(d_orig, nullptr);
        if (total) *total = p->interactions;
        return RBF_OK;
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_neighbor_counts");
    }
}

rbf_status rbf_matvec_device(rbf_problem* p, const double* d_w, double* d_y,
                             rbf_precision precision, rbf_order order, void* stream) {
    if (!p || !d_w || !d_y) return fail(RBF_EINVAL, "NULL argument");
    if (precision != RBF_FP64 && precision != RBF_MIXED) return fail(RBF_EINVAL, "bad precision");
    hipStream_t st = as_stream(stream);
    MarkOnExit mk{p, st};
    try {
        if (order == RBF_ORDER_SORTED) return matvec(p, precision, d_w, d_y, st);
        if (order != RBF_ORDER_ORIGINAL) return fail(RBF_EINVAL, "bad order");
        double *ws, *ys;
        RBF_TRY(p->alloc_n(&ws, p->n));
        RBF_TRY(p->alloc_n(&ys, p->n));
        HIP_TRY(rbf::launch_permute(d_w, p->perm, p->n, ws, st));
        RBF_TRY(matvec(p, precision, ws, ys, st));
        HIP_TRY(rbf::launch_unpermute(ys, p->perm, p->n, d_y, st));
        HIP_TRY(hipStreamSynchronize(st));
        p->release(ws, st);
        p->release(ys, st);
        return RBF_OK;
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_matvec_device");
    }
}

rbf_status rbf_matvec_device_noalloc(rbf_problem* p, const double* d_w, double* d_y,
                                     rbf_precision precision, void* stream) {
    if (!p || !d_w || !d_y) return fail(RBF_EINVAL, "NULL argument");
    if (precision != RBF_FP64 && precision != RBF_MIXED) return fail(RBF_EINVAL, "bad precision");
    if (p->n > rbf::kNoAllocMaxPoints)
        return fail(RBF_ELIMIT, "rbf_matvec_device_noalloc serves at most %lld points (got %lld)",
                    rbf::kNoAllocMaxPoints, p->n);
    hipStream_t st = as_stream(stream);
    MarkOnExit mk{p, st};
    try {
        double* scr = nullptr;
        HIP_TRY(rbf::noalloc_scratch(p->device, &scr));
        double* ws = scr;
        double* ys = scr + rbf::kNoAllocMaxPoints;
        HIP_TRY(rbf::launch_permute(d_w, p->perm, p->n, ws, st));
        RBF_TRY(matvec(p, precision, ws, ys, st));
        HIP_TRY(rbf::launch_unpermute(ys, p->perm, p->n, d_y, st));
        return RBF_OK;
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_matvec_device_noalloc");
    }
}

rbf_status rbf_precond_apply_device(rbf_problem* p, const double* d_v, double* d_z,
                                    rbf_precision precision, rbf_order order, void* stream) {
    if (!p || !d_v || !d_z) return fail(RBF_EINVAL, "NULL argument");
    if (precision != RBF_FP64 && precision != RBF_MIXED && precision != RBF_FP64_PC32)
        return fail(RBF_EINVAL, "bad precision");
    hipStream_t st = as_stream(stream);
    MarkOnExit mk{p, st};
    try {
        if (order == RBF_ORDER_SORTED) return rasm(p, precision, d_v, d_z, st);
        if (order != RBF_ORDER_ORIGINAL) return fail(RBF_EINVAL, "bad order");
        double *vs, *zs;
        RBF_TRY(p->alloc_n(&vs, p->n));
        RBF_TRY(p->alloc_n(&zs, p->n));
        HIP_TRY(rbf::launch_permute(d_v, p->perm, p->n, vs, st));
        rbf_status s = rasm(p, precision, vs, zs, st);
        if (s == RBF_OK) {
            hipError_t e = rbf::launch_unpermute(zs, p->perm, p->n, d_z, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) s = fail(RBF_EDEVICE, "%s", hipGetErrorString(e));
        }
        p->release(vs, st);
        p->release(zs, st);
        return s;
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_precond_apply_device");
    }
}

rbf_status rbf_precond_block(rbf_problem* p, long long c, rbf_precision precision,
                             long long* members, double* z_rows, int* nomega, int* ncentre) {
    if (!p) return fail(RBF_EINVAL, "NULL problem");
    if (c < 0 || c >= p->nsub) return fail(RBF_EINVAL, "subdomain %lld out of range", c);
    try {
        const int no = p->n_omega[c], ncn = p->n_c[c];
        if (nomega) *nomega = no;
        if (ncentre) *ncentre = ncn;
        if (members && p->geo) {
            std::vector<int> perm(p->n);
            long long off = 0;
            HIP_TRY(hipMemcpy(perm.data(), p->perm, sizeof(int) * p->n, hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(&off, p->moff + c, sizeof off, hipMemcpyDeviceToHost));
            std::vector<int> mem(no > 0 ? no : 1);
            if (no > 0)
                HIP_TRY(hipMemcpy(mem.data(), p->mem + off, sizeof(int) * no, hipMemcpyDeviceToHost));
            for (int k = 0; k < no; ++k) members[k] = perm[mem[k]];
        } else if (members) {
            std::vector<int> perm(p->n);
            HIP_TRY(hipMemcpy(perm.data(), p->perm, sizeof(int) * p->n, hipMemcpyDeviceToHost));
            const Grid& g = p->g;
            int cx = (int)(c % g.ncx), cy = (int)(c / g.ncx), ov = p->overlap;
            int xlo = std::max(cx - ov, 0), xhi = std::min(cx + ov, g.ncx - 1);
            long long k = 0;
            for (int dy = -ov; dy <= ov; ++dy) {
                int ny = cy + dy;
                if (ny < 0 || ny >= g.ncy) continue;
                for (int nx = xlo; nx <= xhi; ++nx) {
                    if (nx == cx && dy == 0) continue;
                    long long cc = (long long)ny * g.ncx + nx;
                    for (int s = p->cs_host[cc]; s < p->cs_host[cc + 1]; ++s) members[k++] = perm[s];
                }
            }
            for (int s = p->cs_host[c]; s < p->cs_host[c + 1]; ++s) members[k++] = perm[s];
        }
        if (z_rows && ncn > 0) {
            RBF_TRY(precond_setup(p, precision, nullptr));
            const long long cnt = (long long)no * ncn;
            if (precision == RBF_FP64) {
                HIP_TRY(hipMemcpy(z_rows, p->Z64 + p->zoff_host[c], sizeof(double) * cnt,
                                  hipMemcpyDeviceToHost));
            } else {
                std::vector<float> t(cnt);
                HIP_TRY(hipMemcpy(t.data(), p->Z32 + p->zoff_host[c], sizeof(float) * cnt,
                                  hipMemcpyDeviceToHost));
                for (long long i = 0; i < cnt; ++i) z_rows[i] = t[i];
            }
        }
        return RBF_OK;
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_precond_block");
    }
}

rbf_status rbf_set_geometry(rbf_problem* p, const rbf_geometry* geo, void* stream) {
    if (!p || !geo) return fail(RBF_EINVAL, "NULL argument");
    const double B = geo->box, D = geo->overlap, T = geo->truncation;
    if (!(B > 0) || !std::isfinite(B) || !(D >= B) || !std::isfinite(D))
        return fail(RBF_EINVAL, "need 0 < box <= overlap, both finite (got %g, %g)", B, D);
    if (!(T == 0 || (T >= B && std::isfinite(T))))
        return fail(RBF_EINVAL, "truncation must be 0 or finite and >= box (got %g)", T);
    hipStream_t st = as_stream(stream);
    MarkOnExit mk{p, st};
    try {
        const double invB = 1.0 / B;
        const double fx = std::floor((p->xmax - p->g.x0) * invB);
        const double fy = std::floor((p->ymax - p->g.y0) * invB);
        if (!(fx < 1e9) || !(fy < 1e9) || (fx + 1) * (fy + 1) > 1e9)
            return fail(RBF_EINVAL, "box grid too large: %.0f x %.0f boxes", fx + 1, fy + 1);
        // the preconditioner of the old subdomains goes
        if (p->Z64) p->release(p->Z64, st);
        if (p->Z32) p->release(p->Z32, st);
        if (p->zoff) p->release(p->zoff, st);
        if (p->mem) p->release(p->mem, st);
        if (p->moff) p->release(p->moff, st);
        if (p->nown) p->release(p->nown, st);
        if (p->tsrc) p->release(p->tsrc, st);
        if (p->tsoff) p->release(p->tsoff, st);
        if (p->boxT) p->interactions = -1;   // counted again for the radial product
        p->tsrc = nullptr;
        p->tsoff = nullptr;
        p->boxT = false;
        p->Z64 = nullptr;
        p->Z32 = nullptr;
        p->zoff = nullptr;
        p->mem = nullptr;
        p->moff = nullptr;
        p->nown = nullptr;
        p->zoff_host.clear();
        p->geo = false;
        rbf::BoxGeometry bg;
        bg.x0 = p->g.x0;
        bg.y0 = p->g.y0;
        bg.B = B;
        bg.invB = invB;
        bg.halfD = 0.5 * D;
        bg.nbx = (int)fx + 1;
        bg.nby = (int)fy + 1;
        const long long nb = (long long)bg.nbx * bg.nby;
        int *cnt = nullptr, *own = nullptr;
        long long* moff = nullptr;
        RBF_TRY(p->alloc_n(&cnt, nb));
        RBF_TRY(p->alloc_n(&own, nb));
        RBF_TRY(p->alloc_n(&moff, nb + 1));
        rbf::PrecondArgs a = p->pc_args();
        HIP_TRY(rbf::launch_box_members(a, bg, cnt, own, nullptr, nullptr, st));
        std::vector<int> hc(nb), ho(nb);
        HIP_TRY(hipMemcpyAsync(hc.data(), cnt, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(ho.data(), own, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        std::vector<long long> off(nb + 1, 0);
        int maxo = 0, maxc = 0;
        for (long long b = 0; b < nb; ++b) {
            off[b + 1] = off[b] + hc[b];
            if (ho[b] > 0) maxo = std::max(maxo, hc[b]);
            maxc = std::max(maxc, ho[b]);
        }
        int* mem = nullptr;
        RBF_TRY(p->alloc_n(&mem, off[nb]));
        HIP_TRY(hipMemcpyAsync(moff, off.data(), sizeof(long long) * (nb + 1), hipMemcpyHostToDevice, st));
        HIP_TRY(rbf::launch_box_members(a, bg, cnt, own, moff, mem, st));
        HIP_TRY(hipStreamSynchronize(st));
        p->release(cnt, st);
        p->geo = true;
        p->bg = bg;
        p->mem = mem;
        p->moff = moff;
        p->nown = own;
        p->nsub = nb;
        p->n_omega.assign(hc.begin(), hc.end());
        p->n_c.assign(ho.begin(), ho.end());
        p->np_max = (maxo + 63) / 64 * 64;
        p->nc_max = maxc;
        if (T > 0) {   // the squares of the box truncation, listed per box
            // one 256-thread workgroup per box, at most 2^32 - 1 threads per launch
            if (nb > (1LL << 24) - 1)
                return fail(RBF_ELIMIT, "box truncation over %lld boxes (at most 2^24 - 1)", nb);
            p->halfT = 0.5 * T;
            int* ns = nullptr;
            long long* soff = nullptr;
            RBF_TRY(p->alloc_n(&ns, nb));
            RBF_TRY(p->alloc_n(&soff, nb + 1));
            rbf::BoxTrunc bt = p->bt_args();
            const rbf::MatvecArgs ma = p->mv_args();
            HIP_TRY(rbf::launch_box_square(ma, bt, ns, nullptr, st));
            std::vector<int> hs(nb);
            HIP_TRY(hipMemcpyAsync(hs.data(), ns, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            std::vector<long long> so(nb + 1, 0);
            long long pairs = 0;
            for (long long b = 0; b < nb; ++b) {
                so[b + 1] = so[b] + hs[b];
                pairs += (long long)ho[b] * hs[b];
            }
            int* src = nullptr;
            RBF_TRY(p->alloc_n(&src, so[nb]));
            HIP_TRY(hipMemcpyAsync(soff, so.data(), sizeof(long long) * (nb + 1),
                                   hipMemcpyHostToDevice, st));
            bt.src = src;
            bt.soff = soff;
            HIP_TRY(rbf::launch_box_square(ma, bt, ns, src, st));
            HIP_TRY(hipStreamSynchronize(st));
            p->release(ns, st);
            p->tsrc = src;
            p->tsoff = soff;
            p->boxT = true;
            p->interactions = pairs;
        }
        return RBF_OK;
    } catch (...) {
        return fail(RBF_ENOMEM, "host exception in rbf_set_geometry");
    }
}

rbf_status rbf_set_graphs(rbf_problem* p, int enable) {
    if (!p) return fail(RBF_EINVAL, "NULL handle");
    p->use_graphs = enable != 0;
    return RBF_OK;
}

rbf_status rbf_set_profiling(rbf_problem* p, int enable) {
    if (!p) return fail(RBF_EINVAL, "NULL handle");
    p->profiling = enable != 0;
    return RBF_OK;
}

rbf_status rbf_setup_kernel_times(const rbf_problem* p, rbf_precision precision, double* ms,
                                  int* launches) {
    if (!p || !ms || !launches) return fail(RBF_EINVAL, "NULL argument");
    if (precision != RBF_FP64 && precision != RBF_MIXED && precision != RBF_FP64_PC32)
        return fail(RBF_EINVAL, "unknown precision %d", (int)precision);
    const int pi = precision == RBF_FP64 ? 0 : 1;   // the FP64 or the FP32 local factors
    if (!p->ktimes_valid[pi]) return fail(RBF_ESTATE, "no profiled setup of this precision");
    for (int k = 0; k < RBF_K_SETUP_KINDS; ++k) {
        ms[k] = p->kms[pi][k];
        launches[k] = p->kcount[pi][k];
    }
    return RBF_OK;
}

const char* rbf_status_string(rbf_status s) {
    switch (s) {
        case RBF_OK: return "RBF_OK";
        case RBF_EINVAL: return "RBF_EINVAL";
        case RBF_EDUPLICATE: return "RBF_EDUPLICATE";
        case RBF_ENOMEM: return "RBF_ENOMEM";
        case RBF_EDEVICE: return "RBF_EDEVICE";
        case RBF_ENOTPD: return "RBF_ENOTPD";
        case RBF_ENOCONV: return "RBF_ENOCONV";
        case RBF_EBREAKDOWN: return "RBF_EBREAKDOWN";
        case RBF_ENAN: return "RBF_ENAN";
        case RBF_ESTATE: return "RBF_ESTATE";
        case RBF_ELIMIT: return "RBF_ELIMIT";
    }
    return "RBF_UNKNOWN";
}

const char* rbf_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
