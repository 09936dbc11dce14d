// matvec.hip -- cutoff-truncated Gaussian matrix-vector product on gfx950.
//
// y_i = (2 pi sigma^2)^-1 sum_j w_j exp(-|x_i - x_j|^2 / (2 sigma^2)) over the
// sources j with |x_i - x_j| <= r_c (the normalised Gaussian of Section 2.3 and
// its banded/truncated product).  Cells have side r_c, so every in-cutoff source
// of a target lies in the 3x3 block of cells around the target's cell, and in
// the cell-sorted order each row of three cells is one contiguous range.
//
// Two forms.  The candidate kernels (evaluation at arbitrary targets, the
// neighbour counts, and products whose 3x3 blocks are too large to stage):
// one wavefront per target cell (lanes = the cell's targets, in chunks of 64),
// cells strided over all waves of a persistent grid; the sources are
// wave-uniform, so they stream through the scalar cache into SGPRs, and the
// cutoff is a per-lane select.  The list kernels (every product of the
// solver): per-target lists of in-cutoff sources built once at setup, one
// workgroup per run of cells of one cell row, the run's neighbourhood staged
// once in LDS and only listed pairs evaluated.  Every target sums its sources
// in a fixed order (rows, then sorted order), so results are bit-reproducible.
#include "rbf_device.hpp"
#include "rbf_internal.hpp"

namespace rbf {

namespace {

constexpr int kMvThreads = 256;
constexpr int kMvWaves = kMvThreads / 64;

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

constexpr int kBatch = 8;   // sources loaded together before their 8 candidate chains

// One candidate: the cutoff is applied as a select, so the 8 chains of a batch
// carry no control flow and interleave freely.  The exponent is clamped into
// the table's range first (pairs beyond the cutoff are discarded anyway).
template <bool kTable>
__device__ __forceinline__ double pair_term(double xi, double yi, double xs, double ys, double ws,
                                            double rc2, double mk, double xlo,
                                            const double* __restrict__ T, bool* in) {
    const double dx = xi - xs, dy = yi - ys;
    const double d2 = __builtin_fma(dx, dx, dy * dy);
    *in = d2 <= rc2;
    double ex;
    if (kTable) {
        ex = exp_neg_tab(__builtin_fmax(d2 * mk, xlo), T);
    } else {
        ex = exp_neg(__builtin_fmax(d2 * mk, -700.0));
    }
    return *in ? ws * ex : 0.0;
}

template <bool kTable, bool kCount>
__global__ __launch_bounds__(kMvThreads) void k_matvec64(
    MatvecArgs a, const double* __restrict__ sx, const double* __restrict__ sy,
    const double* __restrict__ w, const int* __restrict__ scell,
    const double* __restrict__ tx, const double* __restrict__ ty, const int* __restrict__ tcell,
    double* __restrict__ y, int* __restrict__ nnb, const double* __restrict__ etab, int ntab) {
    __shared__ double T[kTable ? kExpTableMax : 1];
    if (kTable) {
        for (int k = threadIdx.x; k < ntab; k += kMvThreads) T[k] = etab[k];
        __syncthreads();
    }
    const double xlo = kTable ? -(double)(ntab - 1) * 0x1p-7 : -700.0;
    const int lane = threadIdx.x & 63;
    const int wave = uniform(threadIdx.x >> 6);
    const int ncx = a.g.ncx, ncy = a.g.ncy;
    const int ncells = ncx * ncy;
    const int nwaves = gridDim.x * kMvWaves;
    for (int c = blockIdx.x * kMvWaves + wave; c < ncells; c += nwaves) {
        const int t0 = uniform(tcell[c]), t1 = uniform(tcell[c + 1]);
        if (t0 >= t1) continue;
        const int cx = c % ncx, cy = c / ncx;
        const int xlo_c = cx > 0 ? cx - 1 : 0;
        const int xhi_c = cx + 1 < ncx ? cx + 1 : ncx - 1;
        for (int tb = t0; tb < t1; tb += 64) {
            const int i = tb + lane;
            const bool act = i < t1;
            const double xi = act ? tx[i] : 0.0, yi = act ? ty[i] : 0.0;
            double acc = 0.0;
            int cnt = 0;
            for (int ny = cy - 1; ny <= cy + 1; ++ny) {
                if (ny < 0 || ny >= ncy) continue;
                const int b = uniform(scell[ny * ncx + xlo_c]);
                const int e = uniform(scell[ny * ncx + xhi_c + 1]);
                int s = b;
                for (; s + kBatch <= e; s += kBatch) {
                    double xs[kBatch], ys[kBatch], ws[kBatch];
#pragma unroll
                    for (int k = 0; k < kBatch; ++k) {
                        xs[k] = sx[s + k];
                        ys[k] = sy[s + k];
                        ws[k] = w[s + k];
                    }
#pragma unroll
                    for (int k = 0; k < kBatch; ++k) {
                        bool in;
                        acc += pair_term<kTable>(xi, yi, xs[k], ys[k], ws[k], a.rc2, a.mk, xlo, T, &in);
                        if (kCount) cnt += in;
                    }
                }
                for (; s < e; ++s) {
                    bool in;
                    acc += pair_term<kTable>(xi, yi, sx[s], sy[s], w[s], a.rc2, a.mk, xlo, T, &in);
                    if (kCount) cnt += in;
                }
            }
            if (act) {
                y[i] = acc * a.norm;
                if (kCount) nnb[i] = cnt;
            }
        }
    }
}

__global__ __launch_bounds__(kMvThreads) void k_to_f32(const double* __restrict__ w, long long n,
                                                      float* __restrict__ w32) {
    for (long long i = (long long)blockIdx.x * kMvThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kMvThreads)
        w32[i] = (float)w[i];
}

// FP32 form: scaled cell-centre-relative coordinates (the squared scaled
// distance is directly the negated base-2 exponent), sources streamed per cell
// with the cell offset folded into the target coordinates, Kahan-compensated
// FP32 accumulation, FP64 output.
__global__ __launch_bounds__(kMvThreads) void k_matvec32(Matvec32Args a, const float* __restrict__ sx,
                                                        const float* __restrict__ sy,
                                                        const float* __restrict__ w32,
                                                        const int* __restrict__ scell,
                                                        double* __restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int wave = uniform(threadIdx.x >> 6);
    const int ncx = a.g.ncx, ncy = a.g.ncy;
    const int ncells = ncx * ncy;
    const int nwaves = gridDim.x * kMvWaves;
    for (int c = blockIdx.x * kMvWaves + wave; c < ncells; c += nwaves) {
        const int t0 = uniform(scell[c]), t1 = uniform(scell[c + 1]);
        if (t0 >= t1) continue;
        const int cx = c % ncx, cy = c / ncx;
        for (int tb = t0; tb < t1; tb += 64) {
            const int i = tb + lane;
            const bool act = i < t1;
            const float xi = act ? sx[i] : 0.f, yi = act ? sy[i] : 0.f;
            Kahan32 acc;
            for (int ny = cy - 1; ny <= cy + 1; ++ny) {
                if (ny < 0 || ny >= ncy) continue;
                const float ty = yi - (float)(ny - cy) * a.Ls;
                for (int nx = cx - 1; nx <= cx + 1; ++nx) {
                    if (nx < 0 || nx >= ncx) continue;
                    const float tx = xi - (float)(nx - cx) * a.Ls;
                    const int b = uniform(scell[ny * ncx + nx]);
                    const int e = uniform(scell[ny * ncx + nx + 1]);
                    int s = b;
                    for (; s + kBatch <= e; s += kBatch) {
                        float xs[kBatch], ys[kBatch], ws[kBatch];
#pragma unroll
                        for (int k = 0; k < kBatch; ++k) {
                            xs[k] = sx[s + k];
                            ys[k] = sy[s + k];
                            ws[k] = w32[s + k];
                        }
#pragma unroll
                        for (int k = 0; k < kBatch; ++k) {
                            const float dx = tx - xs[k], dy = ty - ys[k];
                            const float d2 = __builtin_fmaf(dx, dx, dy * dy);
                            const float ex = exp2_f32(-d2);
                            acc.add(d2 <= a.rc2s ? ws[k] * ex : 0.f);
                        }
                    }
                    for (; s < e; ++s) {
                        const float dx = tx - sx[s], dy = ty - sy[s];
                        const float d2 = __builtin_fmaf(dx, dx, dy * dy);
                        const float ex = exp2_f32(-d2);
                        acc.add(d2 <= a.rc2s ? w32[s] * ex : 0.f);
                    }
                }
            }
            if (act) y[i] = acc.value() * a.norm;
        }
    }
}

// ---- neighbour lists ---------------------------------------------------------

// The three row ranges dy = -1, 0, 1 around cell row cy, each from the column
// left of cxa to the column right of cxb (clipped to the grid): sorted-order
// [b, e) per row, empty rows outside the grid, concatenated at base.
struct Rows {
    int b[3], e[3], base[3];   // base: index of the range's first source in the concatenation
    int n;                     // sources in all three rows
};

__device__ __forceinline__ Rows span_rows(const int* __restrict__ scell, const Grid& g, int cy,
                                          int cxa, int cxb) {
    Rows r;
    const int ncx = g.ncx, ncy = g.ncy;
    const int xlo = cxa > 0 ? cxa - 1 : 0;
    const int xhi = cxb + 1 < ncx ? cxb + 1 : ncx - 1;
    int tot = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int ny = cy + d - 1;
        int b = 0, e = 0;
        if (ny >= 0 && ny < ncy) {
            b = uniform(scell[ny * ncx + xlo]);
            e = uniform(scell[ny * ncx + xhi + 1]);
        }
        r.b[d] = b;
        r.e[d] = e;
        r.base[d] = tot;
        tot += e - b;
    }
    r.n = tot;
    return r;
}

struct GroupView {
    int u0, nu, cy, cxa, cxb, t0, t1;
};
__device__ __forceinline__ GroupView load_group(const ListGroup* __restrict__ g, int i) {
    const ListGroup v = g[i];
    return GroupView{uniform(v.u0), uniform(v.nu), uniform(v.cy), uniform(v.cxa),
                     uniform(v.cxb), uniform(v.t0), uniform(v.t1)};
}

// Count (kFill = false) or write (kFill = true) each lane's in-cutoff sources:
// the group's staged rows are scanned cell by cell in local order, and a lane
// takes a source only from the three cell columns around its own target's
// cell and only if d2 <= rc2 -- the decision the candidate kernel takes, bit
// for bit, over the same 3x3 block.  One wave per unit.
template <bool kFill>
__global__ __launch_bounds__(64 * kGroupMaxUnits) void k_list_build(MatvecArgs a, NeighborLists nl,
                                                                   int* __restrict__ len,
                                                                   unsigned short* __restrict__ idx) {
    const GroupView gr = load_group(nl.group, blockIdx.x);
    const int tid = threadIdx.x, lane = tid & 63, wv = uniform(tid >> 6);
    if (wv >= gr.nu) return;
    const int u = gr.u0 + wv;
    const int ncx = a.g.ncx, ncy = a.g.ncy;
    const Rows sp = span_rows(a.scell, a.g, gr.cy, gr.cxa, gr.cxb);
    const int t = gr.t0 + 64 * wv + lane;
    const bool act = t < gr.t1;
    int cxt = gr.cxa;   // the target's cell column
    for (int nx = gr.cxa + 1; nx <= gr.cxb; ++nx)
        if (t >= a.scell[gr.cy * ncx + nx]) cxt = nx;
    const double xi = act ? a.sx[t] : 0.0, yi = act ? a.sy[t] : 0.0;
    const int xlo = gr.cxa > 0 ? gr.cxa - 1 : 0;
    const int xhi = gr.cxb + 1 < ncx ? gr.cxb + 1 : ncx - 1;
    int cnt = 0;
    unsigned short* mine = kFill ? idx + nl.off[u] + 4 * lane : nullptr;
    for (int d = 0; d < 3; ++d) {
        const int ny = gr.cy + d - 1;
        if (ny < 0 || ny >= ncy) continue;
        const int shift = sp.base[d] - sp.b[d];
        for (int nx = xlo; nx <= xhi; ++nx) {
            const bool near = act && nx >= cxt - 1 && nx <= cxt + 1;
            if (!__any(near)) continue;
            const int b = uniform(a.scell[ny * ncx + nx]), e = uniform(a.scell[ny * ncx + nx + 1]);
            for (int s = b; s < e; ++s) {
                const double dx = xi - a.sx[s], dy = yi - a.sy[s];
                const bool in = near && __builtin_fma(dx, dx, dy * dy) <= a.rc2;
                if (in) {
                    if (kFill) mine[256 * (cnt >> 2) + (cnt & 3)] = (unsigned short)(16 * (s + shift));
                    ++cnt;
                }
            }
        }
    }
    if (kFill) {
        const int L = len[u];
        for (int k = cnt; k < L; ++k) mine[256 * (k >> 2) + (k & 3)] = (unsigned short)(16 * sp.n);
    } else {
        int m = cnt;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int v = __shfl_xor(m, o, 64);
            m = v > m ? v : m;
        }
        if (lane == 0) len[u] = (m + 3) & ~3;
    }
}

// LDS layout of the FP64 list matvec (a static allocation, so every address
// offset is a compile-time constant): the staged weights W[q] at byte 8 q, the
// coordinates (x, y)[q] at byte kXYBase + 16 q, so a list entry e = 16 q
// addresses both (e / 2 and e + kXYBase; consecutive sources fall on distinct
// banks in both arrays), then the 32-entry exponential table.
constexpr int kXYBase = 8 * (kGroupSpan + 1);
// FP32 form: (x, y)[q] as float2 at byte 8 q (e / 2), w[q] at kW32Base + 4 q (e / 4).
constexpr int kW32Base = 8 * (kGroupSpan + 1);

// y[t] = norm * sum over the target's list of w[s] 2^(beta d2 / 32).  One
// workgroup per group, one wave per unit; the null source (weight 0) sits at
// the middle of the group; four list entries per 8-byte load, loaded two loop
// passes ahead.
constexpr int kMv64Lds = kXYBase + 16 * (kGroupSpan + 1) + 256;

__device__ __forceinline__ void mv64_lists_group(MatvecArgs a, NeighborLists nl,
                                                 const double* __restrict__ w,
                                                 double* __restrict__ y, int gi, char* lds) {
    const GroupView gr = load_group(nl.group, gi);
    const int tid = threadIdx.x, lane = tid & 63, wv = uniform(tid >> 6);
    const Rows r = span_rows(a.scell, a.g, gr.cy, gr.cxa, gr.cxb);
    const int n = r.n;
    double* W = reinterpret_cast<double*>(lds);
    double2* XY = reinterpret_cast<double2*>(lds + kXYBase);
    double* T32 = reinterpret_cast<double*>(lds + kXYBase + 16 * (kGroupSpan + 1));
    if (tid < 32) T32[tid] = a.t32[tid];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int b = r.b[d], cnt = r.e[d] - r.b[d], base = r.base[d];
        for (int q = tid; q < cnt; q += blockDim.x) {
            XY[base + q] = double2{a.sx[b + q], a.sy[b + q]};
            W[base + q] = w[b + q];
        }
    }
    const double xm = a.g.x0 + (0.5 * (gr.cxa + gr.cxb) + 0.5) * a.g.L;
    const double ym = a.g.y0 + (gr.cy + 0.5) * a.g.L;
    if (tid == 0) {
        XY[n] = double2{xm, ym};
        W[n] = 0.0;
    }
    __syncthreads();
    if (wv >= gr.nu) return;
    const int u = gr.u0 + wv;
    const int t = gr.t0 + 64 * wv + lane;
    const bool act = t < gr.t1;
    const double xi = act ? a.sx[t] : xm;
    const double yi = act ? a.sy[t] : ym;
    const int L = uniform(nl.len[u]);   // multiple of 4, >= 4
    const uint2* lp = reinterpret_cast<const uint2*>(nl.idx + nl.off[u]) + lane;
    // two list registers in turn, each reloaded two passes ahead (no copies)
    uint2 qa = lp[0];
    uint2 qb = L > 4 ? lp[64] : uint2{0u, 0u};
    const double beta = a.beta;
    double acc0 = 0.0, acc1 = 0.0;
    auto pair = [&](unsigned exy, unsigned ew, double& acc) {
        const double2 s = *reinterpret_cast<const double2*>(lds + kXYBase + exy);
        const double ws = *reinterpret_cast<const double*>(lds + ew);
        const double dx = xi - s.x, dy = yi - s.y;
        const double e = exp2_scaled_t32(__builtin_fma(dx, dx, dy * dy), beta, T32);
        acc = __builtin_fma(ws, e, acc);
    };
    auto four = [&](const uint2 q4) {
        pair(q4.x & 0xffffu, (q4.x >> 1) & 0x7fffu, acc0);
        pair(q4.x >> 16, q4.x >> 17, acc1);
        pair(q4.y & 0xffffu, (q4.y >> 1) & 0x7fffu, acc0);
        pair(q4.y >> 16, q4.y >> 17, acc1);
    };
    for (int k = 0; k < L; k += 8) {
        four(qa);
        if (k + 8 < L) qa = lp[64 * (k / 4 + 2)];
        if (k + 4 < L) {
            four(qb);
            if (k + 12 < L) qb = lp[64 * (k / 4 + 3)];
        }
    }
    if (act) y[t] = (acc0 + acc1) * a.norm;
}

__global__ __launch_bounds__(64 * kGroupMaxUnits) void k_matvec64_lists(MatvecArgs a,
                                                                       NeighborLists nl,
                                                                       const double* __restrict__ w,
                                                                       double* __restrict__ y) {
    __shared__ __attribute__((aligned(16))) char lds[kMv64Lds];
    mv64_lists_group(a, nl, w, y, blockIdx.x, lds);
}

// FP32 form: the group's sources are staged in one frame centred on the group
// (scaled coordinates: the cell-centre-relative FP32 ones plus the cell offset,
// summed in FP64 and rounded once), so d2 is the negated base-2 exponent;
// Kahan-compensated FP32 accumulation, FP64 output.
constexpr int kMv32Lds = kW32Base + 4 * (kGroupSpan + 1);

__device__ __forceinline__ void mv32_lists_group(Matvec32Args a, NeighborLists nl,
                                                 const double* __restrict__ w,
                                                 double* __restrict__ y, int gi, char* lds) {
    const GroupView gr = load_group(nl.group, gi);
    const int tid = threadIdx.x, lane = tid & 63, wv = uniform(tid >> 6);
    const Rows r = span_rows(a.scell, a.g, gr.cy, gr.cxa, gr.cxb);
    const int n = r.n;
    float2* XY = reinterpret_cast<float2*>(lds);
    float* W = reinterpret_cast<float*>(lds + kW32Base);
    const int ncx = a.g.ncx;
    const double mid = 0.5 * (gr.cxa + gr.cxb);
    const double Ls = (double)a.Ls;
    const int xlo = gr.cxa > 0 ? gr.cxa - 1 : 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int ny = gr.cy + d - 1;
        const int b = r.b[d], cnt = r.e[d] - r.b[d], base = r.base[d];
        for (int q = tid; q < cnt; q += blockDim.x) {
            const int s = b + q;
            // cell column of s within the row range
            int nx = xlo;
            while (nx + 1 < ncx && a.scell[ny * ncx + nx + 1] <= s) ++nx;
            XY[base + q] = float2{(float)((double)a.sx[s] + (nx - mid) * Ls),
                                  (float)((double)a.sy[s] + (double)(d - 1) * Ls)};
            W[base + q] = (float)w[s];
        }
    }
    if (tid == 0) {
        XY[n] = float2{0.f, 0.f};
        W[n] = 0.f;
    }
    __syncthreads();
    if (wv >= gr.nu) return;
    const int u = gr.u0 + wv;
    const int t = gr.t0 + 64 * wv + lane;
    const bool act = t < gr.t1;
    int cxt = gr.cxa;   // the target's cell column
    for (int nx = gr.cxa + 1; nx <= gr.cxb; ++nx)
        if (t >= a.scell[gr.cy * ncx + nx]) cxt = nx;
    const float xi = act ? (float)((double)a.sx[t] + (cxt - mid) * Ls) : 0.f;
    const float yi = act ? a.sy[t] : 0.f;
    const int L = uniform(nl.len[u]);   // multiple of 4, >= 4
    const uint2* lp = reinterpret_cast<const uint2*>(nl.idx + nl.off[u]) + lane;
    uint2 qa = lp[0];
    uint2 qb = L > 4 ? lp[64] : uint2{0u, 0u};
    Kahan32 acc;
    auto pair = [&](unsigned exy, unsigned ew) {
        const float2 s = *reinterpret_cast<const float2*>(lds + exy);
        const float ws = *reinterpret_cast<const float*>(lds + kW32Base + ew);
        const float dx = xi - s.x, dy = yi - s.y;
        acc.add(ws * exp2_f32(-__builtin_fmaf(dx, dx, dy * dy)));
    };
    auto four = [&](const uint2 q4) {
        pair((q4.x >> 1) & 0x7fffu, (q4.x >> 2) & 0x3fffu);
        pair(q4.x >> 17, q4.x >> 18);
        pair((q4.y >> 1) & 0x7fffu, (q4.y >> 2) & 0x3fffu);
        pair(q4.y >> 17, q4.y >> 18);
    };
    for (int k = 0; k < L; k += 8) {
        four(qa);
        if (k + 8 < L) qa = lp[64 * (k / 4 + 2)];
        if (k + 4 < L) {
            four(qb);
            if (k + 12 < L) qb = lp[64 * (k / 4 + 3)];
        }
    }
    if (act) y[t] = acc.value() * a.norm;
}

__global__ __launch_bounds__(64 * kGroupMaxUnits) void k_matvec32_lists(Matvec32Args a,
                                                                       NeighborLists nl,
                                                                       const double* __restrict__ w,
                                                                       double* __restrict__ y) {
    __shared__ __attribute__((aligned(16))) char lds[kMv32Lds];
    mv32_lists_group(a, nl, w, y, blockIdx.x, lds);
}

// Packed form: workgroup b serves group b - block0[j] of job j (FP64 or FP32
// lists by the job), with the staging sized for the FP64 form.
__device__ __forceinline__ int find_job_mv(const int* __restrict__ block0, int njobs, int b) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (block0[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(64 * kGroupMaxUnits) void k_matvec_lists_packed(
    const MatvecJob* __restrict__ jobs, const int* __restrict__ block0, int njobs) {
    static_assert(kMv64Lds >= kMv32Lds, "the FP64 staging is the larger");
    __shared__ __attribute__((aligned(16))) char lds[kMv64Lds];
    const int j = uniform(find_job_mv(block0, njobs, blockIdx.x));
    const MatvecJob& J = jobs[j];
    const int gi = blockIdx.x - block0[j];
    if (J.skip) return;
    if (J.prec == 0)
        mv64_lists_group(J.a, J.nl, J.w, J.y, gi, lds);
    else
        mv32_lists_group(J.a32, J.nl, J.w, J.y, gi, lds);
}

inline unsigned mv_grid(long long ncells) {
    long long b = (ncells + kMvWaves - 1) / kMvWaves;
    return (unsigned)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

}  // namespace

hipError_t launch_matvec64(const MatvecArgs& a, const double* w, double* y, int* nnb,
                           hipStream_t st) {
    const unsigned grid = mv_grid(a.g.ncells());
    const bool tab = a.etab != nullptr && a.ntab <= kExpTableMax;
    if (nnb) {
        if (tab)
            k_matvec64<true, true><<<grid, kMvThreads, 0, st>>>(a, a.sx, a.sy, w, a.scell, a.tx, a.ty,
                                                                a.tcell, y, nnb, a.etab, a.ntab);
        else
            k_matvec64<false, true><<<grid, kMvThreads, 0, st>>>(a, a.sx, a.sy, w, a.scell, a.tx,
                                                                 a.ty, a.tcell, y, nnb, nullptr, 0);
    } else {
        if (tab)
            k_matvec64<true, false><<<grid, kMvThreads, 0, st>>>(a, a.sx, a.sy, w, a.scell, a.tx,
                                                                 a.ty, a.tcell, y, nullptr, a.etab,
                                                                 a.ntab);
        else
            k_matvec64<false, false><<<grid, kMvThreads, 0, st>>>(a, a.sx, a.sy, w, a.scell, a.tx,
                                                                  a.ty, a.tcell, y, nullptr, nullptr,
                                                                  0);
    }
    return hipGetLastError();
}

hipError_t launch_matvec32(const Matvec32Args& a, const double* w, float* w32, double* y,
                           long long n, hipStream_t st) {
    long long nb = (n + kMvThreads - 1) / kMvThreads;
    k_to_f32<<<(unsigned)(nb < 4096 ? (nb > 0 ? nb : 1) : 4096), kMvThreads, 0, st>>>(w, n, w32);
    k_matvec32<<<mv_grid(a.g.ncells()), kMvThreads, 0, st>>>(a, a.sx, a.sy, w32, a.scell, y);
    return hipGetLastError();
}

hipError_t launch_list_count(const MatvecArgs& a, const NeighborLists& nl, int* len,
                             hipStream_t st) {
    if (nl.ngroups > 0)
        k_list_build<false><<<nl.ngroups, 64 * nl.gunits, 0, st>>>(a, nl, len, nullptr);
    return hipGetLastError();
}

hipError_t launch_list_fill(const MatvecArgs& a, const NeighborLists& nl, unsigned short* idx,
                            hipStream_t st) {
    if (nl.ngroups > 0)
        k_list_build<true><<<nl.ngroups, 64 * nl.gunits, 0, st>>>(a, nl, const_cast<int*>(nl.len),
                                                                   idx);
    return hipGetLastError();
}

hipError_t launch_matvec64_lists(const MatvecArgs& a, const NeighborLists& nl, const double* w,
                                 double* y, hipStream_t st) {
    if (nl.ngroups > 0) k_matvec64_lists<<<nl.ngroups, 64 * nl.gunits, 0, st>>>(a, nl, w, y);
    return hipGetLastError();
}

hipError_t launch_matvec_lists_packed(const MatvecJob* jobs, const int* block0, int njobs,
                                      int nblocks, int threads, hipStream_t st) {
    if (njobs > 0 && nblocks > 0)
        k_matvec_lists_packed<<<nblocks, threads, 0, st>>>(jobs, block0, njobs);
    return hipGetLastError();
}

hipError_t launch_matvec32_lists(const Matvec32Args& a, const NeighborLists& nl, const double* w,
                                 double* y, hipStream_t st) {
    if (nl.ngroups > 0) k_matvec32_lists<<<nl.ngroups, 64 * nl.gunits, 0, st>>>(a, nl, w, y);
    return hipGetLastError();
}

}  // namespace rbf
