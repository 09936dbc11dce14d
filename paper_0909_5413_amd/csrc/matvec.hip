// matvec.hip -- cutoff-truncated Gaussian matrix-vector product on gfx950.
//
// y_i = (2 pi sigma^2)^-1 sum_j w_j exp(-|x_i - x_j|^2 / (2 sigma^2)) over the
// sources j with |x_i - x_j| <= r_c (the normalised Gaussian of Section 2.3 and
// its banded/truncated product).  Cells have side r_c, so every in-cutoff source
// of a target lies in the 3x3 block of cells around the target's cell, and in
// the cell-sorted order each row of three cells is one contiguous range.
//
// Mapping: one wavefront per target cell (lanes = the cell's targets, in chunks
// of 64), cells strided over all waves of a persistent grid.  The sources are
// wave-uniform, so they stream through the scalar cache into SGPRs (no LDS
// staging, no broadcast reads); the per-lane work is the distance, the cutoff
// test and the exponential.  The FP64 exponential reads a table of
// e^{-n/128} kept in LDS (one copy per workgroup).  Every target sums its
// sources in a fixed order (rows, then sorted order), so results are
// bit-reproducible.
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

}  // namespace rbf
