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

// ---- neighbour lists ---------------------------------------------------------

// The three row ranges of cell c's 3x3 block (sorted-order [b, e) per row,
// empty rows outside the grid) and the first cell column of each range.
struct Rows {
    int b[3], e[3], base[3];   // base: local index of the range's first source
    int n;                     // n_nb
    int xlo, cx, cy;
};

__device__ __forceinline__ Rows block_rows(const int* __restrict__ scell, const Grid& g, int c) {
    Rows r;
    const int ncx = g.ncx, ncy = g.ncy;
    r.cx = c % ncx;
    r.cy = c / ncx;
    r.xlo = r.cx > 0 ? r.cx - 1 : 0;
    const int xhi = r.cx + 1 < ncx ? r.cx + 1 : ncx - 1;
    int tot = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int ny = r.cy + d - 1;
        int b = 0, e = 0;
        if (ny >= 0 && ny < ncy) {
            b = scell[ny * ncx + r.xlo];
            e = scell[ny * ncx + xhi + 1];
        }
        r.b[d] = b;
        r.e[d] = e;
        r.base[d] = tot;
        tot += e - b;
    }
    r.n = tot;
    return r;
}

// Count (kFill = false) or write (kFill = true) each lane's in-cutoff sources;
// the decision d2 <= rc2 is the one the candidate kernel takes, bit for bit.
template <bool kFill>
__global__ __launch_bounds__(64) void k_list_build(MatvecArgs a, const int2* __restrict__ unit,
                                                   int* __restrict__ len, int* __restrict__ nb,
                                                   const long long* __restrict__ off,
                                                   unsigned short* __restrict__ idx) {
    const int u = blockIdx.x;
    const int lane = threadIdx.x;
    const int2 uc = unit[u];
    const int c = uniform(uc.x), t0 = uniform(uc.y);
    const int t1 = uniform(a.scell[c + 1]);
    const Rows r = block_rows(a.scell, a.g, c);
    const int t = t0 + lane;
    const bool act = t < t1;
    const double xi = act ? a.sx[t] : 0.0, yi = act ? a.sy[t] : 0.0;
    int cnt = 0;
    unsigned short* mine = kFill ? idx + off[u] + 4 * lane : nullptr;
    for (int d = 0; d < 3; ++d) {
        const int b = uniform(r.b[d]), e = uniform(r.e[d]), base = uniform(r.base[d]);
        for (int s = b; s < e; ++s) {
            const double dx = xi - a.sx[s], dy = yi - a.sy[s];
            const bool in = act && __builtin_fma(dx, dx, dy * dy) <= a.rc2;
            if (in) {
                if (kFill) mine[256 * (cnt >> 2) + (cnt & 3)] = (unsigned short)(base + s - b);
                ++cnt;
            }
        }
    }
    if (kFill) {
        const int L = len[u];
        for (int k = cnt; k < L; ++k) mine[256 * (k >> 2) + (k & 3)] = (unsigned short)r.n;
    } else {
        int m = cnt;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int v = __shfl_xor(m, o, 64);
            m = v > m ? v : m;
        }
        if (lane == 0) {
            len[u] = (m + 3) & ~3;
            nb[u] = r.n;
        }
    }
}

// y[t] = norm * sum over the target's list of w[s] exp(mk d2): the unit's
// sources staged in LDS as 32-byte records (x, y, w), the null source at the
// cell centre with weight 0, the exponential from a 32-entry table (also in
// LDS); four list entries per 8-byte load, loaded two loop passes ahead.
__global__ __launch_bounds__(64) void k_matvec64_lists(MatvecArgs a, NeighborLists nl,
                                                       const double* __restrict__ w,
                                                       double* __restrict__ y) {
    extern __shared__ double smem[];
    const int u = blockIdx.x;
    const int lane = threadIdx.x;
    const int2 uc = nl.unit[u];
    const int c = uniform(uc.x), t0 = uniform(uc.y);
    const int t1 = uniform(a.scell[c + 1]);
    const Rows r = block_rows(a.scell, a.g, c);
    const int n = r.n;
    double* T32 = smem;                 // 32 entries
    double4* S = reinterpret_cast<double4*>(smem + 32);
    if (lane < 32) T32[lane] = a.t32[lane];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int b = r.b[d], cnt = r.e[d] - r.b[d], base = r.base[d];
        for (int q = lane; q < cnt; q += 64)
            S[base + q] = double4{a.sx[b + q], a.sy[b + q], w[b + q], 0.0};
    }
    const double xc = a.g.x0 + (r.cx + 0.5) * a.g.L, yc = a.g.y0 + (r.cy + 0.5) * a.g.L;
    if (lane == 0) S[n] = double4{xc, yc, 0.0, 0.0};
    const int t = t0 + lane;
    const bool act = t < t1;
    const double xi = act ? a.sx[t] : xc;
    const double yi = act ? a.sy[t] : yc;
    const int L = uniform(nl.len[u]);   // multiple of 4, >= 4
    const uint2* lp = reinterpret_cast<const uint2*>(nl.idx + nl.off[u]) + lane;
    // two list registers in turn, each reloaded two passes ahead (no copies)
    uint2 qa = lp[0];
    uint2 qb = L > 4 ? lp[64] : uint2{0u, 0u};
    __syncthreads();
    double acc0 = 0.0, acc1 = 0.0;
    auto four = [&](const uint2 q4) {
        const int q[4] = {(int)(q4.x & 0xffff), (int)(q4.x >> 16), (int)(q4.y & 0xffff),
                          (int)(q4.y >> 16)};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double4 s = S[q[j]];
            const double dx = xi - s.x, dy = yi - s.y;
            const double e = exp_neg_t32(__builtin_fma(dx, dx, dy * dy) * a.mk, T32);
            if (j & 1)
                acc1 = __builtin_fma(s.z, e, acc1);
            else
                acc0 = __builtin_fma(s.z, e, acc0);
        }
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

// FP32 form: the staged sources are moved into the target cell's frame (the
// scaled cell-relative coordinates plus the cell offset), so d2 is the negated
// base-2 exponent; Kahan-compensated FP32 accumulation, FP64 output.
__global__ __launch_bounds__(64) void k_matvec32_lists(Matvec32Args a, NeighborLists nl,
                                                       const double* __restrict__ w,
                                                       double* __restrict__ y) {
    extern __shared__ double smem[];
    const int u = blockIdx.x;
    const int lane = threadIdx.x;
    const int2 uc = nl.unit[u];
    const int c = uniform(uc.x), t0 = uniform(uc.y);
    const int t1 = uniform(a.scell[c + 1]);
    const Rows r = block_rows(a.scell, a.g, c);
    const int n = r.n;
    float2* XY = reinterpret_cast<float2*>(smem);
    float* W = reinterpret_cast<float*>(smem) + 2 * (nl.max_nb + 1);
    const int ncx = a.g.ncx;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int ny = r.cy + d - 1;
        const int b = r.b[d], cnt = r.e[d] - r.b[d], base = r.base[d];
        for (int q = lane; q < cnt; q += 64) {
            const int s = b + q;
            // cell column of s within the row range
            int nx = r.xlo;
            while (nx + 1 < ncx && a.scell[ny * ncx + nx + 1] <= s) ++nx;
            XY[base + q] = float2{a.sx[s] + (float)(nx - r.cx) * a.Ls,
                                  a.sy[s] + (float)(d - 1) * a.Ls};
            W[base + q] = (float)w[s];
        }
    }
    if (lane == 0) {
        XY[n] = float2{0.f, 0.f};
        W[n] = 0.f;
    }
    const int t = t0 + lane;
    const bool act = t < t1;
    const float xi = act ? a.sx[t] : 0.f, yi = act ? a.sy[t] : 0.f;
    __syncthreads();
    const int L = uniform(nl.len[u]);   // multiple of 4, >= 4
    const uint2* lp = reinterpret_cast<const uint2*>(nl.idx + nl.off[u]) + lane;
    uint2 qa = lp[0];
    uint2 qb = L > 4 ? lp[64] : uint2{0u, 0u};
    Kahan32 acc;
    auto four = [&](const uint2 q4) {
        const int q[4] = {(int)(q4.x & 0xffff), (int)(q4.x >> 16), (int)(q4.y & 0xffff),
                          (int)(q4.y >> 16)};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float2 s = XY[q[j]];
            const float dx = xi - s.x, dy = yi - s.y;
            acc.add(W[q[j]] * exp2_f32(-__builtin_fmaf(dx, dx, dy * dy)));
        }
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

hipError_t launch_list_count(const MatvecArgs& a, const int2* unit, int nunits, int* len, int* nb,
                             hipStream_t st) {
    if (nunits > 0)
        k_list_build<false><<<nunits, 64, 0, st>>>(a, unit, len, nb, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_list_fill(const MatvecArgs& a, const int2* unit, int nunits,
                            const long long* off, const int* len, unsigned short* idx,
                            hipStream_t st) {
    if (nunits > 0)
        k_list_build<true><<<nunits, 64, 0, st>>>(a, unit, const_cast<int*>(len), nullptr, off,
                                                  idx);
    return hipGetLastError();
}

hipError_t launch_matvec64_lists(const MatvecArgs& a, const NeighborLists& nl, const double* w,
                                 double* y, hipStream_t st) {
    const size_t lds = sizeof(double) * (32 + 4 * (size_t)(nl.max_nb + 1));
    if (nl.nunits > 0) k_matvec64_lists<<<nl.nunits, 64, lds, st>>>(a, nl, w, y);
    return hipGetLastError();
}

hipError_t launch_matvec32_lists(const Matvec32Args& a, const NeighborLists& nl, const double* w,
                                 double* y, hipStream_t st) {
    const size_t lds = sizeof(float) * 3 * (size_t)(nl.max_nb + 1);
    if (nl.nunits > 0) k_matvec32_lists<<<nl.nunits, 64, lds, st>>>(a, nl, w, y);
    return hipGetLastError();
}

}  // namespace rbf
