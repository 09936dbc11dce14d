// matvec.hip -- cutoff-truncated Gaussian matrix-vector product on gfx950.
//
// y_i = (2 pi sigma^2)^-1 sum_j w_j exp(-|x_i - x_j|^2 / (2 sigma^2)) over the
// sources j with |x_i - x_j| <= r_c (the normalised Gaussian of Section 2.3 and
// its banded/truncated product).  Cells have side r_c, so every in-cutoff source
// of a target lies in the 3x3 block of cells around the target's cell, and in
// the cell-sorted order each of the three rows of that block is one contiguous
// range: sources are read with coalesced loads, staged in LDS, and broadcast to
// a wavefront whose lanes are the targets of one cell.  Every target sums its
// sources in a fixed order (rows, then sorted order), so the result is
// bit-reproducible.
#include "rbf_device.hpp"
#include "rbf_internal.hpp"

namespace rbf {

namespace {

constexpr int kMvCap = 640;   // sources staged in LDS per pass

struct Rows {
    int b[3], e[3];
    int nr, tot;
};

__device__ __forceinline__ Rows source_rows(const int* __restrict__ scell, const Grid& g,
                                            int cx, int cy) {
    Rows r;
    r.nr = 0;
    r.tot = 0;
    int xlo = cx > 0 ? cx - 1 : 0;
    int xhi = cx + 1 < g.ncx ? cx + 1 : g.ncx - 1;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        int ny = cy + dy;
        if (ny < 0 || ny >= g.ncy) continue;
        int b = scell[ny * g.ncx + xlo], e = scell[ny * g.ncx + xhi + 1];
        r.b[r.nr] = b;
        r.e[r.nr] = e;
        r.tot += e - b;
        ++r.nr;
    }
    return r;
}

// q-th source of the concatenated rows
__device__ __forceinline__ int row_source(const Rows& r, int q) {
    int l0 = r.e[0] - r.b[0];
    if (q < l0) return r.b[0] + q;
    q -= l0;
    int l1 = r.nr > 1 ? r.e[1] - r.b[1] : 0;
    if (q < l1) return r.b[1] + q;
    return r.b[2] + (q - l1);
}

template <bool COUNT>
__global__ __launch_bounds__(64) void k_matvec64(MatvecArgs a, const double* __restrict__ w,
                                                 double* __restrict__ y, int* __restrict__ nnb) {
    __shared__ double sx[kMvCap], sy[kMvCap], sw[kMvCap];
    const int c = blockIdx.x;
    const int cx = c % a.g.ncx, cy = c / a.g.ncx;
    const int t0 = a.tcell[c], t1 = a.tcell[c + 1];
    if (t0 >= t1) return;
    const Rows r = source_rows(a.scell, a.g, cx, cy);
    for (int tb = t0; tb < t1; tb += 64) {
        const int i = tb + (int)threadIdx.x;
        const bool act = i < t1;
        const double xi = act ? a.tx[i] : 0.0, yi = act ? a.ty[i] : 0.0;
        double acc = 0.0;
        int cnt = 0;
        for (int base = 0; base < r.tot; base += kMvCap) {
            const int m = r.tot - base < kMvCap ? r.tot - base : kMvCap;
            __syncthreads();
            for (int k = threadIdx.x; k < m; k += 64) {
                int s = row_source(r, base + k);
                sx[k] = a.sx[s];
                sy[k] = a.sy[s];
                sw[k] = w[s];
            }
            __syncthreads();
            for (int k = 0; k < m; ++k) {
                double dx = xi - sx[k], dy = yi - sy[k];
                double d2 = __builtin_fma(dx, dx, dy * dy);
                if (d2 <= a.rc2) {
                    acc = __builtin_fma(sw[k], exp_neg(d2 * a.mk), acc);
                    if (COUNT) ++cnt;
                }
            }
        }
        if (act) {
            y[i] = acc * a.norm;
            if (COUNT) nnb[i] = cnt;
        }
    }
}

// FP32 form: scaled cell-centre-relative coordinates, the squared scaled
// distance is directly the negated base-2 exponent; Kahan FP32 accumulation.
__global__ __launch_bounds__(64) void k_matvec32(Matvec32Args a, const double* __restrict__ w,
                                                 double* __restrict__ y) {
    constexpr int kCap = 2 * kMvCap;
    __shared__ float sx[kCap], sy[kCap], sw[kCap];
    const int c = blockIdx.x;
    const int cx = c % a.g.ncx, cy = c / a.g.ncx;
    const int t0 = a.scell[c], t1 = a.scell[c + 1];
    if (t0 >= t1) return;
    const Rows r = source_rows(a.scell, a.g, cx, cy);
    const int xlo = cx > 0 ? cx - 1 : 0;
    int rowy[3], k = 0;
    for (int dy = -1; dy <= 1; ++dy)
        if (cy + dy >= 0 && cy + dy < a.g.ncy) rowy[k++] = cy + dy;
    for (int tb = t0; tb < t1; tb += 64) {
        const int i = tb + (int)threadIdx.x;
        const bool act = i < t1;
        const float xi = act ? a.sx[i] : 0.f, yi = act ? a.sy[i] : 0.f;
        Kahan32 acc;
        for (int base = 0; base < r.tot; base += kCap) {
            const int m = r.tot - base < kCap ? r.tot - base : kCap;
            __syncthreads();
            for (int q = threadIdx.x; q < m; q += 64) {
                // locate the row and the cell of the q-th source to shift it into
                // the frame of the target cell
                int qq = base + q, ri = 0;
                while (qq >= r.e[ri] - r.b[ri]) {
                    qq -= r.e[ri] - r.b[ri];
                    ++ri;
                }
                int s = r.b[ri] + qq;
                int ny = rowy[ri];
                int scx = xlo;
                while (a.scell[ny * a.g.ncx + scx + 1] <= s) ++scx;
                sx[q] = a.sx[s] + (float)(scx - cx) * a.Ls;
                sy[q] = a.sy[s] + (float)(ny - cy) * a.Ls;
                sw[q] = (float)w[s];
            }
            __syncthreads();
            for (int q = 0; q < m; ++q) {
                float dx = xi - sx[q], dy = yi - sy[q];
                float d2 = __builtin_fmaf(dx, dx, dy * dy);
                if (d2 <= a.rc2s) acc.add(sw[q] * exp2_f32(-d2));
            }
        }
        if (act) y[i] = acc.value() * a.norm;
    }
}

}  // namespace

hipError_t launch_matvec64(const MatvecArgs& a, const double* w, double* y, int* nnb,
                           hipStream_t st) {
    unsigned grid = (unsigned)a.g.ncells();
    if (nnb)
        k_matvec64<true><<<grid, 64, 0, st>>>(a, w, y, nnb);
    else
        k_matvec64<false><<<grid, 64, 0, st>>>(a, w, y, nullptr);
    return hipGetLastError();
}

hipError_t launch_matvec32(const Matvec32Args& a, const double* w, double* y,
                           hipStream_t st) {
    unsigned grid = (unsigned)a.g.ncells();
    k_matvec32<<<grid, 64, 0, st>>>(a, w, y);
    return hipGetLastError();
}

}  // namespace rbf
