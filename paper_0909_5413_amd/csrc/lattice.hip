// lattice.hip -- the interpolant on a regular lattice of targets (remeshing
// onto a lattice, the use that motivates the method: Sections 1 and 5) on gfx950.
//
// Targets t(a, b) = (x0 + a hx, y0 + b hy).  The lattice's columns (rows) are
// grouped by the cell column (row) that the cell rule gives their coordinate,
// and cut into chunks of at most 8; one wave serves the 8 x 8 targets of a
// (column chunk, row chunk) pair, which all lie in one cell and so share its
// 3x3 block of sources -- the same candidates, in the same order, as for any
// single target of that cell.  The Gaussian factorises along the axes,
// exp(-(dx^2 + dy^2) / (2 sigma^2)) = exp(-dx^2 / (2 sigma^2)) exp(-dy^2 / (2 sigma^2)),
// and dx depends only on the target's column, dy only on its row, so per batch
// of 8 sources the wave evaluates 8 x 8 column factors and 8 x 8 row factors
// (one exponential per lane for each) instead of 8 x 64 pair exponentials, and
// each pair costs two fused multiply-adds, a compare and a select.  The cutoff
// decision is the one of every other product, fma(dx, dx, dy*dy) <= r_c^2 with
// dy*dy rounded first, so the in-cutoff sets are exactly the oracle's.
#include "rbf_device.hpp"
#include "rbf_internal.hpp"

namespace rbf {

namespace {

constexpr int kLatThreads = 64;   // one wave per (column chunk, row chunk)

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Per batch of 8 sources, the factors the pair phase reads: for column k and
// source q, (dx, w exp(-dx^2 / (2 sigma^2))) at C[q][k]; for row k, (dy^2,
// exp(-dy^2 / (2 sigma^2))) at R[q][k].  A source past the row's end has
// dx = 1e300 (its d2 overflows to +inf, outside every cutoff) and weight 0.
__global__ __launch_bounds__(kLatThreads) void k_evaluate_lattice(MatvecArgs a, LatticeArgs L,
                                                                 const double* __restrict__ w,
                                                                 double* __restrict__ out) {
    __shared__ double2 C[kLatticeChunk][kLatticeChunk];
    __shared__ double2 R[kLatticeChunk][kLatticeChunk];
    __shared__ double T32[32];
    const int lane = threadIdx.x;
    if (lane < 32) T32[lane] = a.t32[lane];
    const int ci = (int)(blockIdx.x % (unsigned)L.ncol), ri = (int)(blockIdx.x / (unsigned)L.ncol);
    const LatticeChunk cc = L.col[ci], rr = L.row[ri];
    const int ncol = uni(cc.nt), nrow = uni(rr.nt);
    const int cx = uni(cc.c), cy = uni(rr.c);
    // factor phase: lane = (k, q), column / row k of the chunk, source q of the batch
    const int k = lane & 7, q = lane >> 3;
    const double txk = L.x0 + (double)(cc.t0 + (k < ncol ? k : ncol - 1)) * L.hx;
    const double tyk = L.y0 + (double)(rr.t0 + (k < nrow ? k : nrow - 1)) * L.hy;
    // pair phase: lane = (ta, tb), the target of column ta and row tb
    const int ta = lane & 7, tb = lane >> 3;
    const double beta = a.beta, rc2 = a.rc2;
    const int ncx = a.g.ncx, ncy = a.g.ncy;
    const int xlo = cx > 0 ? cx - 1 : 0;
    const int xhi = cx + 1 < ncx ? cx + 1 : ncx - 1;
    double acc = 0.0;
    for (int ny = cy - 1; ny <= cy + 1; ++ny) {
        if (ny < 0 || ny >= ncy) continue;
        const int b = uni(a.scell[ny * ncx + xlo]), e = uni(a.scell[ny * ncx + xhi + 1]);
        for (int s0 = b; s0 < e; s0 += kLatticeChunk) {
            const int s = s0 + q;
            const bool valid = s < e;
            const int sv = valid ? s : b;
            const double dx = txk - a.sx[sv], dy = tyk - a.sy[sv];
            const double dy2 = dy * dy;
            const double ex = exp2_scaled_t32(dx * dx, beta, T32);
            const double ey = exp2_scaled_t32(dy2, beta, T32);
            const double wex = w[sv] * ex;
            __syncthreads();   // the previous batch's factors are read
            C[q][k] = double2{valid ? dx : 1e300, valid ? wex : 0.0};
            R[q][k] = double2{dy2, ey};
            __syncthreads();
#pragma unroll
            for (int p = 0; p < kLatticeChunk; ++p) {
                const double2 cf = C[p][ta];
                const double2 rf = R[p][tb];
                const double d2 = __builtin_fma(cf.x, cf.x, rf.x);
                const double nv = __builtin_fma(cf.y, rf.y, acc);
                acc = d2 <= rc2 ? nv : acc;
            }
        }
    }
    if (ta < ncol && tb < nrow) out[(rr.t0 + tb) * L.nx + cc.t0 + ta] = acc * a.norm;
}

// tx[i], ty[i] of lattice target i = b nx + a (for products that take target arrays)
__global__ __launch_bounds__(256) void k_lattice_points(LatticeArgs L, long long ny,
                                                       double* __restrict__ tx,
                                                       double* __restrict__ ty) {
    const long long m = L.nx * ny;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < m;
         i += (long long)gridDim.x * 256) {
        const long long bb = i / L.nx, aa = i - bb * L.nx;
        tx[i] = L.x0 + (double)aa * L.hx;
        ty[i] = L.y0 + (double)bb * L.hy;
    }
}

}  // namespace

hipError_t launch_evaluate_lattice(const MatvecArgs& a, const LatticeArgs& L, const double* w,
                                   double* out, hipStream_t st) {
    const long long blocks = (long long)L.ncol * L.nrow;
    if (blocks > 0)
        k_evaluate_lattice<<<(unsigned)blocks, kLatThreads, 0, st>>>(a, L, w, out);
    return hipGetLastError();
}

hipError_t launch_lattice_points(const LatticeArgs& L, long long ny, double* tx, double* ty,
                                 hipStream_t st) {
    const long long m = L.nx * ny;
    if (m <= 0) return hipSuccess;
    const long long want = (m + 255) / 256;
    k_lattice_points<<<(unsigned)(want < 65536 ? want : 65536), 256, 0, st>>>(L, ny, tx, ty);
    return hipGetLastError();
}

}  // namespace rbf
