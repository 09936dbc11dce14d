// boxtrunc.hip -- the box-truncated Gaussian product of the paper's subdomain
// geometry (Section 3.1, Fig. 3) on gfx950.
//
// With subdomain boxes of side B the paper truncates the product by boxes, not
// by a radius: a target keeps every source inside the square of side T
// (T >= B) centred on its own box.  All targets of a box then share one source
// set, and the product is, box by box, a dense (own points) x (square) block.
// The square's points are listed once per box at set-up (sorted-order
// indices; each row of cells under the square is one contiguous sorted range,
// so the list comes out in sorted order).  The product stages one box's
// sources in LDS and spreads the block's pairs over the lanes as 4 targets x
// 16 source phases per wave, so a box of 25 or 39 targets still keeps its
// lanes busy; each target sums its 64 phases (16 lanes x 4 waves) in a fixed
// order, so results are bit-reproducible.
#include "rbf_device.hpp"
#include "rbf_internal.hpp"

namespace rbf {

namespace {

constexpr int kBtThreads = 256;
constexpr int kBtWaves = kBtThreads / 64;
constexpr int kBtChunk = 1024;                    // sources staged at once
constexpr int kBtTargets = kBtThreads / kBtWaves;  // targets per pass: 16 groups of 4

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// floor((v - v0) * inv) clamped to [0, n - 1]: the cell rule, with the box side
__device__ __forceinline__ int axis_coord(double v, double v0, double inv, int n) {
    double t = floor((v - v0) * inv);
    if (!(t >= 0.0)) t = 0.0;
    if (t > (double)(n - 1)) t = (double)(n - 1);
    return (int)t;
}

// Count (kFill = false) or write the points of box b's square: the cells of
// the square's corners widened by one cell (rounding at its edges) and
// clamped, scanned row by row, a point taken when |x - c| <= T/2 along both
// axes, c = x0 + (b + 1/2) B the box's centre.  One wave per box.
template <bool kFill>
__global__ __launch_bounds__(kBtThreads) void k_box_square(MatvecArgs a, BoxTrunc bt,
                                                          int* __restrict__ nsrc,
                                                          int* __restrict__ src) {
    const int lane = threadIdx.x & 63;
    const long long b = (long long)blockIdx.x * kBtWaves + (threadIdx.x >> 6);
    if (b >= bt.nbox) return;
    const BoxGeometry& bg = bt.bg;
    const int bx = (int)(b % bg.nbx), by = (int)(b / bg.nbx);
    const double cx = bg.x0 + ((double)bx + 0.5) * bg.B;
    const double cy = bg.y0 + ((double)by + 0.5) * bg.B;
    const double h = bt.halfT;
    const Grid& g = a.g;
    int xa = axis_coord(cx - h, g.x0, g.invL, g.ncx) - 1;
    int xb = axis_coord(cx + h, g.x0, g.invL, g.ncx) + 1;
    int ya = axis_coord(cy - h, g.y0, g.invL, g.ncy) - 1;
    int yb = axis_coord(cy + h, g.y0, g.invL, g.ncy) + 1;
    xa = xa < 0 ? 0 : xa;
    ya = ya < 0 ? 0 : ya;
    xb = xb > g.ncx - 1 ? g.ncx - 1 : xb;
    yb = yb > g.ncy - 1 ? g.ncy - 1 : yb;
    int* out = kFill ? src + bt.soff[b] : nullptr;
    int k = 0;
    for (int ny = ya; ny <= yb; ++ny) {
        const int j0 = a.scell[ny * g.ncx + xa], j1 = a.scell[ny * g.ncx + xb + 1];
        for (int jb = j0; jb < j1; jb += 64) {
            const int j = jb + lane;
            const bool take = j < j1 && fabs(a.sx[j] - cx) <= h && fabs(a.sy[j] - cy) <= h;
            const unsigned long long m = __ballot(take);
            if (kFill && take) out[k + __popcll(m & ((1ull << lane) - 1ull))] = j;
            k += __popcll(m);
        }
    }
    if (!kFill && lane == 0) nsrc[b] = k;
}

// y at the own points of box b (one workgroup per box).  Lane l of wave v
// serves, for each group g of four targets, target 4 g + l / 16 with the
// source phase p = 16 v + l % 16: the staged sources q = p, p + 64, ...  A
// wave's 16 phases are summed by a butterfly, the waves' sums in wave order,
// chunk after chunk.  kCap: squares so wide that a pair's exponent can pass
// the exponential's range, so d2 is capped (else no pair can, and the cap is
// left out).
template <bool kCap>
__global__ __launch_bounds__(kBtThreads) void k_matvec64_box(MatvecArgs a, BoxTrunc bt,
                                                            const double* __restrict__ w,
                                                            double* __restrict__ y) {
    __shared__ double2 XY[kBtChunk];
    __shared__ double W[kBtChunk];
    __shared__ double T32[32];
    __shared__ double part[kBtWaves * kBtTargets];
    const long long b = blockIdx.x;
    const int nown = uni(bt.nown[b]);
    if (nown == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = uni(tid >> 6);
    const long long s0 = bt.soff[b];
    const int ns = uni((int)(bt.soff[b + 1] - s0));
    const int* __restrict__ own = bt.mem + (bt.moff[b + 1] - nown);
    if (tid < 32) T32[tid] = a.t32[tid];
    const int gi = lane >> 4, ph = 16 * wv + (lane & 15);
    const double beta = a.beta, d2max = bt.d2max;
    int staged = -1;   // first source of the chunk in LDS
    for (int tb = 0; tb < nown; tb += kBtTargets) {
        const int nt = min(kBtTargets, nown - tb);
        const int ng = (nt + 3) >> 2;
        part[tid] = 0.0;
        __syncthreads();
        for (int c0 = 0; c0 < ns; c0 += kBtChunk) {
            const int nc = min(kBtChunk, ns - c0);
            if (staged != c0) {
                __syncthreads();   // the previous chunk is no longer read
                for (int q = tid; q < nc; q += kBtThreads) {
                    const int s = bt.src[s0 + c0 + q];
                    XY[q] = double2{a.sx[s], a.sy[s]};
                    W[q] = w[s];
                }
                staged = c0;
                __syncthreads();
            }
            for (int g = 0; g < ng; ++g) {
                const int t = 4 * g + gi;
                const bool act = t < nt;
                const int ti = own[tb + (act ? t : 0)];
                const double xi = a.sx[ti], yi = a.sy[ti];
                double acc0 = 0.0, acc1 = 0.0;
                auto pair = [&](int q, double& acc) {
                    const double2 s = XY[q];
                    const double dx = xi - s.x, dy = yi - s.y;
                    double d2 = __builtin_fma(dx, dx, dy * dy);
                    if (kCap) d2 = __builtin_fmin(d2, d2max);
                    acc = __builtin_fma(W[q], exp2_scaled_t32(d2, beta, T32), acc);
                };
                int q = ph;
                for (; q + 64 < nc; q += 128) {
                    pair(q, acc0);
                    pair(q + 64, acc1);
                }
                if (q < nc) pair(q, acc0);
                double acc = acc0 + acc1;
                acc += __shfl_xor(acc, 8, 64);
                acc += __shfl_xor(acc, 4, 64);
                acc += __shfl_xor(acc, 2, 64);
                acc += __shfl_xor(acc, 1, 64);
                if ((lane & 15) == 0 && act) part[wv * kBtTargets + t] += acc;
            }
        }
        __syncthreads();
        if (tid < nt) {
            double s = part[tid] + part[kBtTargets + tid];
            s += part[2 * kBtTargets + tid];
            s += part[3 * kBtTargets + tid];
            y[own[tb + tid]] = s * a.norm;
        }
        __syncthreads();   // part is read before the next pass clears it
    }
}

// The same product at m arbitrary targets (tx, ty): target i takes the square
// of the box that the box rule gives its coordinates (clamped to the grid, as
// for points outside the nodes' bounding box) and sums that box's list in its
// order.  One thread per target, grid-stride.
template <bool kCount>
__global__ __launch_bounds__(kBtThreads) void k_evaluate_box(MatvecArgs a, BoxTrunc bt,
                                                            const double* __restrict__ tx,
                                                            const double* __restrict__ ty,
                                                            long long m,
                                                            const double* __restrict__ w,
                                                            double* __restrict__ y,
                                                            int* __restrict__ nnb) {
    __shared__ double T32[32];
    if (threadIdx.x < 32) T32[threadIdx.x] = a.t32[threadIdx.x];
    __syncthreads();
    const BoxGeometry& bg = bt.bg;
    const double beta = a.beta, d2max = bt.d2max;
    for (long long i = (long long)blockIdx.x * kBtThreads + threadIdx.x; i < m;
         i += (long long)gridDim.x * kBtThreads) {
        const double xi = tx[i], yi = ty[i];
        const long long bb = (long long)axis_coord(yi, bg.y0, bg.invB, bg.nby) * bg.nbx +
                             axis_coord(xi, bg.x0, bg.invB, bg.nbx);
        const long long e0 = bt.soff[bb], e1 = bt.soff[bb + 1];
        double acc = 0.0;
        for (long long e = e0; e < e1; ++e) {
            const int s = bt.src[e];
            const double dx = xi - a.sx[s], dy = yi - a.sy[s];
            const double d2 = __builtin_fmin(__builtin_fma(dx, dx, dy * dy), d2max);
            acc = __builtin_fma(w[s], exp2_scaled_t32(d2, beta, T32), acc);
        }
        y[i] = acc * a.norm;
        if (kCount) nnb[i] = (int)(e1 - e0);
    }
}

}  // namespace

hipError_t launch_box_square(const MatvecArgs& a, const BoxTrunc& bt, int* nsrc, int* src,
                             hipStream_t st) {
    if (bt.nbox == 0) return hipSuccess;
    const unsigned grid = (unsigned)((bt.nbox + kBtWaves - 1) / kBtWaves);
    if (src)
        k_box_square<true><<<grid, kBtThreads, 0, st>>>(a, bt, nsrc, src);
    else
        k_box_square<false><<<grid, kBtThreads, 0, st>>>(a, bt, nsrc, src);
    return hipGetLastError();
}

hipError_t launch_matvec64_box(const MatvecArgs& a, const BoxTrunc& bt, const double* w,
                               double* y, hipStream_t st) {
    if (bt.nbox <= 0) return hipSuccess;
    // a target lies within B/2 of its box's centre (up to rounding, taken
    // here as 1%), a source within T/2, along each axis
    const double reach = 1.01 * (0.5 * bt.bg.B + bt.halfT);
    if (2.0 * reach * reach < bt.d2max)
        k_matvec64_box<false><<<(unsigned)bt.nbox, kBtThreads, 0, st>>>(a, bt, w, y);
    else
        k_matvec64_box<true><<<(unsigned)bt.nbox, kBtThreads, 0, st>>>(a, bt, w, y);
    return hipGetLastError();
}

hipError_t launch_evaluate_box(const MatvecArgs& a, const BoxTrunc& bt, const double* tx,
                               const double* ty, long long m, const double* w, double* y,
                               int* nnb, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    const long long want = (m + kBtThreads - 1) / kBtThreads;
    const unsigned grid = (unsigned)(want < 65536 ? want : 65536);
    if (nnb)
        k_evaluate_box<true><<<grid, kBtThreads, 0, st>>>(a, bt, tx, ty, m, w, y, nnb);
    else
        k_evaluate_box<false><<<grid, kBtThreads, 0, st>>>(a, bt, tx, ty, m, w, y, nnb);
    return hipGetLastError();
}

}  // namespace rbf
