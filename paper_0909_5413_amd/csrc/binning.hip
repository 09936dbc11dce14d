// binning.hip -- cell binning of the points on gfx950.
//
// The points are binned into square cells of side L = cutoff anchored at the
// minimum corner of the point set (the non-overlapping subdomains of the
// paper's domain decomposition, Section 2.2, Fig. 1), then sorted by
// (cell, original index) so that every cell, and every row of three
// neighbouring cells, is one contiguous range of the sorted arrays.
//
// Pipeline: min/max reduction -> (host computes the grid) -> cell index and
// arrival slot (integer atomics) -> exclusive scan of the counts -> scatter by
// slot -> per-cell sort of original indices (restores the stable order the
// atomics scrambled, so the result is deterministic) -> gather of coordinates.
#include "rbf_device.hpp"
#include "rbf_internal.hpp"

namespace rbf {

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_minmax(const double* __restrict__ pts,
                                                   const double* __restrict__ vals,
                                                   long long n, double* __restrict__ work,
                                                   int* __restrict__ bad) {
    __shared__ double s[4][kBlock];
    double xmin = __builtin_inf(), ymin = __builtin_inf();
    double xmax = -__builtin_inf(), ymax = -__builtin_inf();
    int nonfinite = 0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        double x = pts[2 * i], y = pts[2 * i + 1];
        double f = vals ? vals[i] : 0.0;
        if (!__builtin_isfinite(x) || !__builtin_isfinite(y) || !__builtin_isfinite(f)) {
            nonfinite = 1;
            continue;
        }
        xmin = fmin(xmin, x);
        xmax = fmax(xmax, x);
        ymin = fmin(ymin, y);
        ymax = fmax(ymax, y);
    }
    if (nonfinite) atomicOr(bad, 1);
    s[0][threadIdx.x] = xmin;
    s[1][threadIdx.x] = ymin;
    s[2][threadIdx.x] = xmax;
    s[3][threadIdx.x] = ymax;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + o]);
            s[1][threadIdx.x] = fmin(s[1][threadIdx.x], s[1][threadIdx.x + o]);
            s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + o]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) work[4 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(kBlock) void k_minmax_final(const double* __restrict__ work,
                                                         int nb, double* __restrict__ out4) {
    __shared__ double s[4][kBlock];
    double v[4] = {__builtin_inf(), __builtin_inf(), -__builtin_inf(), -__builtin_inf()};
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        v[0] = fmin(v[0], work[4 * b + 0]);
        v[1] = fmin(v[1], work[4 * b + 1]);
        v[2] = fmax(v[2], work[4 * b + 2]);
        v[3] = fmax(v[3], work[4 * b + 3]);
    }
    for (int k = 0; k < 4; ++k) s[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + o]);
            s[1][threadIdx.x] = fmin(s[1][threadIdx.x], s[1][threadIdx.x + o]);
            s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + o]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) out4[threadIdx.x] = s[threadIdx.x][0];
}

// cell coordinate floor((v - v0) * invL) clamped to [0, nc - 1]; the product is
// rounded once, exactly as the oracle computes it.
__device__ __forceinline__ int cell_coord(double v, double v0, double invL, int nc) {
    double t = floor((v - v0) * invL);
    if (!(t >= 0.0)) t = 0.0;
    if (t > (double)(nc - 1)) t = (double)(nc - 1);
    return (int)t;
}

__global__ __launch_bounds__(kBlock) void k_cell_count(const double* __restrict__ pts,
                                                       long long n, Grid g,
                                                       int* __restrict__ cell_of,
                                                       int* __restrict__ slot,
                                                       int* __restrict__ counts) {
    long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int cx = cell_coord(pts[2 * i], g.x0, g.invL, g.ncx);
    int cy = cell_coord(pts[2 * i + 1], g.y0, g.invL, g.ncy);
    int c = cy * g.ncx + cx;
    cell_of[i] = c;
    slot[i] = atomicAdd(&counts[c], 1);
}

// ---- exclusive scan: per-block sums, scan of the sums, per-block scan --------
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;   // 1024 elements per block

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int* total) {
    // Hillis-Steele over the block in shared memory
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        int t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int incl = sh[threadIdx.x];
    *total = sh[kBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_tile_sums(const int* __restrict__ in,
                                                           long long n, int* __restrict__ sums) {
    __shared__ int sh[kBlock];
    long long base = (long long)blockIdx.x * kScanTile;
    int v = 0;
    for (int k = 0; k < kScanItems; ++k) {
        long long i = base + (long long)threadIdx.x * kScanItems + k;
        if (i < n) v += in[i];
    }
    int total;
    block_exclusive_scan(v, sh, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// one block scans all tile sums in place (exclusive), carrying across chunks
__global__ __launch_bounds__(kBlock) void k_scan_sums(int* __restrict__ sums, long long nt) {
    __shared__ int sh[kBlock];
    int carry = 0;
    for (long long b = 0; b < nt; b += kBlock) {
        long long i = b + threadIdx.x;
        int v = i < nt ? sums[i] : 0;
        int total;
        int ex = block_exclusive_scan(v, sh, &total);
        if (i < nt) sums[i] = ex + carry;
        carry += total;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_tiles(const int* __restrict__ in, long long n,
                                                       const int* __restrict__ sums,
                                                       int* __restrict__ out) {
    __shared__ int sh[kBlock];
    long long base = (long long)blockIdx.x * kScanTile;
    int v[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        long long i = base + (long long)threadIdx.x * kScanItems + k;
        v[k] = i < n ? in[i] : 0;
        s += v[k];
    }
    int total;
    int ex = block_exclusive_scan(s, sh, &total) + sums[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        long long i = base + (long long)threadIdx.x * kScanItems + k;
        if (i < n) out[i] = ex;
        ex += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) out[n] = ex;
}

__global__ __launch_bounds__(kBlock) void k_scatter(const int* __restrict__ cell_of,
                                                    const int* __restrict__ slot,
                                                    const int* __restrict__ cell_start,
                                                    long long n, int* __restrict__ tmp) {
    long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    tmp[cell_start[cell_of[i]] + slot[i]] = (int)i;
}

// One wave per cell: rank sort of the cell's original indices in LDS (the
// indices are distinct, so rank = number of smaller indices).
constexpr int kSortCap = 1536;
__global__ __launch_bounds__(64) void k_sort_cells(const int* __restrict__ tmp,
                                                   const int* __restrict__ cell_start,
                                                   long long ncells, int* __restrict__ perm,
                                                   int max_pts, int* __restrict__ overflow) {
    __shared__ int s[kSortCap];
    long long c = blockIdx.x;
    if (c >= ncells) return;
    int a = cell_start[c], b = cell_start[c + 1];
    int m = b - a;
    if (m <= 1) {
        if (m == 1 && threadIdx.x == 0) perm[a] = tmp[a];
        return;
    }
    if (m > max_pts || m > kSortCap) {
        if (threadIdx.x == 0) atomicAdd(overflow, 1);
        return;
    }
    for (int k = threadIdx.x; k < m; k += 64) s[k] = tmp[a + k];
    __syncthreads();
    for (int k = threadIdx.x; k < m; k += 64) {
        int v = s[k], r = 0;
        for (int j = 0; j < m; ++j) r += s[j] < v;
        perm[a + r] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_gather(const double* __restrict__ pts,
                                                   const double* __restrict__ vals,
                                                   const int* __restrict__ perm,
                                                   const int* __restrict__ cell_of, long long n,
                                                   Grid g, double sc, double* __restrict__ xs,
                                                   double* __restrict__ ys, double* __restrict__ fs,
                                                   float* __restrict__ xr, float* __restrict__ yr) {
    long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    int i = perm[s];
    double x = pts[2 * (long long)i], y = pts[2 * (long long)i + 1];
    xs[s] = x;
    ys[s] = y;
    if (fs) fs[s] = vals ? vals[i] : 0.0;
    int c = cell_of[i];
    int cx = c % g.ncx, cy = c / g.ncx;
    // cell-centre-relative coordinates, scaled so that the squared scaled
    // distance is the base-2 exponent of the Gaussian
    double ox = g.x0 + ((double)cx + 0.5) * g.L;
    double oy = g.y0 + ((double)cy + 0.5) * g.L;
    xr[s] = (float)((x - ox) * sc);
    yr[s] = (float)((y - oy) * sc);
}

__global__ __launch_bounds__(64) void k_dup_check(const double* __restrict__ xs,
                                                  const double* __restrict__ ys,
                                                  const int* __restrict__ cell_start,
                                                  long long ncells, int* __restrict__ dup) {
    long long c = blockIdx.x;
    if (c >= ncells) return;
    int a = cell_start[c], b = cell_start[c + 1];
    int found = 0;
    for (int i = a + threadIdx.x; i < b; i += 64) {
        double x = xs[i], y = ys[i];
        for (int j = i + 1; j < b; ++j) found |= (xs[j] == x) & (ys[j] == y);
    }
    if (found) atomicOr(dup, 1);
}

__global__ __launch_bounds__(kBlock) void k_unpermute(const double* __restrict__ src,
                                                      const int* __restrict__ perm, long long n,
                                                      double* __restrict__ dst) {
    long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s < n) dst[perm[s]] = src[s];
}

__global__ __launch_bounds__(kBlock) void k_unpermute_int(const int* __restrict__ src,
                                                          const int* __restrict__ perm,
                                                          long long n, int* __restrict__ dst) {
    long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s < n) dst[perm[s]] = src[s];
}

__global__ __launch_bounds__(kBlock) void k_permute(const double* __restrict__ src,
                                                    const int* __restrict__ perm, long long n,
                                                    double* __restrict__ dst) {
    long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s < n) dst[s] = src[perm[s]];
}

inline unsigned blocks_for(long long n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_minmax(const double* pts, const double* vals, long long n, double* work,
                         double* out4, int* bad, hipStream_t st) {
    long long nb = blocks_for(n, kBlock);
    int grid = (int)(nb < kReduceBlocks ? nb : kReduceBlocks);
    if (grid < 1) grid = 1;
    k_minmax<<<grid, kBlock, 0, st>>>(pts, vals, n, work, bad);
    k_minmax_final<<<1, kBlock, 0, st>>>(work, grid, out4);
    return hipGetLastError();
}

hipError_t launch_cell_count(const double* pts, long long n, Grid g, int* cell_of, int* slot,
                             int* counts, hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_cell_count<<<blocks_for(n, kBlock), kBlock, 0, st>>>(pts, n, g, cell_of, slot, counts);
    return hipGetLastError();
}

long long scan_work_ints(long long n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_exclusive_scan(const int* in, int* out, long long n, int* work,
                                 hipStream_t st) {
    long long nt = (n + kScanTile - 1) / kScanTile;
    if (nt == 0) {
        return hipMemsetAsync(out, 0, sizeof(int), st);
    }
    k_scan_tile_sums<<<(unsigned)nt, kBlock, 0, st>>>(in, n, work);
    k_scan_sums<<<1, kBlock, 0, st>>>(work, nt);
    k_scan_tiles<<<(unsigned)nt, kBlock, 0, st>>>(in, n, work, out);
    return hipGetLastError();
}

hipError_t launch_scatter(const int* cell_of, const int* slot, const int* cell_start,
                          long long n, int* tmp, hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_scatter<<<blocks_for(n, kBlock), kBlock, 0, st>>>(cell_of, slot, cell_start, n, tmp);
    return hipGetLastError();
}

hipError_t launch_sort_cells(const int* tmp, const int* cell_start, long long ncells,
                             int* perm, int max_pts, int* overflow, hipStream_t st) {
    if (ncells == 0) return hipSuccess;
    k_sort_cells<<<(unsigned)ncells, 64, 0, st>>>(tmp, cell_start, ncells, perm, max_pts,
                                                  overflow);
    return hipGetLastError();
}

hipError_t launch_gather(const double* pts, const double* vals, const int* perm,
                         const int* cell_of, long long n, Grid g, double sc, double* xs,
                         double* ys, double* fs, float* xr, float* yr, hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_gather<<<blocks_for(n, kBlock), kBlock, 0, st>>>(pts, vals, perm, cell_of, n, g, sc, xs,
                                                       ys, fs, xr, yr);
    return hipGetLastError();
}

hipError_t launch_dup_check(const double* xs, const double* ys, const int* cell_start,
                            long long ncells, int* dup, hipStream_t st) {
    if (ncells == 0) return hipSuccess;
    k_dup_check<<<(unsigned)ncells, 64, 0, st>>>(xs, ys, cell_start, ncells, dup);
    return hipGetLastError();
}

hipError_t launch_unpermute(const double* src, const int* perm, long long n, double* dst,
                            hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_unpermute<<<blocks_for(n, kBlock), kBlock, 0, st>>>(src, perm, n, dst);
    return hipGetLastError();
}

hipError_t launch_unpermute_int(const int* src, const int* perm, long long n, int* dst,
                                hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_unpermute_int<<<blocks_for(n, kBlock), kBlock, 0, st>>>(src, perm, n, dst);
    return hipGetLastError();
}

hipError_t launch_permute(const double* src, const int* perm, long long n, double* dst,
                          hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_permute<<<blocks_for(n, kBlock), kBlock, 0, st>>>(src, perm, n, dst);
    return hipGetLastError();
}

}  // namespace rbf
