// precond.hip -- restricted additive Schwarz preconditioner on gfx950.
//
// RASM (Section 2.2, eq. rasm): z = sum_c Rt_c^T A_c^{-1} R_c v.  Cell c is the
// non-overlapping subdomain; its overlapping subdomain is the (2*overlap+1)^2
// block of cells around it.  Only the rows of A_c^{-1} that belong to c's own
// points are ever used, so setup stores exactly those: Z_c = (A_c^{-1})[centre
// rows, :], an n_c x n_omega block, and every application is one batched
// gather-GEMV z[c's points] = Z_c v[members of c].
//
// Setup per cell (one 256-thread workgroup, cells strided over a persistent
// grid, a private n_p x n_p scratch matrix per workgroup):
//  1. members: neighbour cells in (dy, dx) order, each a contiguous sorted
//     range, the cell's own points last; padded to n_p = 32 * ceil(n/32) by
//     leading identity rows so every block boundary is aligned;
//  2. A_c[p][q] = phi(|x_p - x_q|), the untruncated normalised Gaussian;
//  3. A_c = L L^T by a left-looking blocked Cholesky (32-column block columns,
//     the update of a block column as a register-tiled GEMM over LDS-staged
//     panels, the 32x32 diagonal block factored in LDS, the rows below by
//     substitution);
//  4. X = A_c^{-1} E_C (E_C = the centre columns of the identity) by a blocked
//     forward solve L W = E_C on the trailing rows only, then a blocked back
//     solve L^T X = W; X's columns, without the padding rows, are Z_c's rows
//     and are written straight into the Z buffer.
// The FP32 form (mixed precision) assembles in FP64, factors in FP32, and on a
// failed pivot retries with a diagonal shift mu = s * n * u32 * phi(0),
// s in {1, 10, 100, 1000} (shifted low-precision Cholesky).
#include "rbf_device.hpp"
#include "rbf_internal.hpp"
#include "../../include/rbf.h"

namespace rbf {

namespace {

constexpr int kNB = 32;        // block size of the factorisation
constexpr int kKC = 16;        // k-chunk staged per pass of the update
constexpr int kRS = 256;       // rows per super-block of the update
constexpr int kThreads = 256;
constexpr int kMaxRanges = 2 * 16 + 3;
constexpr int kZCols = 64;     // right-hand-side columns per pass of the solves

template <typename T>
struct SetupLds {
    union {
        struct {
            T Ls[kKC][kRS];
            T Lb[kKC][kNB];
        } upd;
        struct {
            T Lc[kNB][kNB + 1];
            T Xc[kNB][kZCols + 1];
            T acc[kNB][kZCols + 1];
        } zs;
        struct {
            double mx[RBF_MAX_BLOCK];
            double my[RBF_MAX_BLOCK];
        } coords;
    } u;
    T D[kNB][kNB + 1];
    T invd[kNB];
    int rb[kMaxRanges], re[kMaxRanges];
    int nranges, n_omega, n_c, flag;
};

// Member ranges of cell c's overlapping subdomain (sorted-order indices).
__device__ void block_ranges(const int* __restrict__ cs, const Grid& g, int ov, long long c,
                             int* rb, int* re, int* nranges, int* n_omega, int* n_c) {
    int cx = (int)(c % g.ncx), cy = (int)(c / g.ncx);
    int xlo = cx - ov < 0 ? 0 : cx - ov;
    int xhi = cx + ov > g.ncx - 1 ? g.ncx - 1 : cx + ov;
    int k = 0, tot = 0;
    for (int dy = -ov; dy <= ov; ++dy) {
        int ny = cy + dy;
        if (ny < 0 || ny >= g.ncy) continue;
        int row = ny * g.ncx;
        if (dy != 0) {
            rb[k] = cs[row + xlo];
            re[k] = cs[row + xhi + 1];
            tot += re[k] - rb[k];
            ++k;
        } else {
            if (cx > xlo) {
                rb[k] = cs[row + xlo];
                re[k] = cs[row + cx];
                tot += re[k] - rb[k];
                ++k;
            }
            if (cx < xhi) {
                rb[k] = cs[row + cx + 1];
                re[k] = cs[row + xhi + 1];
                tot += re[k] - rb[k];
                ++k;
            }
        }
    }
    rb[k] = cs[c];
    re[k] = cs[c + 1];
    *n_c = re[k] - rb[k];
    tot += *n_c;
    ++k;
    *nranges = k;
    *n_omega = tot;
}

__device__ __forceinline__ int member_index(const int* rb, const int* re, int nr, int q) {
    for (int k = 0; k < nr; ++k) {
        int l = re[k] - rb[k];
        if (q < l) return rb[k] + q;
        q -= l;
    }
    return -1;
}

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}

template <typename T>
__device__ __forceinline__ T sqrt_t(T v) {
    return __builtin_sqrt(v);
}
template <>
__device__ __forceinline__ float sqrt_t<float>(float v) {
    return __builtin_sqrtf(v);
}

// Left-looking blocked Cholesky of the n_p x n_p column-major matrix A (lower
// part).  Returns 0, or the 1-based index of the first non-positive pivot.
template <typename T>
__device__ int cholesky_blocked(T* __restrict__ A, int np, SetupLds<T>& s) {
    const int tid = threadIdx.x;
    const int cg = tid & 7, rg = tid >> 3;
    for (int J = 0; J < np; J += kNB) {
        if (J > 0) {
            for (int R = J; R < np; R += kRS) {
                T acc[8][4];
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[i][q] = T(0);
                for (int K = 0; K < J; K += kKC) {
                    __syncthreads();
                    for (int idx = tid; idx < kKC * kRS; idx += kThreads) {
                        int kk = idx / kRS, r = idx % kRS;
                        s.u.upd.Ls[kk][r] =
                            (R + r < np) ? A[(size_t)(K + kk) * np + R + r] : T(0);
                    }
                    for (int idx = tid; idx < kKC * kNB; idx += kThreads) {
                        int kk = idx / kNB, q = idx % kNB;
                        s.u.upd.Lb[kk][q] = A[(size_t)(K + kk) * np + J + q];
                    }
                    __syncthreads();
#pragma unroll 4
                    for (int kk = 0; kk < kKC; ++kk) {
                        T b0 = s.u.upd.Lb[kk][4 * cg + 0], b1 = s.u.upd.Lb[kk][4 * cg + 1];
                        T b2 = s.u.upd.Lb[kk][4 * cg + 2], b3 = s.u.upd.Lb[kk][4 * cg + 3];
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            T av = s.u.upd.Ls[kk][rg + 32 * i];
                            acc[i][0] = fma_t(av, b0, acc[i][0]);
                            acc[i][1] = fma_t(av, b1, acc[i][1]);
                            acc[i][2] = fma_t(av, b2, acc[i][2]);
                            acc[i][3] = fma_t(av, b3, acc[i][3]);
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    int row = R + rg + 32 * i;
                    if (row < np) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            size_t ad = (size_t)(J + 4 * cg + q) * np + row;
                            A[ad] = A[ad] - acc[i][q];
                        }
                    }
                }
            }
            __syncthreads();
        }
        // factor the diagonal block in LDS
        for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
            int i = idx % kNB, j = idx / kNB;
            s.D[i][j] = A[(size_t)(J + j) * np + J + i];
        }
        __syncthreads();
        for (int k = 0; k < kNB; ++k) {
            if (tid == 0) {
                T piv = s.D[k][k];
                if (!(piv > T(0))) {
                    s.flag = J + k + 1;
                } else {
                    T l = sqrt_t(piv);
                    s.D[k][k] = l;
                    s.invd[k] = T(1) / l;
                }
            }
            __syncthreads();
            if (s.flag) return s.flag;
            if (tid > k && tid < kNB) s.D[tid][k] = s.D[tid][k] * s.invd[k];
            __syncthreads();
            for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
                int i = idx % kNB, j = idx / kNB;
                if (j > k && i >= j) s.D[i][j] = s.D[i][j] - s.D[i][k] * s.D[j][k];
            }
            __syncthreads();
        }
        for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
            int i = idx % kNB, j = idx / kNB;
            if (i >= j) A[(size_t)(J + j) * np + J + i] = s.D[i][j];
        }
        // rows below: x L_JJ^T = a
        for (int row = J + kNB + tid; row < np; row += kThreads) {
            T x[kNB];
#pragma unroll
            for (int q = 0; q < kNB; ++q) x[q] = A[(size_t)(J + q) * np + row];
#pragma unroll
            for (int q = 0; q < kNB; ++q) {
                x[q] = x[q] * s.invd[q];
#pragma unroll
                for (int q2 = q + 1; q2 < kNB; ++q2) x[q2] = fma_t(-x[q], s.D[q2][q], x[q2]);
                // keep the LDS reads of the next column from being hoisted here
                __asm__ volatile("" ::: "memory");
            }
#pragma unroll
            for (int q = 0; q < kNB; ++q) A[(size_t)(J + q) * np + row] = x[q];
        }
        __syncthreads();
    }
    return 0;
}

// acc[r][c] over one 32-row block, staged through LDS, c < ncol, then
// s.u.zs.acc[r][c] = rhs(r, c) - acc[r][c], and the diagonal block L(I0.., I0..)
// with the reciprocals of its diagonal in s.D / s.invd.
// Forward: acc = sum_{k in [k_lo, k_hi)} L[I0 + r][k] X[k][c0 + c], rhs = E_C
// Backward: acc = sum_{k in [k_lo, k_hi)} L[k][I0 + r] X[k][c0 + c], rhs = W (the
// forward result, stored in X's place, zero above row w_lo).
template <typename T, bool kBackward>
__device__ void solve_block_rhs(const T* __restrict__ A, int np, int I0, int k_lo, int k_hi,
                                const T* __restrict__ Zc, int ldz, int p, int c0, int ncol,
                                int q0, int w_lo, SetupLds<T>& s) {
    const int tid = threadIdx.x;
    const int r = tid & 31, cg = tid >> 5;
    T acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = T(0);
    for (int k0 = k_lo; k0 < k_hi; k0 += kNB) {
        const int kn = k_hi - k0 < kNB ? k_hi - k0 : kNB;
        __syncthreads();
        for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
            if (kBackward) {
                int rr = idx / kNB, kk = idx % kNB;
                s.u.zs.Lc[kk][rr] = kk < kn ? A[(size_t)(I0 + rr) * np + k0 + kk] : T(0);
            } else {
                int kk = idx / kNB, rr = idx % kNB;
                s.u.zs.Lc[kk][rr] = kk < kn ? A[(size_t)(k0 + kk) * np + I0 + rr] : T(0);
            }
        }
        for (int idx = tid; idx < kNB * kZCols; idx += kThreads) {
            int cc = idx / kNB, kk = idx % kNB;
            int k = k0 + kk;
            T v = T(0);
            if (cc < ncol && kk < kn && k >= p) v = Zc[(size_t)(c0 + cc) * ldz + (k - p)];
            s.u.zs.Xc[kk][cc] = v;
        }
        __syncthreads();
        for (int kk = 0; kk < kn; ++kk) {
            T l = s.u.zs.Lc[kk][r];
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = fma_t(l, s.u.zs.Xc[kk][cg + 8 * j], acc[j]);
        }
    }
    __syncthreads();
    const int row = I0 + r;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int cc = cg + 8 * j;
        T rhs = T(0);
        if (cc < ncol) {
            if (kBackward)
                rhs = (row >= w_lo && row >= p) ? Zc[(size_t)(c0 + cc) * ldz + (row - p)] : T(0);
            else
                rhs = (row == q0 + c0 + cc) ? T(1) : T(0);
        }
        s.u.zs.acc[r][cc] = rhs - acc[j];
    }
    for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
        int i = idx % kNB, j = idx / kNB;
        s.D[i][j] = A[(size_t)(I0 + j) * np + I0 + i];
    }
    __syncthreads();
    if (tid < kNB) s.invd[tid] = T(1) / s.D[tid][tid];
    __syncthreads();
}

// Z_c = rows of A_c^{-1} for the centre; Zc row-major n_c x n_omega; X(k, c) is
// stored at Zc[c * n_omega + k - p] for k >= p (padding rows are zero).
// The 32 x 32 triangular solves run in place in LDS, one column per thread.
template <typename T>
__device__ void centre_rows_of_inverse(const T* __restrict__ A, int np, int p, int n_omega,
                                       int n_c, T* __restrict__ Zc, SetupLds<T>& s) {
    const int tid = threadIdx.x;
    const int q0 = np - n_c;
    const int ib = q0 / kNB;
    const int nblk = np / kNB;
    for (int c0 = 0; c0 < n_c; c0 += kZCols) {
        const int ncol = n_c - c0 < kZCols ? n_c - c0 : kZCols;
        // forward: L W = E_C on the rows of blocks ib .. nblk-1
        for (int I = ib; I < nblk; ++I) {
            const int I0 = I * kNB;
            solve_block_rhs<T, false>(A, np, I0, ib * kNB, I0, Zc, n_omega, p, c0, ncol, q0, 0, s);
            if (tid < ncol) {
                for (int r = 0; r < kNB; ++r) {
                    T v = s.u.zs.acc[r][tid];
                    for (int r2 = 0; r2 < r; ++r2) v = fma_t(-s.D[r][r2], s.u.zs.acc[r2][tid], v);
                    s.u.zs.acc[r][tid] = v * s.invd[r];
                }
                for (int r = 0; r < kNB; ++r)
                    if (I0 + r >= p) Zc[(size_t)(c0 + tid) * n_omega + (I0 + r - p)] = s.u.zs.acc[r][tid];
            }
        }
        // backward: L^T X = W from the last block up; W is zero above block ib
        for (int I = nblk - 1; I >= 0; --I) {
            const int I0 = I * kNB;
            if (I0 + kNB <= p) break;
            solve_block_rhs<T, true>(A, np, I0, I0 + kNB, np, Zc, n_omega, p, c0, ncol, q0,
                                     ib * kNB, s);
            if (tid < ncol) {
                for (int r = kNB - 1; r >= 0; --r) {
                    T v = s.u.zs.acc[r][tid];
                    for (int r2 = r + 1; r2 < kNB; ++r2)
                        v = fma_t(-s.D[r2][r], s.u.zs.acc[r2][tid], v);
                    s.u.zs.acc[r][tid] = v * s.invd[r];
                }
                for (int r = 0; r < kNB; ++r)
                    if (I0 + r >= p) Zc[(size_t)(c0 + tid) * n_omega + (I0 + r - p)] = s.u.zs.acc[r][tid];
            }
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_precond_setup(PrecondArgs a, T* __restrict__ Z,
                                                            T* __restrict__ scratch,
                                                            int* __restrict__ status) {
    __shared__ SetupLds<T> s;
    const int tid = threadIdx.x;
    T* A = scratch + (size_t)blockIdx.x * a.np_max * a.np_max;
    const int attempts = sizeof(T) == 4 ? 5 : 1;
    for (long long c = blockIdx.x; c < a.ncells; c += gridDim.x) {
        __syncthreads();
        if (tid == 0) {
            block_ranges(a.cell_start, a.g, a.overlap, c, s.rb, s.re, &s.nranges, &s.n_omega,
                         &s.n_c);
            s.flag = 0;
        }
        __syncthreads();
        const int n_omega = s.n_omega, n_c = s.n_c, nr = s.nranges;
        if (n_c == 0) {
            if (tid == 0) status[c] = 0;
            continue;
        }
        const int np = (n_omega + kNB - 1) / kNB * kNB;
        const int p = np - n_omega;
        int fail = 0, level = 0;
        for (int att = 0; att < attempts; ++att) {
            __syncthreads();
            for (int k = tid; k < n_omega; k += kThreads) {
                int m = member_index(s.rb, s.re, nr, k);
                s.u.coords.mx[k] = a.xs[m];
                s.u.coords.my[k] = a.ys[m];
            }
            if (tid == 0) s.flag = 0;
            __syncthreads();
            double shift = 0.0;
            if (att > 0) {
                const double mult[5] = {0.0, 1.0, 10.0, 100.0, 1000.0};
                shift = mult[att] * (double)n_omega * 5.9604644775390625e-08 * a.norm;
            }
            // untruncated Gaussian on the members, lower triangle, leading padding
            for (long long idx = tid; idx < (long long)np * np; idx += kThreads) {
                int j = (int)(idx / np), i = (int)(idx % np);
                if (i < j) continue;
                double v;
                if (i < p || j < p) {
                    v = (i == j) ? 1.0 : 0.0;
                } else {
                    double dx = s.u.coords.mx[i - p] - s.u.coords.mx[j - p];
                    double dy = s.u.coords.my[i - p] - s.u.coords.my[j - p];
                    double d2 = __builtin_fma(dx, dx, dy * dy);
                    v = exp_neg(d2 * a.mk) * a.norm;
                    if (i == j) v += shift;
                }
                A[(size_t)j * np + i] = (T)v;
            }
            __syncthreads();
            fail = cholesky_blocked<T>(A, np, s);
            level = att;
            if (!fail) break;
        }
        if (fail) {
            if (tid == 0) status[c] = fail;
            continue;
        }
        centre_rows_of_inverse<T>(A, np, p, n_omega, n_c, Z + a.zoff[c], s);
        if (tid == 0) status[c] = -level;
    }
}

// ===========================================================================
// FP64 setup on the matrix cores, batched in lockstep.  Each cell of a batch
// (a slot) keeps its n_p x n_p lower triangle in a scratch slot, stored by
// block rows (see roff).  The left-looking blocked Cholesky advances one
// 32-column block column J at a time for every slot together, one launch per
// J: each workgroup takes a 256-row tile below the diagonal block, updates it
// with the finished block columns as MFMA tiles (the result lands in LDS),
// solves x L_JJ^T = a for its rows by substitution (one row per thread, L_JJ
// broadcast from LDS), and writes the rows back.  The
// workgroup of the first tile then also forms and factors the next diagonal
// block, which only needs rows it has just finished.  The centre rows of the
// inverse follow: one launch for the forward solve on the trailing rows, one
// launch per block row of the back solve.  Every launch carries thousands of
// independent workgroups, so one cell's serial steps overlap with other
// cells' work.  Workgroup b serves slot b % nslots_pad (a multiple of 8): a
// slot's workgroups run on one XCD in every launch, and its rows stay in that
// XCD's L2 from launch to launch.
// Operand layout of v_mfma_f64_16x16x4f64 on gfx950: lane l holds
// A[l%16][l/16] and B[l/16][l%16]; result register v holds D[l/16 + 4v][l%16].
// ===========================================================================
typedef double d4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

constexpr int kT2 = 256;        // threads of the assembly and inverse-row kernels (4 waves)
constexpr int kW2 = kT2 / 64;
constexpr int kTS = 256;        // threads of a factorisation step (4 waves)
constexpr int kWS = kTS / 64;
constexpr int kRows2 = 256;     // rows per step tile
constexpr int kRT2 = kRows2 / 16 / kWS;   // row tiles per wave (4)
static_assert(kRows2 == kTS, "the substitution gives one row to each thread");
constexpr int kXS = kRows2 + 1; // padded LDS row of a staged tile (conflict-free MFMA stores)
constexpr int kTri = kNB * (kNB + 1) / 2;

// Index of (k, j), j >= k, in the packed upper triangle of a 32x32 block.
__host__ __device__ constexpr int tri(int k, int j) { return kNB * k - k * (k - 1) / 2 + (j - k); }
constexpr int kZK = 64;         // k per LDS panel in the inverse-row products

// Block-row storage of a slot's lower triangle: the 32 rows of block row I are
// stored with stride 32 (I + 1) (their columns up to the end of the diagonal
// block), block rows one after another, so every row starts on a 256-byte
// boundary and a slot needs 512 B (B + 1) doubles for B block rows.
__device__ __forceinline__ size_t roff(int row) {
    const int I = row >> 5;
    return (size_t)(32 * (I + 1)) * (size_t)(16 * I + (row & 31));
}

struct StepLds {
    union {
        double X[kNB][kXS];               // the tile's rows, one column per thread
        struct {
            double D[kNB][kNB + 1];       // the next diagonal block
            double part[kWS][3][16][17];  // per-wave partial products of its tiles
        } d;
    } u;
    double Lt[kTri];                      // L_JJ transposed (packed), reciprocal pivots on the diagonal
    int flag;
};

struct ZLds {
    double Lc[kZK][kNB + 1];
    double Xc[kZK][kZCols + 1];
    double acc[kNB][kZCols + 1];
    double D[kNB][kNB + 1];
    double invd[kNB];
};

__device__ __forceinline__ double readlane_d(double v, int lane) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}



__device__ __forceinline__ d4v mfma_f64(double a, double b, d4v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ d4v load4(const double* __restrict__ p) {
    return *reinterpret_cast<const d4v*>(p);
}

// X[c][r] = A[R + r][J + c] - sum_{k < J} L[R + r][k] L[J + c][k] for the
// nrow (a multiple of 32, <= 256) rows of the tile, J > 0.  MFMA tiles with
// no LDS staging and no barriers: the contraction index of an MFMA may be
// permuted as long as A and B use the same permutation, so over a chunk of 16
// k values lane group g = l/16 owns k = K+4g .. K+4g+3 and loads them from its
// row with one 32-byte load; step s of the chunk uses element s.  Each wave
// loads its own M row tiles (three register buffers: two chunks in flight
// while one is multiplied) and both column tiles (shared by the waves through
// the caches; two buffers).  Six chunks per loop pass keep every buffer index
// a constant and the body free of branches, so each multiply waits only for
// its own loads.
template <int M>
struct UpdateRegs {
    d4v a[3][M];
    d4v b[2][2];
    d4v acc[M][2];
    const double* arow[M];
    const double* brow[2];

    __device__ __forceinline__ void load_a(int buf, int ch) {
#pragma unroll
        for (int t = 0; t < M; ++t) a[buf][t] = load4(arow[t] + 16 * ch);
    }
    __device__ __forceinline__ void load_b(int buf, int ch) {
        b[buf][0] = load4(brow[0] + 16 * ch);
        b[buf][1] = load4(brow[1] + 16 * ch);
    }
    __device__ __forceinline__ void mma(int ba, int bb) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
#pragma unroll
            for (int t = 0; t < M; ++t) {
                acc[t][0] = mfma_f64(a[ba][t][st], b[bb][0][st], acc[t][0]);
                acc[t][1] = mfma_f64(a[ba][t][st], b[bb][1][st], acc[t][1]);
            }
        }
    }
    // chunks c .. c + min(R, 6) - 1; on entry chunks c, c + 1 of A and chunk c
    // of B are loaded (c is a multiple of 6), no load reaches c + R
    template <int R>
    __device__ __forceinline__ void run(int c) {
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            if (i < R) {
                if (i + 2 < R) load_a((i + 2) % 3, c + i + 2);
                if (i + 1 < R) load_b((i + 1) % 2, c + i + 1);
                mma(i % 3, i % 2);
            }
        }
    }
};

template <int M>
__device__ __forceinline__ void update_core(const double* __restrict__ A, int J, int R, int wave,
                                            double (*X)[kXS]) {
    const int lane = threadIdx.x & 63;
    const int i16 = lane & 15, g = lane >> 4;
    UpdateRegs<M> u;
#pragma unroll
    for (int t = 0; t < M; ++t) {
        u.acc[t][0] = u.acc[t][1] = d4v{0.0, 0.0, 0.0, 0.0};
        u.arow[t] = A + roff(R + 16 * (wave + kWS * t) + i16) + 4 * g;
    }
    u.brow[0] = A + roff(J + i16) + 4 * g;
    u.brow[1] = A + roff(J + 16 + i16) + 4 * g;
    const int nchunk = J / 16;   // >= 2, even
    u.load_a(0, 0);
    u.load_a(1, 1);
    u.load_b(0, 0);
    int c = 0;
    for (; c + 8 <= nchunk; c += 6) u.template run<99>(c);
    const int rest = nchunk - c;   // 2, 4 or 6
    if (rest == 2)
        u.template run<2>(c);
    else if (rest == 4)
        u.template run<4>(c);
    else
        u.template run<6>(c);
#pragma unroll
    for (int t = 0; t < M; ++t) {
        const int tile = wave + kWS * t;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rl = 16 * tile + g + 4 * v;
                const int col = 16 * cb + i16;
                X[col][rl] = A[roff(R + rl) + J + col] - u.acc[t][cb][v];
            }
    }
}

__device__ void update_tile(const double* __restrict__ A, int J, int R, int nrow,
                            double (*X)[kXS]) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ntile = nrow / 16;
    const int mine = (ntile - wave + kWS - 1) / kWS;   // row tiles of this wave (uniform)
    static_assert(kRT2 == 4, "row tiles per wave");
    switch (mine) {
        case 4: update_core<4>(A, J, R, wave, X); break;
        case 3: update_core<3>(A, J, R, wave, X); break;
        case 2: update_core<2>(A, J, R, wave, X); break;
        case 1: update_core<1>(A, J, R, wave, X); break;
        default: break;
    }
}

// X[c][r] = A[R + r][J + c] (coalesced 16-byte loads), r < nrow.
__device__ void load_tile(const double* __restrict__ A, int J, int R, int nrow, double (*X)[kXS]) {
    for (int id = threadIdx.x; id < nrow * (kNB / 2); id += kTS) {
        const int r = id / (kNB / 2), c = 2 * (id % (kNB / 2));
        const d2v v = *reinterpret_cast<const d2v*>(A + roff(R + r) + J + c);
        X[c][r] = v[0];
        X[c + 1][r] = v[1];
    }
}

// A[R + r][J + c] = X[c][r] (coalesced 16-byte stores), r < nrow.
__device__ void store_tile(double* __restrict__ A, int J, int R, int nrow, double (*X)[kXS]) {
    for (int id = threadIdx.x; id < nrow * (kNB / 2); id += kTS) {
        const int r = id / (kNB / 2), c = 2 * (id % (kNB / 2));
        d2v v;
        v[0] = X[c][r];
        v[1] = X[c + 1][r];
        *reinterpret_cast<d2v*>(A + roff(R + r) + J + c) = v;
    }
}

// Row tid of the tile: x L_JJ^T = a in place (column tid of X), column by
// column so that every step is 31 - k independent FMAs.  Lt holds L_JJ
// transposed (Lt[k][j] = L[j][k], j > k) with the reciprocal pivots on its
// diagonal; every lane reads the same Lt entries (LDS broadcasts).
__device__ __forceinline__ void trsm_tile(const double* Lt, int nrow, double (*X)[kXS]) {
    const int tid = threadIdx.x;
    if (tid >= nrow) return;
    double x[kNB];
#pragma unroll
    for (int q = 0; q < kNB; ++q) x[q] = X[q][tid];
#pragma unroll
    for (int k = 0; k < kNB; ++k) {
        x[k] *= Lt[tri(k, k)];
#pragma unroll
        for (int j = k + 1; j < kNB; ++j) x[j] = __builtin_fma(-x[k], Lt[tri(k, j)], x[j]);
    }
#pragma unroll
    for (int q = 0; q < kNB; ++q) X[q][tid] = x[q];
}

// D = A[J0.., J0..] - L[J0.., 0:J0] L[J0.., 0:J0]^T on the three lower 16x16
// tiles of the 32x32 diagonal block, J0 > 0: wave w multiplies all three
// tiles over its quarter of the chunks (three independent MFMA chains), and
// the four partial products are summed through LDS.
__device__ __forceinline__ void syrk_diag(const double* __restrict__ A, int J0,
                                          double (*D)[kNB + 1], double (*part)[3][16][17]) {
    static_assert(kWS == 4, "four partial products");
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i16 = lane & 15, g = lane >> 4;
    const double* r0 = A + roff(J0 + i16) + 4 * g;        // rows J0 .. J0+15
    const double* r1 = A + roff(J0 + 16 + i16) + 4 * g;   // rows J0+16 .. J0+31
    d4v t00 = {0.0, 0.0, 0.0, 0.0}, t10 = t00, t11 = t00;
    auto mma = [&](const d4v& a0, const d4v& a1) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            t00 = mfma_f64(a0[st], a0[st], t00);
            t10 = mfma_f64(a1[st], a0[st], t10);
            t11 = mfma_f64(a1[st], a1[st], t11);
        }
    };
    // chunks wave, wave + 4, ...: two register buffers in turn
    const int nchunk = J0 / 16;
    d4v p0 = {0.0, 0.0, 0.0, 0.0}, p1 = p0, q0 = p0, q1 = p0;
    if (wave < nchunk) {
        p0 = load4(r0 + 16 * wave);
        p1 = load4(r1 + 16 * wave);
    }
    for (int ch = wave; ch < nchunk; ch += 2 * kWS) {
        const bool second = ch + kWS < nchunk;
        if (second) {
            q0 = load4(r0 + 16 * (ch + kWS));
            q1 = load4(r1 + 16 * (ch + kWS));
        }
        mma(p0, p1);
        if (ch + 2 * kWS < nchunk) {
            p0 = load4(r0 + 16 * (ch + 2 * kWS));
            p1 = load4(r1 + 16 * (ch + 2 * kWS));
        }
        if (second) mma(q0, q1);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = g + 4 * v;
        part[wave][0][r][i16] = t00[v];
        part[wave][1][r][i16] = t10[v];
        part[wave][2][r][i16] = t11[v];
    }
    __syncthreads();
    for (int idx = tid; idx < 3 * 256; idx += kTS) {
        const int t = idx >> 8, r = (idx >> 4) & 15, c = idx & 15;
        const double sum = (part[0][t][r][c] + part[1][t][r][c]) + (part[2][t][r][c] + part[3][t][r][c]);
        const int row = 16 * (t == 0 ? 0 : 1) + r, col = 16 * (t == 2 ? 1 : 0) + c;
        D[row][col] = A[roff(J0 + row) + J0 + col] - sum;
    }
}

// Factor the 32x32 diagonal block J0 (lower part of D) in wave 0's registers
// (lane i holds row i; broadcasts by readlane, no barriers).  Step k: the
// pivot, its reciprocal square root (hardware estimate and two Newton steps),
// column k of L written to A and, transposed with the reciprocal pivot on the
// diagonal, to Lt, then the rank-1 update of the rows below.  Returns 0 or J0
// + the failing 1-based pivot index (all threads).
__device__ __forceinline__ int factor_diag_block(double* __restrict__ A, int J0,
                                                 double (*D)[kNB + 1], int* flag,
                                                 double* __restrict__ Lt) {
    const int tid = threadIdx.x;
    if (tid < 64) {
        const int i = tid & 31;
        const bool own = tid < kNB;
        double* arow = A + roff(J0 + i) + J0;
        double r[kNB];
#pragma unroll
        for (int c = 0; c < kNB; ++c) r[c] = (c <= i) ? D[i][c] : 0.0;
        int bad = 0;
#pragma unroll
        for (int k = 0; k < kNB; ++k) {
            const double piv = readlane_d(r[k], k);
            if (!bad && !(piv > 0.0)) bad = k + 1;   // uniform; later values are moot
            double y = __builtin_amdgcn_rsq(piv);
            y = y * __builtin_fma(-0.5 * piv * y, y, 1.5);
            y = y * __builtin_fma(-0.5 * piv * y, y, 1.5);
            const double l = (i == k) ? piv * y : r[k] * y;
            r[k] = l;
#pragma unroll
            for (int j = k + 1; j < kNB; ++j) {
                r[j] = __builtin_fma(-l, readlane_d(l, j), r[j]);
                // the update happens here, not where r[j] is next read: the
                // broadcast values stay short-lived (no SGPR spills)
                __asm__ volatile("" : "+v"(r[j]));
            }
            if (own && i >= k) {
                arow[k] = l;
                Lt[k * kNB + i] = (i == k) ? y : l;
            }
        }
        if (tid == 0) *flag = bad ? J0 + bad : 0;
    }
    __syncthreads();
    return *flag;
}

// s.acc[r][c] = rhs(r, c) - sum_k op(L)[I0 + r][k] X[k][c0 + c] over
// k in [k_lo, k_hi) (MFMA, 8 tiles of 16x16, two per wave), then the diagonal
// block L(I0.., I0..) into s.D / s.invd.
//   forward (kBackward = false): op(L)[r][k] = L[r][k], rhs = E_C
//   backward: op(L)[r][k] = L[k][r], rhs = the forward result W stored in X's
//   place (zero above row w_lo)
template <bool kBackward>
__device__ void zsolve_block(const double* __restrict__ A, int I0, int k_lo, int k_hi,
                             const double* __restrict__ Zc, int ldz, int p, int c0, int ncol,
                             int q0, int w_lo, ZLds& s) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rt = wave >> 1, ct0 = 2 * (wave & 1);
    d4v acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    const int nchunk = (k_hi - k_lo + kZK - 1) / kZK;
    constexpr int kLL = kZK * kNB / kT2;      // 8 L values per thread
    constexpr int kLX = kZK * kZCols / kT2;   // 16 X values per thread
    static_assert(kZK * kNB % kT2 == 0 && kZK * kZCols % kT2 == 0, "panels split evenly");
    double rl[kLL], rx[kLX];
    auto load = [&](int chunk) {
        const int k0 = k_lo + chunk * kZK;
#pragma unroll
        for (int q = 0; q < kLL; ++q) {
            const int idx = tid + kT2 * q;
            double v = 0.0;
            if (kBackward) {   // L[k0 + kk][I0 + rr]: contiguous in rr
                const int kk = idx / kNB, rr = idx % kNB;
                if (k0 + kk < k_hi) v = A[roff(k0 + kk) + I0 + rr];
            } else {           // L[I0 + rr][k0 + kk]: contiguous in kk
                const int rr = idx / kZK, kk = idx % kZK;
                if (k0 + kk < k_hi) v = A[roff(I0 + rr) + k0 + kk];
            }
            rl[q] = v;
        }
#pragma unroll
        for (int q = 0; q < kLX; ++q) {
            const int idx = tid + kT2 * q;
            const int cc = idx / kZK, kk = idx % kZK;
            const int k = k0 + kk;
            double v = 0.0;
            if (cc < ncol && k < k_hi && k >= p) v = Zc[(size_t)(c0 + cc) * ldz + (k - p)];
            rx[q] = v;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < kLL; ++q) {
            const int idx = tid + kT2 * q;
            if (kBackward)
                s.Lc[idx / kNB][idx % kNB] = rl[q];
            else
                s.Lc[idx % kZK][idx / kZK] = rl[q];
        }
#pragma unroll
        for (int q = 0; q < kLX; ++q) {
            const int idx = tid + kT2 * q;
            s.Xc[idx % kZK][idx / kZK] = rx[q];
        }
    };
    __syncthreads();
    if (nchunk > 0) {
        load(0);
        store();
        __syncthreads();
        for (int ch = 0; ch < nchunk; ++ch) {
            if (ch + 1 < nchunk) load(ch + 1);
#pragma unroll
            for (int ks = 0; ks < kZK / 4; ++ks) {
                const int kr = 4 * ks + (lane >> 4);
                const double a = s.Lc[kr][16 * rt + (lane & 15)];
                const double b0 = s.Xc[kr][16 * ct0 + (lane & 15)];
                const double b1 = s.Xc[kr][16 * ct0 + 16 + (lane & 15)];
                acc0 = mfma_f64(a, b0, acc0);
                acc1 = mfma_f64(a, b1, acc1);
            }
            __syncthreads();
            if (ch + 1 < nchunk) {
                store();
                __syncthreads();
            }
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 16 * rt + (lane >> 4) + 4 * v;
            const int cc = 16 * (ct0 + h) + (lane & 15);
            const int row = I0 + r;
            double rhs = 0.0;
            if (cc < ncol) {
                if (kBackward)
                    rhs = (row >= w_lo && row >= p) ? Zc[(size_t)(c0 + cc) * ldz + (row - p)] : 0.0;
                else
                    rhs = (row == q0 + c0 + cc) ? 1.0 : 0.0;
            }
            s.acc[r][cc] = rhs - (h ? acc1[v] : acc0[v]);
        }
    }
    for (int idx = tid; idx < kNB * kNB; idx += kT2) {
        const int i = idx / kNB, j = idx % kNB;
        s.D[i][j] = (j <= i) ? A[roff(I0 + i) + I0 + j] : 0.0;
    }
    __syncthreads();
    if (tid < kNB) s.invd[tid] = 1.0 / s.D[tid][tid];
    __syncthreads();
}

// Per-slot record kept in device memory for the launches of one batch:
// x = n_p, y = n_omega, z = n_c, w = 1 while the slot's cell is being built
// (0: empty cell, beyond the last cell, or a failed pivot).
struct AssembleLds {
    double mx[RBF_MAX_BLOCK];
    double my[RBF_MAX_BLOCK];
    double D[kNB][kNB + 1];
    int rb[kMaxRanges], re[kMaxRanges];
    int nranges, n_omega, n_c, flag;
};

// Slot b: members of cell c0 + b, the untruncated Gaussian on them (lower
// triangle, leading identity padding), the slot record, status 0, and the
// factor of the first diagonal block.
__global__ __launch_bounds__(kT2, 2) void k_setup_assemble_f64(PrecondArgs a, long long c0,
                                                               int nslots,
                                                               double* __restrict__ scratch,
                                                               int4* __restrict__ meta,
                                                               int* __restrict__ status,
                                                               double* __restrict__ lt_out) {
    __shared__ AssembleLds s;
    const int slot = blockIdx.x;
    const long long c = c0 + slot;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (slot >= nslots || c >= a.ncells) {
        if (tid == 0) meta[slot] = int4{0, 0, 0, 0};
        return;
    }
    if (tid == 0)
        block_ranges(a.cell_start, a.g, a.overlap, c, s.rb, s.re, &s.nranges, &s.n_omega, &s.n_c);
    __syncthreads();
    const int n_omega = s.n_omega, n_c = s.n_c, nr = s.nranges;
    const int np = (n_omega + kNB - 1) / kNB * kNB;
    if (tid == 0) {
        meta[slot] = int4{np, n_omega, n_c, n_c > 0 ? 1 : 0};
        status[c] = 0;
    }
    if (n_c == 0) return;
    const int p = np - n_omega;
    double* A = scratch + (size_t)slot * slot_elems64(a.np_max);
    for (int k = tid; k < n_omega; k += kT2) {
        const int m = member_index(s.rb, s.re, nr, k);
        s.mx[k] = a.xs[m];
        s.my[k] = a.ys[m];
    }
    __syncthreads();
    // wave w fills rows w, w + 4, ...; the first 32 rows also go to D
    for (int i = wave; i < np; i += kW2) {
        double* arow = A + roff(i);
        for (int j = lane; j <= i; j += 64) {
            double v;
            if (i < p || j < p) {
                v = (i == j) ? 1.0 : 0.0;
            } else {
                const double dx = s.mx[i - p] - s.mx[j - p];
                const double dy = s.my[i - p] - s.my[j - p];
                v = exp_neg(__builtin_fma(dx, dx, dy * dy) * a.mk) * a.norm;
            }
            arow[j] = v;
            if (i < kNB) s.D[i][j] = v;
        }
    }
    __syncthreads();
    const int f = factor_diag_block(A, 0, s.D, &s.flag, lt_out + (size_t)slot * kNB * kNB);
    if (f && tid == 0) {
        status[c] = f;
        meta[slot].w = 0;
    }
}

// Block column J: workgroup b takes the 256-row tile b / nslots_pad below the
// diagonal block of slot b % nslots_pad; the first tile's workgroup then
// factors diagonal block J + 32.  lt_in / lt_out: per slot, L_JJ and L_{J+32}
// transposed with reciprocal pivots (two buffers, alternating with J).
__global__ __launch_bounds__(kTS, 2) void k_chol_step(PrecondArgs a, long long c0, int J,
                                                      int nslots_pad, double* __restrict__ scratch,
                                                      int4* __restrict__ meta,
                                                      int* __restrict__ status,
                                                      const double* __restrict__ lt_in,
                                                      double* __restrict__ lt_out) {
    __shared__ StepLds s;
    const int slot = blockIdx.x % nslots_pad, tile = blockIdx.x / nslots_pad;
    const int4 m = meta[slot];
    const int np = m.x;
    const int R = J + kNB + kRows2 * tile;
    if (!m.w || R >= np) return;
    const int tid = threadIdx.x;
    double* A = scratch + (size_t)slot * slot_elems64(a.np_max);
    const int nrow = np - R < kRows2 ? np - R : kRows2;
    for (int e = tid; e < kNB * kNB; e += kTS) {
        const int k = e / kNB, j = e % kNB;
        if (j >= k) s.Lt[tri(k, j)] = lt_in[(size_t)slot * kNB * kNB + e];
    }
    if (J > 0)
        update_tile(A, J, R, nrow, s.u.X);
    else
        load_tile(A, J, R, nrow, s.u.X);
    __syncthreads();
    trsm_tile(s.Lt, nrow, s.u.X);
    __syncthreads();
    store_tile(A, J, R, nrow, s.u.X);
    if (tile == 0) {
        __syncthreads();
        syrk_diag(A, J + kNB, s.u.d.D, s.u.d.part);
        __syncthreads();
        const int f = factor_diag_block(A, J + kNB, s.u.d.D, &s.flag,
                                        lt_out + (size_t)slot * kNB * kNB);
        if (f && tid == 0) {
            status[c0 + slot] = f;
            meta[slot].w = 0;
        }
    }
}

// Centre rows, forward part: L W = E_C on the trailing block rows; workgroup
// b takes the 64 right-hand sides (b / nslots_pad) of slot b % nslots_pad.
// X(k, col) lives at Zc[col * n_omega + k - p] (padding rows are zero).
__global__ __launch_bounds__(kT2, 2) void k_z_forward(PrecondArgs a, long long c0, int nslots_pad,
                                                      const double* __restrict__ scratch,
                                                      const int4* __restrict__ meta,
                                                      double* __restrict__ Z) {
    __shared__ ZLds s;
    const int slot = blockIdx.x % nslots_pad, cp = blockIdx.x / nslots_pad;
    const int4 m = meta[slot];
    const int np = m.x, n_omega = m.y, n_c = m.z;
    const int col0 = cp * kZCols;
    if (!m.w || col0 >= n_c) return;
    const int tid = threadIdx.x;
    const int ncol = n_c - col0 < kZCols ? n_c - col0 : kZCols;
    const int p = np - n_omega, q0 = np - n_c, ib = q0 / kNB, nblk = np / kNB;
    const double* A = scratch + (size_t)slot * slot_elems64(a.np_max);
    double* Zc = Z + a.zoff[c0 + slot];
    for (int I = ib; I < nblk; ++I) {
        const int I0 = I * kNB;
        zsolve_block<false>(A, I0, ib * kNB, I0, Zc, n_omega, p, col0, ncol, q0, 0, s);
        if (tid < ncol) {
            for (int r = 0; r < kNB; ++r) {
                double v = s.acc[r][tid];
                for (int r2 = 0; r2 < r; ++r2) v = __builtin_fma(-s.D[r][r2], s.acc[r2][tid], v);
                s.acc[r][tid] = v * s.invd[r];
            }
            for (int r = 0; r < kNB; ++r)
                if (I0 + r >= p) Zc[(size_t)(col0 + tid) * n_omega + (I0 + r - p)] = s.acc[r][tid];
        }
    }
}

// Centre rows, back solve of block row I: L_II^T X_I = W_I - L[below, I]^T
// X[below]; the slot's block rows are visited from its last one up.  One wave
// per (slot, 64 right-hand sides): the product (32 rows x 64 columns, eight
// 16x16 MFMA tiles) takes its operands straight from memory into registers,
// each loaded once, the next chunk of 16 k in flight; W_I and the result move
// through LDS with coalesced accesses, and the 32x32 triangular solve runs one
// right-hand side per lane, unrolled in registers.
constexpr int kZT = 64;   // threads of the back-solve kernel (one wave)

struct ZBackLds {
    double T[kNB][kZCols + 1];   // W_I - product, then X_I
    double L[kNB][kNB + 1];      // L_II
    double invd[kNB];
};

__global__ __launch_bounds__(kZT) void k_z_back(PrecondArgs a, long long c0, int I,
                                                int nslots_pad,
                                                const double* __restrict__ scratch,
                                                const int4* __restrict__ meta,
                                                double* __restrict__ Z) {
    __shared__ ZBackLds s;
    const int slot = blockIdx.x % nslots_pad, cp = blockIdx.x / nslots_pad;
    const int4 m = meta[slot];
    const int np = m.x, n_omega = m.y, n_c = m.z;
    const int col0 = cp * kZCols;
    const int I0 = I * kNB;
    const int p = np - n_omega;
    if (!m.w || col0 >= n_c || I0 >= np || I0 + kNB <= p) return;
    const int lane = threadIdx.x;
    const int ncol = n_c - col0 < kZCols ? n_c - col0 : kZCols;
    const int w_lo = (np - n_c) / kNB * kNB;   // W is zero above this row
    const double* A = scratch + (size_t)slot * slot_elems64(a.np_max);
    double* Zc = Z + a.zoff[c0 + slot] + (size_t)col0 * n_omega - p;   // Zc[c * n_omega + k]
    // W_I (zero above w_lo and in the padding rows), coalesced along each Z row
    for (int idx = lane; idx < kNB * kZCols; idx += kZT) {
        const int c = idx / kNB, r = idx % kNB;
        const int row = I0 + r;
        s.T[r][c] = (c < ncol && row >= w_lo && row >= p) ? Zc[(size_t)c * n_omega + row] : 0.0;
    }
    for (int idx = lane; idx < kNB * kNB; idx += kZT) {
        const int i = idx / kNB, j = idx % kNB;
        s.L[i][j] = (j <= i) ? A[roff(I0 + i) + I0 + j] : 0.0;
    }
    // product over k in [I0 + 32, np)
    const int i16 = lane & 15, g = lane >> 4;
    const int nchunk = (np - I0 - kNB) / 16;   // even
    d4v acc[2][4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = d4v{0.0, 0.0, 0.0, 0.0};
    if (nchunk > 0) {
        const double* zr[4];
        bool zv[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            zv[ct] = 16 * ct + i16 < ncol;
            zr[ct] = Zc + (size_t)(zv[ct] ? 16 * ct + i16 : 0) * n_omega;
        }
        struct Buf {
            double a[2][4], b[4][4];
        } q0, q1;
        auto load = [&](Buf& d, int ch) {
            const int k = I0 + kNB + 16 * ch + 4 * g;
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const double* lr = A + roff(k + st) + I0 + i16;
                d.a[0][st] = lr[0];
                d.a[1][st] = lr[16];
            }
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                for (int st = 0; st < 4; ++st) d.b[ct][st] = zv[ct] ? zr[ct][k + st] : 0.0;
        };
        auto mma = [&](const Buf& d) {
#pragma unroll
            for (int st = 0; st < 4; ++st)
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct)
                        acc[rt][ct] = mfma_f64(d.a[rt][st], d.b[ct][st], acc[rt][ct]);
        };
        // two register buffers in turn (nchunk is even)
        load(q0, 0);
        for (int ch = 0; ch < nchunk; ch += 2) {
            load(q1, ch + 1);
            mma(q0);
            if (ch + 2 < nchunk) load(q0, ch + 2);
            mma(q1);
        }
    }
    __syncthreads();
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) s.T[16 * rt + g + 4 * v][16 * ct + i16] -= acc[rt][ct][v];
    if (lane < kNB) s.invd[lane] = 1.0 / s.L[lane][lane];
    __syncthreads();
    // L_II^T x = t for right-hand side `lane`, from the last row up
    {
        double x[kNB];
#pragma unroll
        for (int r = 0; r < kNB; ++r) x[r] = s.T[r][lane];
#pragma unroll
        for (int r = kNB - 1; r >= 0; --r) {
            x[r] *= s.invd[r];
#pragma unroll
            for (int r2 = 0; r2 < r; ++r2) x[r2] = __builtin_fma(-s.L[r][r2], x[r], x[r2]);
        }
#pragma unroll
        for (int r = 0; r < kNB; ++r) s.T[r][lane] = x[r];
    }
    __syncthreads();
    for (int idx = lane; idx < kNB * kZCols; idx += kZT) {
        const int c = idx / kNB, r = idx % kNB;
        const int row = I0 + r;
        if (c < ncol && row >= p) Zc[(size_t)c * n_omega + row] = s.T[r][c];
    }
}

// z[c's points] = Z_c v[members of c], one workgroup per cell: the member
// values of v gathered into LDS, then Z_c streamed once from HBM.  Each wave
// takes four rows at a time, a 16-lane group per row (so one load instruction
// reads four 128-byte row segments), four independent loads per lane in
// flight, and one 16-lane reduction per row.  FP32 rows accumulate with Kahan
// compensation.
template <typename T>
__device__ __forceinline__ double row_dot(const T* __restrict__ zr, const T* vs, int n_omega,
                                          int ph) {
    if (sizeof(T) == 8) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int q = ph;
        for (; q + 48 < n_omega; q += 64) {
            const double z0 = zr[q], z1 = zr[q + 16], z2 = zr[q + 32], z3 = zr[q + 48];
            a0 = __builtin_fma(z0, (double)vs[q], a0);
            a1 = __builtin_fma(z1, (double)vs[q + 16], a1);
            a2 = __builtin_fma(z2, (double)vs[q + 32], a2);
            a3 = __builtin_fma(z3, (double)vs[q + 48], a3);
        }
        for (; q < n_omega; q += 16) a0 = __builtin_fma((double)zr[q], (double)vs[q], a0);
        return (a0 + a1) + (a2 + a3);
    } else {
        Kahan32 a0, a1;
        int q = ph;
        for (; q + 16 < n_omega; q += 32) {
            const float z0 = (float)zr[q], z1 = (float)zr[q + 16];
            a0.add(z0 * (float)vs[q]);
            a1.add(z1 * (float)vs[q + 16]);
        }
        for (; q < n_omega; q += 16) a0.add((float)zr[q] * (float)vs[q]);
        return a0.value() + a1.value();
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_rasm_apply(PrecondArgs a, const T* __restrict__ Z,
                                                         const double* __restrict__ v,
                                                         double* __restrict__ z) {
    __shared__ T vs[RBF_MAX_BLOCK];
    __shared__ int rb[kMaxRanges], re[kMaxRanges];
    __shared__ int nr_s, n_omega_s, n_c_s;
    const long long c = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid == 0) block_ranges(a.cell_start, a.g, a.overlap, c, rb, re, &nr_s, &n_omega_s, &n_c_s);
    __syncthreads();
    const int n_omega = n_omega_s, n_c = n_c_s, nr = nr_s;
    if (n_c == 0) return;
    for (int k = tid; k < n_omega; k += kThreads) vs[k] = (T)v[member_index(rb, re, nr, k)];
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int grp = lane >> 4, ph = lane & 15;
    const T* Zc = Z + a.zoff[c];
    const int own = a.cell_start[c];
    for (int r0 = 4 * wave; r0 < n_c; r0 += 4 * (kThreads / 64)) {
        const int r = r0 + grp;
        double sum = 0.0;
        if (r < n_c) sum = row_dot<T>(Zc + (size_t)r * n_omega, vs, n_omega, ph);
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) sum += __shfl_xor(sum, o, RBF_WAVE);
        if (ph == 0 && r < n_c) z[own + r] = sum;
    }
}

}  // namespace

hipError_t launch_precond_setup64(const PrecondArgs& a, double* Z, double* scratch, int nslots,
                                  int4* meta, double* lt, int* status, hipStream_t st) {
    const int pad = (nslots + 7) / 8 * 8;
    const int ncp = (a.nc_max + kZCols - 1) / kZCols;
    double* lt_buf[2] = {lt, lt + (size_t)pad * kNB * kNB};
    for (long long c0 = 0; c0 < a.ncells; c0 += nslots) {
        k_setup_assemble_f64<<<pad, kT2, 0, st>>>(a, c0, nslots, scratch, meta, status, lt_buf[0]);
        for (int J = 0; J + kNB < a.np_max; J += kNB) {
            const int tiles = (a.np_max - J - kNB + kRows2 - 1) / kRows2;
            const int b = (J / kNB) & 1;
            k_chol_step<<<pad * tiles, kTS, 0, st>>>(a, c0, J, pad, scratch, meta, status,
                                                     lt_buf[b], lt_buf[b ^ 1]);
        }
        if (ncp > 0) {
            k_z_forward<<<pad * ncp, kT2, 0, st>>>(a, c0, pad, scratch, meta, Z);
            for (int I = a.np_max / kNB - 1; I >= 0; --I)
                k_z_back<<<pad * ncp, kZT, 0, st>>>(a, c0, I, pad, scratch, meta, Z);
        }
    }
    return hipGetLastError();
}

hipError_t launch_precond_setup32(const PrecondArgs& a, float* Z, float* scratch, int nslots,
                                  int* status, hipStream_t st) {
    k_precond_setup<float><<<nslots, kThreads, 0, st>>>(a, Z, scratch, status);
    return hipGetLastError();
}

hipError_t launch_rasm_apply64(const PrecondArgs& a, const double* Z, const double* v, double* z,
                               hipStream_t st) {
    k_rasm_apply<double><<<(unsigned)a.ncells, kThreads, 0, st>>>(a, Z, v, z);
    return hipGetLastError();
}

hipError_t launch_rasm_apply32(const PrecondArgs& a, const float* Z, const double* v, double* z,
                               hipStream_t st) {
    k_rasm_apply<float><<<(unsigned)a.ncells, kThreads, 0, st>>>(a, Z, v, z);
    return hipGetLastError();
}

}  // namespace rbf
