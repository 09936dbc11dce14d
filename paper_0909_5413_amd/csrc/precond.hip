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
// FP64 setup on the matrix cores.  Two 256-thread workgroups per CU, each
// holding one cell's matrix at a time (n_p x n_p, lower triangle, ROW-major:
// element (i, j) at A[i * n_p + j], so every row segment is contiguous) in a
// private global scratch; the two workgroups hide each other's memory stalls.
// The block-column update of the left-looking Cholesky and the substitution
// products of the inverse rows run as v_mfma_f64_16x16x4f64 tiles fed from LDS
// panels, the next panel being loaded into registers while the current one is
// multiplied.  Operand layout of that instruction on gfx950: lane l holds
// A[l%16][l/16] and B[l/16][l%16]; the four result registers v hold
// D[l/16 + 4v][l%16].
// ===========================================================================
typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int kT2 = 256;        // threads (4 waves)
constexpr int kW2 = kT2 / 64;
constexpr int kKC2 = 8;         // k per LDS panel in the update
constexpr int kRows2 = 256;     // rows per super-block of the update
constexpr int kRT2 = kRows2 / 16 / kW2;   // row tiles per wave (8)
constexpr int kRPT = kRows2 / kT2;        // panel rows loaded per thread (2)
static_assert(kRows2 % kT2 == 0, "row super-block must split evenly");
constexpr int kZK = 64;         // k per LDS panel in the inverse-row products

struct SetupLds2 {
    union {
        struct {
            double P[kKC2][kRows2];      // rows of the panel, k-major
            double Pb[kKC2][kNB];        // the block column's own rows
        } g;
        struct {
            double X[kNB][kT2];          // rows being solved, one column per thread
        } t;
        struct {
            double Lc[kZK][kNB + 1];
            double Xc[kZK][kZCols + 1];
            double acc[kNB][kZCols + 1];
        } z;
        struct {
            double mx[RBF_MAX_BLOCK];
            double my[RBF_MAX_BLOCK];
        } coords;
    } u;
    double D[kNB][kNB + 1];
    double invd[kNB];
    int rb[kMaxRanges], re[kMaxRanges];
    int nranges, n_omega, n_c, flag;
};

__device__ __forceinline__ double readlane_d(double v, int lane) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ d4v mfma_f64(double a, double b, d4v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// A[rows R.., cols J..J+31] -= L[rows, 0:J] L[J..J+31, 0:J]^T for one row
// super-block (MFMA tiles; J > 0).  The tiles of rows J..J+31 also go to s.D.
// No LDS and no barriers: the contraction index of an MFMA may be permuted as
// long as A and B use the same permutation, so over a chunk of 16 k values lane
// group g = l/16 owns k = K+4g .. K+4g+3 and loads them from its row with one
// 32-byte load; step s of the chunk uses element s.  Each wave loads its own
// row tiles and both column tiles (the latter shared through the caches), and
// the next chunk is loaded while the current one is multiplied.
struct d4pack {
    d4v a[kRT2];
    d4v b[2];
};

__device__ __forceinline__ d4v load4(const double* __restrict__ p) {
    return *reinterpret_cast<const d4v*>(p);
}

__device__ void update_block_column(double* __restrict__ A, int np, int J, int R,
                                    SetupLds2& s) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i16 = lane & 15, g = lane >> 4;
    const int nrow = np - R < kRows2 ? np - R : kRows2;   // multiple of 32
    const int ntile = nrow / 16;
    d4v acc[kRT2][2];
#pragma unroll
    for (int t = 0; t < kRT2; ++t) acc[t][0] = acc[t][1] = d4v{0.0, 0.0, 0.0, 0.0};
    // row pointers (offset by this lane's k group)
    const double* arow[kRT2];
#pragma unroll
    for (int t = 0; t < kRT2; ++t) {
        const int tile = wave + kW2 * t;
        const int row = R + 16 * (tile < ntile ? tile : 0) + i16;
        arow[t] = A + (size_t)row * np + 4 * g;
    }
    const double* brow0 = A + (size_t)(J + i16) * np + 4 * g;
    const double* brow1 = A + (size_t)(J + 16 + i16) * np + 4 * g;
    d4pack cur, nxt;
    auto load = [&](d4pack& d, int K) {
#pragma unroll
        for (int t = 0; t < kRT2; ++t)
            if (wave + kW2 * t < ntile) d.a[t] = load4(arow[t] + K);
        d.b[0] = load4(brow0 + K);
        d.b[1] = load4(brow1 + K);
    };
    const int nchunk = J / 16;   // J is a multiple of 32
    load(cur, 0);
    for (int ch = 0; ch < nchunk; ++ch) {
        if (ch + 1 < nchunk) load(nxt, 16 * (ch + 1));
#pragma unroll
        for (int st = 0; st < 4; ++st) {
#pragma unroll
            for (int t = 0; t < kRT2; ++t) {
                if (wave + kW2 * t < ntile) {
                    acc[t][0] = mfma_f64(cur.a[t][st], cur.b[0][st], acc[t][0]);
                    acc[t][1] = mfma_f64(cur.a[t][st], cur.b[1][st], acc[t][1]);
                }
            }
        }
        cur = nxt;
    }
#pragma unroll
    for (int t = 0; t < kRT2; ++t) {
        const int tile = wave + kW2 * t;
        if (tile < ntile) {
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rl = 16 * tile + g + 4 * v;
                    const int col = 16 * cb + i16;
                    double* ad = A + (size_t)(R + rl) * np + J + col;
                    const double nv = *ad - acc[t][cb][v];
                    *ad = nv;
                    if (R == J && rl < kNB) s.D[rl][col] = nv;
                }
        }
    }
}

// Factor the 32x32 diagonal block (in s.D) in wave 0's registers (lane i holds
// row i; broadcasts by readlane, no barriers), write it back and keep it in
// s.D / s.invd.  Returns 0 or the failing 1-based pivot index (all threads).
__device__ int factor_diag_block(double* __restrict__ A, int np, int J, SetupLds2& s) {
    const int tid = threadIdx.x;
    if (tid < 64) {
        const int i = tid & 31;
        double r[kNB];
#pragma unroll
        for (int c = 0; c < kNB; ++c) r[c] = (c <= i) ? s.D[i][c] : 0.0;
        int bad = 0;
#pragma unroll
        for (int k = 0; k < kNB; ++k) {
            const double piv = readlane_d(r[k], k);
            if (!bad && !(piv > 0.0)) bad = k + 1;   // uniform; later values are moot
            const double lkk = __builtin_sqrt(piv);
            const double inv = 1.0 / lkk;
            r[k] = (i == k) ? lkk : r[k] * inv;
#pragma unroll
            for (int j = k + 1; j < kNB; ++j) {
                const double ljk = readlane_d(r[k], j);
                r[j] = __builtin_fma(-r[k], ljk, r[j]);
            }
        }
        if (tid == 0) s.flag = bad ? J + bad : 0;
        if (!bad && tid < kNB) {
            double* arow = A + (size_t)(J + i) * np + J;
#pragma unroll
            for (int c = 0; c < kNB; ++c) {
                if (c <= i) {
                    arow[c] = r[c];
                    s.D[i][c] = r[c];
                }
            }
            s.invd[i] = 1.0 / r[i];
        }
    }
    __syncthreads();
    return s.flag;
}

// Rows J+32 .. np-1 of block column J: x L_JJ^T = a, one row per thread, the
// row staged in LDS (column tid of s.u.t.X) and solved in 4 groups of 8.
__device__ void trsm_rows(double* __restrict__ A, int np, int J, SetupLds2& s) {
    const int tid = threadIdx.x;
    for (int r0 = J + kNB; r0 < np; r0 += kT2) {
        const int row = r0 + tid;
        double* xr = A + (size_t)row * np + J;
        if (row < np) {
            double x[kNB];
#pragma unroll
            for (int q = 0; q < kNB; ++q) x[q] = xr[q];
#pragma unroll
            for (int q = 0; q < kNB; ++q) s.u.t.X[q][tid] = x[q];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                double y[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) y[q] = s.u.t.X[8 * g + q][tid];
#pragma unroll
                for (int c = 0; c < 8 * g; ++c) {
                    const double xc = s.u.t.X[c][tid];
#pragma unroll
                    for (int q = 0; q < 8; ++q) y[q] = __builtin_fma(-xc, s.D[8 * g + q][c], y[q]);
                    __asm__ volatile("" ::: "memory");
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    y[q] = y[q] * s.invd[8 * g + q];
#pragma unroll
                    for (int q2 = q + 1; q2 < 8; ++q2)
                        y[q2] = __builtin_fma(-y[q], s.D[8 * g + q2][8 * g + q], y[q2]);
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    s.u.t.X[8 * g + q][tid] = y[q];
                    xr[8 * g + q] = y[q];
                }
                __asm__ volatile("" ::: "memory");
            }
        }
    }
}

__device__ int cholesky_mfma(double* __restrict__ A, int np, SetupLds2& s) {
    const int tid = threadIdx.x;
    for (int J = 0; J < np; J += kNB) {
        if (J > 0) {
            for (int R = J; R < np; R += kRows2) update_block_column(A, np, J, R, s);
        } else {
            for (int idx = tid; idx < kNB * kNB; idx += kT2) {
                const int i = idx / kNB, j = idx % kNB;
                if (j <= i) s.D[i][j] = A[(size_t)i * np + j];
            }
        }
        __syncthreads();
        const int f = factor_diag_block(A, np, J, s);
        if (f) return f;
        trsm_rows(A, np, J, s);
        __syncthreads();
    }
    return 0;
}

// s.u.z.acc[r][c] = rhs(r, c) - sum_k op(L)[I0 + r][k] X[k][c0 + c] over
// k in [k_lo, k_hi) (MFMA, 8 tiles of 16x16, two per wave), then the diagonal
// block L(I0.., I0..) into s.D / s.invd.
//   forward (kBackward = false): op(L)[r][k] = L[r][k], rhs = E_C
//   backward: op(L)[r][k] = L[k][r], rhs = the forward result W stored in X's
//   place (zero above row w_lo)
template <bool kBackward>
__device__ void zsolve_block(const double* __restrict__ A, int np, int I0, int k_lo, int k_hi,
                             const double* __restrict__ Zc, int ldz, int p, int c0, int ncol,
                             int q0, int w_lo, SetupLds2& s) {
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
                if (k0 + kk < k_hi) v = A[(size_t)(k0 + kk) * np + I0 + rr];
            } else {           // L[I0 + rr][k0 + kk]: contiguous in kk
                const int rr = idx / kZK, kk = idx % kZK;
                if (k0 + kk < k_hi) v = A[(size_t)(I0 + rr) * np + k0 + kk];
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
                s.u.z.Lc[idx / kNB][idx % kNB] = rl[q];
            else
                s.u.z.Lc[idx % kZK][idx / kZK] = rl[q];
        }
#pragma unroll
        for (int q = 0; q < kLX; ++q) {
            const int idx = tid + kT2 * q;
            s.u.z.Xc[idx % kZK][idx / kZK] = rx[q];
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
                const double a = s.u.z.Lc[kr][16 * rt + (lane & 15)];
                const double b0 = s.u.z.Xc[kr][16 * ct0 + (lane & 15)];
                const double b1 = s.u.z.Xc[kr][16 * ct0 + 16 + (lane & 15)];
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
            s.u.z.acc[r][cc] = rhs - (h ? acc1[v] : acc0[v]);
        }
    }
    for (int idx = tid; idx < kNB * kNB; idx += kT2) {
        const int i = idx / kNB, j = idx % kNB;
        s.D[i][j] = A[(size_t)(I0 + i) * np + I0 + j];
    }
    __syncthreads();
    if (tid < kNB) s.invd[tid] = 1.0 / s.D[tid][tid];
    __syncthreads();
}

__device__ void centre_rows_mfma(const double* __restrict__ A, int np, int p, int n_omega,
                                 int n_c, double* __restrict__ Zc, SetupLds2& s) {
    const int tid = threadIdx.x;
    const int q0 = np - n_c;
    const int ib = q0 / kNB;
    const int nblk = np / kNB;
    for (int c0 = 0; c0 < n_c; c0 += kZCols) {
        const int ncol = n_c - c0 < kZCols ? n_c - c0 : kZCols;
        for (int I = ib; I < nblk; ++I) {
            const int I0 = I * kNB;
            zsolve_block<false>(A, np, I0, ib * kNB, I0, Zc, n_omega, p, c0, ncol, q0, 0, s);
            if (tid < ncol) {
                for (int r = 0; r < kNB; ++r) {
                    double v = s.u.z.acc[r][tid];
                    for (int r2 = 0; r2 < r; ++r2)
                        v = __builtin_fma(-s.D[r][r2], s.u.z.acc[r2][tid], v);
                    s.u.z.acc[r][tid] = v * s.invd[r];
                }
                for (int r = 0; r < kNB; ++r)
                    if (I0 + r >= p) Zc[(size_t)(c0 + tid) * n_omega + (I0 + r - p)] = s.u.z.acc[r][tid];
            }
        }
        for (int I = nblk - 1; I >= 0; --I) {
            const int I0 = I * kNB;
            if (I0 + kNB <= p) break;
            zsolve_block<true>(A, np, I0, I0 + kNB, np, Zc, n_omega, p, c0, ncol, q0, ib * kNB, s);
            if (tid < ncol) {
                for (int r = kNB - 1; r >= 0; --r) {
                    double v = s.u.z.acc[r][tid];
                    for (int r2 = r + 1; r2 < kNB; ++r2)
                        v = __builtin_fma(-s.D[r2][r], s.u.z.acc[r2][tid], v);
                    s.u.z.acc[r][tid] = v * s.invd[r];
                }
                for (int r = 0; r < kNB; ++r)
                    if (I0 + r >= p) Zc[(size_t)(c0 + tid) * n_omega + (I0 + r - p)] = s.u.z.acc[r][tid];
            }
        }
        __syncthreads();
    }
}

// The FP64 setup runs as three kernels over a batch of cells, one workgroup per
// cell and a private scratch matrix per workgroup, so that each phase gets its
// own register allocation: assemble the local matrix, factor it, form the
// centre rows of its inverse.  Cell of workgroup b: c0 + b.

struct AssembleLds {
    double mx[RBF_MAX_BLOCK];
    double my[RBF_MAX_BLOCK];
    int rb[kMaxRanges], re[kMaxRanges];
    int nranges, n_omega, n_c, flag;
};

template <typename S>
__device__ __forceinline__ bool load_cell_ranges(const PrecondArgs& a, long long c, S& s) {
    if (threadIdx.x == 0) {
        block_ranges(a.cell_start, a.g, a.overlap, c, s.rb, s.re, &s.nranges, &s.n_omega,
                     &s.n_c);
        s.flag = 0;
    }
    __syncthreads();
    return s.n_c > 0;
}

__global__ __launch_bounds__(kT2, 2) void k_setup_assemble_f64(PrecondArgs a, long long c0,
                                                               double* __restrict__ scratch) {
    __shared__ AssembleLds s;
    const long long c = c0 + blockIdx.x;
    if (c >= a.ncells) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (!load_cell_ranges(a, c, s)) return;
    const int n_omega = s.n_omega, nr = s.nranges;
    const int np = (n_omega + kNB - 1) / kNB * kNB;
    const int p = np - n_omega;
    double* A = scratch + (size_t)blockIdx.x * a.np_max * a.np_max;
    for (int k = tid; k < n_omega; k += kT2) {
        const int m = member_index(s.rb, s.re, nr, k);
        s.mx[k] = a.xs[m];
        s.my[k] = a.ys[m];
    }
    __syncthreads();
    // untruncated Gaussian, lower triangle (row-major), leading identity
    // padding; wave w fills rows w, w + 4, ...
    for (int i = wave; i < np; i += kW2) {
        double* arow = A + (size_t)i * np;
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
        }
    }
}

__global__ __launch_bounds__(kT2, 2) void k_setup_factor_f64(PrecondArgs a, long long c0,
                                                             double* __restrict__ scratch,
                                                             int* __restrict__ status) {
    __shared__ SetupLds2 s;
    const long long c = c0 + blockIdx.x;
    if (c >= a.ncells) return;
    if (!load_cell_ranges(a, c, s)) {
        if (threadIdx.x == 0) status[c] = 0;
        return;
    }
    const int np = (s.n_omega + kNB - 1) / kNB * kNB;
    double* A = scratch + (size_t)blockIdx.x * a.np_max * a.np_max;
    const int fail = cholesky_mfma(A, np, s);
    if (threadIdx.x == 0) status[c] = fail;
}

__global__ __launch_bounds__(kT2, 2) void k_setup_centre_rows_f64(PrecondArgs a, long long c0,
                                                                  double* __restrict__ Z,
                                                                  const double* __restrict__ scratch,
                                                                  const int* __restrict__ status) {
    __shared__ SetupLds2 s;
    const long long c = c0 + blockIdx.x;
    if (c >= a.ncells || status[c] != 0) return;
    if (!load_cell_ranges(a, c, s)) return;
    const int n_omega = s.n_omega, n_c = s.n_c;
    const int np = (n_omega + kNB - 1) / kNB * kNB;
    const double* A = scratch + (size_t)blockIdx.x * a.np_max * a.np_max;
    centre_rows_mfma(A, np, np - n_omega, n_omega, n_c, Z + a.zoff[c], s);
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
    const T* Zc = Z + a.zoff[c];
    const int own = a.cell_start[c];
    for (int r = wave; r < n_c; r += kThreads / 64) {
        const T* zr = Zc + (size_t)r * n_omega;
        double sum;
        if (sizeof(T) == 8) {
            double acc = 0.0;
            for (int q = lane; q < n_omega; q += 64)
                acc = __builtin_fma((double)zr[q], (double)vs[q], acc);
            sum = wave_sum(acc);
        } else {
            Kahan32 acc;
            for (int q = lane; q < n_omega; q += 64) acc.add((float)zr[q] * (float)vs[q]);
            sum = wave_sum(acc.value());
        }
        if (lane == 0) z[own + r] = sum;
    }
}

}  // namespace

hipError_t launch_precond_setup64(const PrecondArgs& a, double* Z, double* scratch, int nslots,
                                  int* status, hipStream_t st) {
    for (long long c0 = 0; c0 < a.ncells; c0 += nslots) {
        const long long left = a.ncells - c0;
        const unsigned grid = (unsigned)(left < nslots ? left : nslots);
        k_setup_assemble_f64<<<grid, kT2, 0, st>>>(a, c0, scratch);
        k_setup_factor_f64<<<grid, kT2, 0, st>>>(a, c0, scratch, status);
        k_setup_centre_rows_f64<<<grid, kT2, 0, st>>>(a, c0, Z, scratch, status);
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
