// precond.hip -- restricted additive Schwarz preconditioner on gfx950.
//
// RASM (Section 2.2, eq. rasm): z = sum_c Rt_c^T A_c^{-1} R_c v.  Cell c is the
// non-overlapping subdomain; its overlapping subdomain is the (2*overlap+1)^2
// block of cells around it.  Only the rows of A_c^{-1} that belong to c's own
// points are ever used, so setup stores exactly those: Z_c = (A_c^{-1})[centre
// rows, :], an n_c x n_omega block, and every application is one batched
// gather-GEMV z[c's points] = Z_c v[members of c].
//
// Setup, for every cell:
//  1. members: neighbour cells in (dy, dx) order, each a contiguous sorted
//     range, the cell's own points last; padded to n_p = 64 * ceil(n/64) by
//     leading identity rows so every block boundary is aligned;
//  2. A_c[p][q] = phi(|x_p - x_q|), the untruncated normalised Gaussian;
//  3. A_c = L L^T by a left-looking blocked Cholesky (64-column block columns);
//  4. X = A_c^{-1} E_C (E_C = the centre columns of the identity) by a blocked
//     forward solve L W = E_C on the trailing rows only, then a blocked back
//     solve L^T X = W; X's columns, without the padding rows, are Z_c's rows
//     and are written straight into the Z buffer.
// The same kernels run in FP64 and, for the mixed-precision form, in FP32
// (assembly in FP64, rounded once); an FP32 block whose factorisation meets a
// non-positive pivot is rebuilt with a diagonal shift mu = s * n * u32 *
// phi(0), s in {1, 10, 100, 1000} (shifted low-precision Cholesky).
#include <vector>

#include "rbf_device.hpp"
#include "rbf_internal.hpp"
#include "../../include/rbf.h"

namespace rbf {

namespace {

constexpr int kNB = 32;        // block size of the factorisation
constexpr int kThreads = 256;
constexpr int kMaxRanges = 2 * 16 + 3;
constexpr int kZCols = 64;     // right-hand-side columns per pass of the solves

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


// ===========================================================================
// Setup on the matrix cores, batched in lockstep.  Each cell of a batch (a
// slot) keeps its n_p x n_p lower triangle in a scratch slot, stored by
// 32-row block rows (see roff).  The left-looking blocked Cholesky advances one
// 64-column block column J at a time for every slot together, one launch per
// J: each workgroup takes a 64-row tile below the diagonal block, updates it
// with the finished block columns as MFMA tiles (accumulators in registers),
// solves x L_JJ^T = a for its rows in two 32-column halves (substitution, one
// row per thread, the diagonal blocks broadcast from LDS; the coupling block on
// MFMA), and writes the rows back.  A second launch then forms and factors the
// next 64x64 diagonal block of every slot, one small single-wave workgroup
// each.  64 columns per step halve the re-reads of the finished columns that
// a left-looking update makes, against 32.  The centre rows of the inverse follow: one
// launch for the forward solve on the trailing rows, one launch per block row
// of the back solve.  Every launch carries thousands of independent
// workgroups, so one cell's serial steps overlap with other cells' work.
// Workgroup b serves slot b % nslots_pad (a multiple of 8; the step launch
// orders its tiles differently, with the same slot-to-XCD map): a slot's
// workgroups run on one XCD in every launch, and its rows stay in that XCD's
// L2 from launch to launch.
// MFMA tiles are 16x16x4 (v_mfma_f64_16x16x4f64, v_mfma_f32_16x16x4f32).  On
// gfx950 both take lane l's operands as A[l%16][l/16] and B[l/16][l%16]; result
// register v of lane l holds D[r][l%16] with r = l/16 + 4v (FP64) or
// r = 4(l/16) + v (FP32).
// ===========================================================================
template <typename T> struct Vec;
template <> struct Vec<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    typedef double v2 __attribute__((ext_vector_type(2)));
};
template <> struct Vec<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    typedef float v2 __attribute__((ext_vector_type(2)));
};
template <typename T> using v4 = typename Vec<T>::v4;
template <typename T> using v2 = typename Vec<T>::v2;

__device__ __forceinline__ v4<double> mfma(double a, double b, v4<double> c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4<float> mfma(float a, float b, v4<float> c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// row (within its 16x16 tile) of result register v of lane group g
template <typename T>
__device__ __forceinline__ constexpr int out_row(int g, int v) {
    return sizeof(T) == 8 ? g + 4 * v : 4 * g + v;
}

template <typename T>
__device__ __forceinline__ v4<T> load4(const T* __restrict__ p) {
    return *reinterpret_cast<const v4<T>*>(p);
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

__device__ __forceinline__ double readlane_t(double v, int lane) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane_t(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// 1/sqrt(x): hardware estimate refined by Newton steps
__device__ __forceinline__ double rsqrt_t(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * __builtin_fma(-0.5 * x * y, y, 1.5);
    return y * __builtin_fma(-0.5 * x * y, y, 1.5);
}
__device__ __forceinline__ float rsqrt_t(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    return y * __builtin_fmaf(-0.5f * x * y, y, 1.5f);
}

constexpr int kT2 = 256;        // threads of the assembly and forward-solve kernels (4 waves)
constexpr int kW2 = kT2 / 64;
constexpr int kFB = 2 * kNB;    // columns of a factorisation block column; n_p is a multiple
constexpr int kTS = 256;        // threads of a factorisation step (4 waves)
constexpr int kWS = kTS / 64;
// Rows per step tile: one 16-row MFMA tile per wave.  Small tiles keep the
// step kernel near 128 registers, so four workgroups share a CU (its LDS is
// the limit) and cover each other's latency.
constexpr int kRows = 64;
static_assert(kRows <= kTS, "the substitution gives one row to each thread");
static_assert(kRows == 16 * kWS, "one row tile per wave");
// LDS row of a step tile's column: odd (conflict-free MFMA stores), and long
// enough for the update's two staged chunks, which borrow the tile buffer
constexpr int kXS = 81;
constexpr int kTileGroup = 16;  // slots whose step tiles are interleaved on an XCD
constexpr int kTri = kNB * (kNB + 1) / 2;
constexpr int kLtElems = 2 * kNB * kNB;   // per slot: both diagonal 32x32 blocks of L_JJ

// Index of (k, j), j >= k, in the packed upper triangle of a 32x32 block.
__host__ __device__ constexpr int tri(int k, int j) { return kNB * k - k * (k - 1) / 2 + (j - k); }
constexpr int kZK = 64;         // k per LDS panel in the forward solve

// Block-row storage of a slot's lower triangle: the 32 rows of block row I are
// stored with stride 32 (I + 1) (their columns up to the end of the diagonal
// block), block rows one after another, so every row starts on a 32-element
// boundary and a slot needs 512 B (B + 1) elements for B block rows.
__device__ __forceinline__ size_t roff(int row) {
    const int I = row >> 5;
    return (size_t)(32 * (I + 1)) * (size_t)(16 * I + (row & 31));
}


// The update of a step tile: acc[t][cb] += sum_{k0 <= k < J} L[row][k] L[J + 16 cb + col][k]
// for the wave's row tiles t (rows R + 16 (wave + 4 t) ..) and the four 16-column
// tiles of the block column, as MFMA tiles.  The contraction index of an MFMA
// may be permuted as long as A and B use the same permutation, so over a chunk
// of 16 k values lane group g = l/16 owns k = K+4g .. K+4g+3 and loads them
// from its row with one vector load; step s of the chunk uses element s.  Each
// wave loads its own M row tiles straight into registers (two register
// buffers: the next chunk in flight while one is multiplied).  The 64 block rows
// J .. J + 63, which every wave multiplies with, are loaded once per workgroup
// (one vector load per thread and chunk, a chunk ahead) into an LDS buffer of
// two chunks, where each wave reads its operands; one barrier per chunk.  Six
// chunks per loop pass keep every buffer index a constant.  Columns below k0
// are zero in every row involved (leading identity padding) and are skipped.
// A staged chunk row of 16 values is padded to 18 doubles (20 floats), so rows
// start 16 bytes apart modulo 128 and the 16 rows a read instruction touches
// spread over the LDS banks; every row start stays 16-byte aligned.
template <typename T>
constexpr int kBS = sizeof(T) == 8 ? 18 : 20;

template <typename T, int M>
struct StepUpdate {
    static_assert(2 * 64 * kBS<T> <= kNB * kXS, "two staged chunks fit in the tile buffer");
    v4<T> a[2][M];
    v4<T> acc[M][4];
    v4<T> bst;             // this thread's part of the next chunk of the block rows
    const T* arow[M];
    const T* bsrc;         // row J + tid / 4, k = k0 + 4 (tid % 4)
    T (*bs)[64][kBS<T>];   // two chunk buffers in LDS

    __device__ __forceinline__ void load_a(int buf, int ch) {
#pragma unroll
        for (int t = 0; t < M; ++t) a[buf][t] = load4(arow[t] + 16 * ch);
    }
    __device__ __forceinline__ void load_b(int ch) { bst = load4(bsrc + 16 * ch); }
    __device__ __forceinline__ void store_b(int buf) {
        const int tid = threadIdx.x;
        T* d = &bs[buf][tid >> 2][4 * (tid & 3)];
        *reinterpret_cast<v2<T>*>(d) = v2<T>{bst[0], bst[1]};
        *reinterpret_cast<v2<T>*>(d + 2) = v2<T>{bst[2], bst[3]};
    }
    __device__ __forceinline__ void mma(int ba, int bb) {
        const int lane = threadIdx.x & 63;
        const int i16 = lane & 15, g = lane >> 4;
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            T b[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) b[cb] = bs[bb][16 * cb + i16][4 * g + st];
#pragma unroll
            for (int t = 0; t < M; ++t) {
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    acc[t][cb] = mfma(a[ba][t][st], b[cb], acc[t][cb]);
            }
        }
    }
    // chunks c .. c + min(R, 6) - 1; on entry chunk c of A is in a[0], chunk c
    // of the block rows in bs[0] and chunk c + 1 in bst (c is a multiple of 6);
    // no load reaches c + R
    template <int R>
    __device__ __forceinline__ void run(int c) {
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            if (i < R) {
                if (i + 1 < R) load_a((i + 1) % 2, c + i + 1);
                mma(i % 2, i % 2);
                if (i + 1 < R) {
                    store_b((i + 1) % 2);
                    if (i + 2 < R) load_b(c + i + 2);
                }
                __syncthreads();
            }
        }
    }
    // the first loads of the update (J > 0)
    __device__ __forceinline__ void prologue(const T* __restrict__ A, int J, int k0, int R,
                                             int wave, T* lds) {
        const int tid = threadIdx.x, lane = tid & 63;
        const int i16 = lane & 15, g = lane >> 4;
        bs = reinterpret_cast<T (*)[64][kBS<T>]>(lds);
#pragma unroll
        for (int t = 0; t < M; ++t) arow[t] = A + roff(R + 16 * (wave + kWS * t) + i16) + k0 + 4 * g;
        bsrc = A + roff(J + (tid >> 2)) + k0 + 4 * (tid & 3);
        load_a(0, 0);
        load_b(0);
    }
    // acc[t][cb] += the products over (J - k0) / 16 chunks (J > 0; after the
    // prologue; the caller initialises acc).  The chunk buffers borrow the
    // tile's LDS buffer, which is free again after the last chunk's barrier.
    __device__ __forceinline__ void update(int J, int k0) {
        const int nchunk = (J - k0) / 16;   // >= 2, even
        store_b(0);
        load_b(1);
        __syncthreads();
        int c = 0;
        for (; c + 8 <= nchunk; c += 6) run<99>(c);
        const int rest = nchunk - c;   // 2, 4 or 6
        if (rest == 2)
            run<2>(c);
        else if (rest == 4)
            run<4>(c);
        else
            run<6>(c);
    }
};

// X[c][r] = A[R + r][J + c] (coalesced pair loads), r < nrow.
template <typename T>
__device__ void load_tile(const T* __restrict__ A, int J, int R, int nrow, T (*X)[kXS]) {
    for (int id = threadIdx.x; id < nrow * (kNB / 2); id += kTS) {
        const int r = id / (kNB / 2), c = 2 * (id % (kNB / 2));
        const v2<T> v = *reinterpret_cast<const v2<T>*>(A + roff(R + r) + J + c);
        X[c][r] = v[0];
        X[c + 1][r] = v[1];
    }
}

// A[R + r][J + c] = X[c][r] (coalesced pair stores), r < nrow.
template <typename T>
__device__ void store_tile(T* __restrict__ A, int J, int R, int nrow, T (*X)[kXS]) {
    for (int id = threadIdx.x; id < nrow * (kNB / 2); id += kTS) {
        const int r = id / (kNB / 2), c = 2 * (id % (kNB / 2));
        v2<T> v;
        v[0] = X[c][r];
        v[1] = X[c + 1][r];
        *reinterpret_cast<v2<T>*>(A + roff(R + r) + J + c) = v;
    }
}

// Rows of the tile: x L_DD^T = a in place (thread tid: column tid of X) for
// a 32x32 diagonal block D of L_JJ, split at column 16: the first 16 columns
// by substitution (column by column, 15 - k independent FMAs at step k), the
// last 16 updated by one MFMA pass, x[16..31] -= x[0..15] L[16..31][0..15]^T
// (each wave its row tiles), then their substitution.  Lt holds L_DD
// transposed and packed (Lt[tri(k, j)] = L[j][k], j > k) with the reciprocal
// pivots on its diagonal; every lane reads the same Lt entries (LDS
// broadcasts).  Ends with a barrier.
template <typename T, int M>
__device__ __forceinline__ void trsm_tile(const T* Lt, int wave, T (*X)[kXS]) {
    constexpr int nrow = 16 * kWS * M, kH = kNB / 2;
    const int tid = threadIdx.x, lane = tid & 63, i16 = lane & 15, g = lane >> 4;
    if (tid < nrow) {
        T x[kH];
#pragma unroll
        for (int q = 0; q < kH; ++q) x[q] = X[q][tid];
#pragma unroll
        for (int k = 0; k < kH; ++k) {
            x[k] *= Lt[tri(k, k)];
#pragma unroll
            for (int j = k + 1; j < kH; ++j) x[j] = fma_t(-x[k], Lt[tri(k, j)], x[j]);
        }
#pragma unroll
        for (int q = 0; q < kH; ++q) X[q][tid] = x[q];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < M; ++t) {
        const int rt = wave + kWS * t;
        v4<T> d = {0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < kH / 4; ++s4) {
            const int k = 4 * s4 + g;
            d = mfma(X[k][16 * rt + i16], Lt[tri(k, kH + i16)], d);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) X[kH + i16][16 * rt + out_row<T>(g, v)] -= d[v];
    }
    __syncthreads();
    if (tid < nrow) {
        T x[kH];
#pragma unroll
        for (int q = 0; q < kH; ++q) x[q] = X[kH + q][tid];
#pragma unroll
        for (int k = 0; k < kH; ++k) {
            x[k] *= Lt[tri(kH + k, kH + k)];
#pragma unroll
            for (int j = k + 1; j < kH; ++j) x[j] = fma_t(-x[k], Lt[tri(kH + k, kH + j)], x[j]);
        }
#pragma unroll
        for (int q = 0; q < kH; ++q) X[kH + q][tid] = x[q];
    }
    __syncthreads();
}

// Factor the 64x32 panel at J0 (rows J0 .. J0 + 63, columns J0 .. J0 + 31):
// its top 32x32 block Dt (lower part) is the diagonal block, its bottom block
// Db (NULL: a 32x32 block alone) the rows below.  Wave 0's registers, lane i
// holding panel row i; broadcasts by readlane, no barriers.  Step k: the pivot,
// its reciprocal square root, column k of L written to A, to Dt / Db (below
// the diagonal; the reciprocal pivot on it) and, for the diagonal block,
// transposed with the reciprocal pivot on the diagonal, to Lt (full 32x32
// layout, column k at Lt[k * 32 ..]), then the rank-1 update of the rows
// below, bottom rows included.  Returns 0 or J0 + the failing 1-based pivot
// index (all threads).
template <typename T>
__device__ __forceinline__ int factor_panel(T* __restrict__ A, int J0, T (*Dt)[kNB + 1],
                                            T (*Db)[kNB + 1], int* flag, T* __restrict__ Lt) {
    const int tid = threadIdx.x;
    if (tid < 64) {
        const bool top = tid < kNB;
        const bool own = top || Db != nullptr;
        const int i = tid & 31;
        T* arow = A + roff(J0 + (top ? i : kNB + i)) + J0;
        T r[kNB];
#pragma unroll
        for (int c = 0; c < kNB; ++c)
            r[c] = top ? ((c <= i) ? Dt[i][c] : T(0)) : (Db ? Db[i][c] : T(0));
        int bad = 0;
#pragma unroll
        for (int k = 0; k < kNB; ++k) {
            const T piv = readlane_t(r[k], k);
            if (!bad && !(piv > T(0))) bad = k + 1;   // uniform; later values are moot
            const T y = rsqrt_t(piv);
            const T l = (top && i == k) ? piv * y : r[k] * y;
            r[k] = l;
#pragma unroll
            for (int j = k + 1; j < kNB; ++j) {
                r[j] = fma_t(-l, readlane_t(l, j), r[j]);
                // the update happens here, not where r[j] is next read: the
                // broadcast values stay short-lived (no SGPR spills)
                __asm__ volatile("" : "+v"(r[j]));
            }
            if (own && (!top || i >= k)) {
                arow[k] = l;
                if (top) {
                    const T lk = (i == k) ? y : l;
                    Lt[k * kNB + i] = lk;
                    Dt[i][k] = lk;
                } else {
                    Db[i][k] = l;
                }
            }
        }
        if (tid == 0) *flag = bad ? J0 + bad : 0;
    }
    __syncthreads();
    return *flag;
}

// The 64x64 diagonal block L_JJ at J0 from D = A_JJ - (finished columns),
// held as its three lower 32x32 blocks: the panel [D11; D21] factored in one
// pass (L11, L21), D22 -= L21 L21^T on MFMA, D22 factored.  L_JJ goes to A;
// lt receives the two diagonal blocks transposed with reciprocal pivots
// (lt[0 .. 1023] and lt[1024 .. 2047], full layout).  Any block size >= 64
// threads; wave 0 works.  Returns 0 or J0 + the failing 1-based pivot index
// (all threads).
template <typename T>
struct Diag64 {
    T D11[kNB][kNB + 1], D21[kNB][kNB + 1], D22[kNB][kNB + 1];
    int flag;
};

// Diagonal shift mu of the FP32 retry levels (level 0: none).
__device__ __forceinline__ double diag_shift(int level, int n_omega, double norm) {
    if (level <= 0) return 0.0;
    const double mult = level == 1 ? 1.0 : level == 2 ? 10.0 : level == 3 ? 100.0 : 1000.0;
    return mult * (double)n_omega * 0x1p-24 * norm;
}

// phi(|x_i - x_j|) in FP64 (plus the shift on the diagonal), rounded once to T.
template <typename T>
__device__ __forceinline__ T gauss_entry(double2 pi, double2 pj, bool diag, double mk, double norm,
                                         double shift) {
    const double dx = pi.x - pj.x, dy = pi.y - pj.y;
    double v = exp_neg(__builtin_fma(dx, dx, dy * dy) * mk) * norm;
    if (diag) v += shift;
    return (T)v;
}

// Entry (i, j) of a slot's padded local matrix: the leading p rows and
// columns are the identity, the rest the Gaussian on the members, whose
// coordinates xy holds in padded order.  The matrix is never stored: every
// kernel that needs an entry evaluates it with this function, so all see the
// same value.
template <typename T>
__device__ __forceinline__ T a_entry(const double2* __restrict__ xy, int p, int i, int j, double mk,
                                     double norm, double shift) {
    if (i < p || j < p) return (i == j) ? T(1) : T(0);
    return gauss_entry<T>(xy[i], xy[j], i == j, mk, norm, shift);
}

template <typename T>
struct StepLds;

// Entry (R + rl, J + c) of a slot's padded local matrix, J + c < R, from the
// coordinates a step tile staged in LDS (same value as a_entry).
template <typename T>
__device__ __forceinline__ T lds_entry(const StepLds<T>& s, int p, int R, int J, int rl, int c,
                                       double mk, double norm) {
    if (J + c < p) return T(0);
    return gauss_entry<T>(s.xr[rl], s.xc[c], false, mk, norm, 0.0);
}

template <typename T>
struct StepLds {
    T X[kNB][kXS];            // 32 columns of the tile's rows, one column per thread
    T Lt1[kTri], Lt2[kTri];   // diagonal 32x32 blocks of L_JJ transposed (packed), reciprocal pivots
    T L21[kNB][kNB + 1];      // L21[j][k] = L[J + 32 + j][J + k]
    double2 xr[kRows];        // member coordinates of the tile's rows
    double2 xc[kFB];          // and of the block column's 64 columns
};

template <typename T>
__device__ __forceinline__ void diag64_put(Diag64<T>& d, int r, int c, T v) {
    if (r < kNB)
        d.D11[r][c] = v;
    else if (c < kNB)
        d.D21[r - kNB][c] = v;
    else
        d.D22[r - kNB][c - kNB] = v;
}

template <typename T>
__device__ int factor_diag64(T* __restrict__ A, int J0, Diag64<T>& d, T* __restrict__ lt) {
    const int tid = threadIdx.x;
    const int f1 = factor_panel<T>(A, J0, d.D11, d.D21, &d.flag, lt);
    if (tid < 64) {
        const int i16 = tid & 15, g = tid >> 4;
        v4<T> t00 = {0, 0, 0, 0}, t10 = t00, t11 = t00;
#pragma unroll
        for (int s8 = 0; s8 < kNB / 4; ++s8) {
            const int k = 4 * s8 + g;
            const T a0 = d.D21[i16][k], a1 = d.D21[16 + i16][k];
            t00 = mfma(a0, a0, t00);
            t10 = mfma(a1, a0, t10);
            t11 = mfma(a1, a1, t11);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = out_row<T>(g, v);
            d.D22[r][i16] -= t00[v];
            d.D22[16 + r][i16] -= t10[v];
            d.D22[16 + r][16 + i16] -= t11[v];
        }
    }
    __syncthreads();
    const int f2 = factor_panel<T>(A, J0 + kNB, d.D22, nullptr, &d.flag, lt + kNB * kNB);
    return f1 ? f1 : f2;
}

template <typename T>
struct ZLds {
    T Lc[kZK][kNB + 1];
    T Xc[kZK][kZCols + 1];
    T acc[kNB][kZCols + 1];
    T D[kNB][kNB + 1];
    T invd[kNB];
};

// Forward solve block row I0 of L W = E_C: s.acc[r][c] = E_C(I0 + r, c0 + c)
// - sum_{k in [k_lo, k_hi)} L[I0 + r][k] W[k][c0 + c] (MFMA, 8 tiles of 16x16,
// two per wave, over LDS panels), then the diagonal block L(I0.., I0..) into
// s.D / s.invd.  W(k, c) lives at Zc[c * ldz + k - p].
template <typename T>
__device__ void zsolve_forward(const T* __restrict__ A, int I0, int k_lo, int k_hi,
                               const T* __restrict__ Zc, int ldz, int p, int c0, int ncol,
                               int q0, ZLds<T>& s) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rt = wave >> 1, ct0 = 2 * (wave & 1);
    v4<T> acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    const int nchunk = (k_hi - k_lo + kZK - 1) / kZK;
    constexpr int kLL = kZK * kNB / kT2;      // 8 L values per thread
    constexpr int kLX = kZK * kZCols / kT2;   // 16 W values per thread
    static_assert(kZK * kNB % kT2 == 0 && kZK * kZCols % kT2 == 0, "panels split evenly");
    T rl[kLL], rx[kLX];
    auto load = [&](int chunk) {
        const int k0 = k_lo + chunk * kZK;
#pragma unroll
        for (int q = 0; q < kLL; ++q) {
            const int idx = tid + kT2 * q;
            const int rr = idx / kZK, kk = idx % kZK;   // L[I0 + rr][k0 + kk]: contiguous in kk
            rl[q] = (k0 + kk < k_hi) ? A[roff(I0 + rr) + k0 + kk] : T(0);
        }
#pragma unroll
        for (int q = 0; q < kLX; ++q) {
            const int idx = tid + kT2 * q;
            const int cc = idx / kZK, kk = idx % kZK;
            const int k = k0 + kk;
            rx[q] = (cc < ncol && k < k_hi && k >= p) ? Zc[(size_t)(c0 + cc) * ldz + (k - p)] : T(0);
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < kLL; ++q) {
            const int idx = tid + kT2 * q;
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
                const T av = s.Lc[kr][16 * rt + (lane & 15)];
                const T b0 = s.Xc[kr][16 * ct0 + (lane & 15)];
                const T b1 = s.Xc[kr][16 * ct0 + 16 + (lane & 15)];
                acc0 = mfma(av, b0, acc0);
                acc1 = mfma(av, b1, acc1);
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
            const int r = 16 * rt + out_row<T>(lane >> 4, v);
            const int cc = 16 * (ct0 + h) + (lane & 15);
            const T rhs = (cc < ncol && I0 + r == q0 + c0 + cc) ? T(1) : T(0);
            s.acc[r][cc] = rhs - (h ? acc1[v] : acc0[v]);
        }
    }
    for (int idx = tid; idx < kNB * kNB; idx += kT2) {
        const int i = idx / kNB, j = idx % kNB;
        s.D[i][j] = (j <= i) ? A[roff(I0 + i) + I0 + j] : T(0);
    }
    __syncthreads();
    if (tid < kNB) s.invd[tid] = T(1) / s.D[tid][tid];
    __syncthreads();
}

// Per-slot record kept in device memory for the launches of one batch:
// x = n_p, y = n_omega, z = n_c, w = 1 while the slot's cell is being built
// (0: empty cell, beyond the last cell, or a failed pivot).
template <typename T>
struct AssembleLds {
    double2 mxy[kFB];         // coordinates of the first 64 members (padded order)
    Diag64<T> d;
    int rb[kMaxRanges], re[kMaxRanges];
    int nranges, n_omega, n_c;
};

// Slot b: members of cell c0 + b, the untruncated Gaussian on them (lower
// triangle, leading identity padding to a multiple of 64), the slot record,
// and the factor of the first 64x64 diagonal block.  status[c] becomes -level (the diagonal shift level,
// 0 for none) and turns into the failing pivot if a factorisation step fails.
// With retry set only the cells whose last attempt failed are rebuilt, one
// shift level up (FP32 only).
template <typename T>
__global__ __launch_bounds__(kT2, 2) void k_setup_assemble(PrecondArgs a, long long c0, int nslots,
                                                           int retry, T* __restrict__ scratch,
                                                           int4* __restrict__ meta,
                                                           int* __restrict__ lvl,
                                                           int* __restrict__ status,
                                                           T* __restrict__ lt_out) {
    __shared__ AssembleLds<T> s;
    const int slot = blockIdx.x;
    const long long c = c0 + slot;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (slot >= nslots || c >= a.ncells) {
        if (tid == 0) meta[slot] = int4{0, 0, 0, 0};
        return;
    }
    int level = 0;
    if (retry) {
        if (status[c] <= 0) {   // built: keep it
            if (tid == 0) meta[slot].w = 0;
            return;
        }
        level = lvl[slot] + 1;
    }
    if (tid == 0) {
        if (a.mem) {
            s.n_omega = (int)(a.moff[c + 1] - a.moff[c]);
            s.n_c = a.nown[c];
            s.nranges = 0;
        } else {
            block_ranges(a.cell_start, a.g, a.overlap, c, s.rb, s.re, &s.nranges, &s.n_omega,
                         &s.n_c);
        }
    }
    __syncthreads();
    const int n_omega = s.n_omega, n_c = s.n_c, nr = s.nranges;
    const int* mlist = a.mem ? a.mem + a.moff[c] : nullptr;
    const int np = (n_omega + kFB - 1) / kFB * kFB;
    if (tid == 0) {
        meta[slot] = int4{np, n_omega, n_c, n_c > 0 ? 1 : 0};
        lvl[slot] = level;
        status[c] = -level;
    }
    if (n_c == 0) return;
    const int p = np - n_omega;
    T* A = scratch + (size_t)slot * slot_elems64(a.np_max);
    double2* xy = a.xy + (size_t)slot * a.np_max;
    for (int k = tid; k < n_omega; k += kT2) {
        const int m = mlist ? mlist[k] : member_index(s.rb, s.re, nr, k);
        const double2 q = {a.xs[m], a.ys[m]};
        if (p + k < kFB) s.mxy[p + k] = q;
        xy[p + k] = q;
    }
    const double shift = diag_shift(level, n_omega, a.norm);
    __syncthreads();
    // the first 64x64 diagonal block (the rest of the matrix is evaluated
    // where it is used)
    for (int i = wave; i < kFB; i += kW2)
        for (int j = lane; j <= i; j += 64) {
            const T v = (i < p || j < p) ? T(i == j ? 1 : 0)
                                         : gauss_entry<T>(s.mxy[i], s.mxy[j], i == j, a.mk, a.norm,
                                                          shift);
            diag64_put<T>(s.d, i, j, v);
        }
    __syncthreads();
    const int f = factor_diag64<T>(A, 0, s.d, lt_out + (size_t)slot * kLtElems);
    if (f && tid == 0) {
        status[c] = f;
        meta[slot].w = 0;
    }
}

// Stage what the panel solve of a step tile needs in LDS: the diagonal 32x32
// blocks of L_JJ (transposed, packed, reciprocal pivots) from lt, the coupling
// block L21 from A, and the member coordinates of the tile's rows and of the
// block column.
template <typename T>
__device__ __forceinline__ void stage_step(const T* __restrict__ A, const T* __restrict__ lt,
                                           const double2* __restrict__ xy, int np, int J, int R,
                                           StepLds<T>& s) {
    const int tid = threadIdx.x;
    constexpr int kE = kNB * kNB / kTS;
    T l1[kE], l2[kE], l21[kE];
#pragma unroll
    for (int q = 0; q < kE; ++q) {
        const int e = tid + kTS * q, k = e / kNB, j = e % kNB;
        l1[q] = lt[e];
        l2[q] = lt[kNB * kNB + e];
        l21[q] = A[roff(J + kNB + k) + J + j];
    }
    const int nrow = np - R < kRows ? np - R : kRows;
    double2 xr = {0.0, 0.0}, xc = {0.0, 0.0};
    if (tid < nrow) xr = xy[R + tid];
    if (tid < kFB) xc = xy[J + tid];
#pragma unroll
    for (int q = 0; q < kE; ++q) {
        const int e = tid + kTS * q, k = e / kNB, j = e % kNB;
        if (j >= k) {
            s.Lt1[tri(k, j)] = l1[q];
            s.Lt2[tri(k, j)] = l2[q];
        }
        s.L21[k][j] = l21[q];
    }
    if (tid < nrow) s.xr[tid] = xr;
    if (tid < kFB) s.xc[tid] = xc;
}

// One step tile: rows R .. R + 16 kWS M - 1 of block column J.  The update
// (MFMA, registers: the accumulators sum L[row][k] L[col][k] over the finished
// columns), then the tile a = A - sum, its matrix entries evaluated from the
// staged coordinates, then the panel solve x L_JJ^T = a split at the middle of
// L_JJ: x1 = a1 L11^-T by substitution, a2 -= x1 L21^T on MFMA into the
// update's accumulators, x2 = a2 L22^-T; both halves pass through LDS once.
template <typename T, int M>
__device__ __forceinline__ void step_tile(T* __restrict__ A, const T* __restrict__ lt,
                                          const double2* __restrict__ xy, int np, int p,
                                          double mk, double norm, int J, int k0, int R, int wave,
                                          StepLds<T>& s) {
    constexpr int nrow = 16 * kWS * M;
    const int lane = threadIdx.x & 63;
    const int i16 = lane & 15, g = lane >> 4;
    StepUpdate<T, M> u;
#pragma unroll
    for (int t = 0; t < M; ++t)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) u.acc[t][cb] = v4<T>{0, 0, 0, 0};
    // the update's first operand loads go out before the staging loads, so
    // the two wait for memory together; the update stages its block rows in
    // s.X, which the panel solve needs only afterwards
    if (J > 0) u.prologue(A, J, k0, R, wave, &s.X[0][0]);
    stage_step<T>(A, lt, xy, np, J, R, s);
    if (J > 0) u.update(J, k0);
    __syncthreads();   // the staged blocks and coordinates
#pragma unroll
    for (int t = 0; t < M; ++t)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rl = 16 * (wave + kWS * t) + out_row<T>(g, v);
                const int col = 16 * cb + i16;
                s.X[col][rl] = lds_entry<T>(s, p, R, J, rl, col, mk, norm) - u.acc[t][cb][v];
            }
    __syncthreads();
    trsm_tile<T, M>(s.Lt1, wave, s.X);
#pragma unroll
    for (int s8 = 0; s8 < kNB / 4; ++s8) {
        const int k = 4 * s8 + g;
        const T b0 = s.L21[i16][k], b1 = s.L21[16 + i16][k];
#pragma unroll
        for (int t = 0; t < M; ++t) {
            const T av = s.X[k][16 * (wave + kWS * t) + i16];
            u.acc[t][2] = mfma(av, b0, u.acc[t][2]);
            u.acc[t][3] = mfma(av, b1, u.acc[t][3]);
        }
    }
    store_tile<T>(A, J, R, nrow, s.X);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < M; ++t)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rl = 16 * (wave + kWS * t) + out_row<T>(g, v);
                const int col = 16 * cb + i16;
                s.X[col][rl] = lds_entry<T>(s, p, R, J, rl, kNB + col, mk, norm) -
                               u.acc[t][2 + cb][v];
            }
    __syncthreads();
    trsm_tile<T, M>(s.Lt2, wave, s.X);
    store_tile<T>(A, J + kNB, R, nrow, s.X);
}

// Block column J (64 columns): the launch has nslots_pad x tiles workgroups,
// one per (slot, 64-row tile below the slot's diagonal block), ordered as
// below.  lt_in: per slot, the diagonal 32x32 blocks of L_JJ transposed with
// reciprocal pivots.
template <typename T>
__global__ __launch_bounds__(kTS, 3) void k_chol_step(PrecondArgs a, int J, int nslots_pad,
                                                      T* __restrict__ scratch,
                                                      const int4* __restrict__ meta,
                                                      const T* __restrict__ lt_in) {
    __shared__ StepLds<T> s;
    // workgroup b runs on XCD b % 8 and serves a slot of that XCD (slot % 8 ==
    // b % 8, as in the other setup kernels); along each XCD's sequence of
    // workgroups the tiles of groups of kTileGroup slots are interleaved, so a
    // slot's tiles run close together in time and share its block rows
    // through that XCD's L2
    int slot, tile;
    {
        const int tiles = gridDim.x / nslots_pad;
        const int x = blockIdx.x & 7, q = blockIdx.x >> 3;
        const int per = nslots_pad >> 3, full = per / kTileGroup, span = kTileGroup * tiles;
        int grp, j;
        if (q < full * span) {
            grp = q / span;
            const int r = q - grp * span;
            tile = r / kTileGroup;
            j = r - tile * kTileGroup;
        } else {   // the last, smaller group
            const int gl = per - full * kTileGroup, r = q - full * span;
            grp = full;
            tile = r / gl;
            j = r - tile * gl;
        }
        slot = 8 * (grp * kTileGroup + j) + x;
    }
    const int4 m = meta[slot];
    const int np = m.x;
    const int R = J + kFB + kRows * tile;
    if (!m.w || R >= np) return;
    const int tid = threadIdx.x;
    T* A = scratch + (size_t)slot * slot_elems64(a.np_max);
    const T* lt = lt_in + (size_t)slot * kLtElems;
    // rows at or past the padding are zero in the padding columns
    const int k0 = (np - m.y) / kNB * kNB;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double2* xy = a.xy + (size_t)slot * a.np_max;
    const int p = np - m.y;
    step_tile<T, 1>(A, lt, xy, np, p, a.mk, a.norm, J, k0, R, wave, s);
}

// Diagonal block J0 > 0 of every slot, one workgroup of two waves per slot:
// D = A[J0.., J0..] - L[J0.., k0:J0] L[J0.., k0:J0]^T on its ten lower 16x16
// tiles.  The 16-column chunks of k0:J0 are dealt to the waves in pairs (wave
// w takes pairs w, w + 2, ...; MFMA chains, operands in two register buffers);
// wave 0 writes the evaluated block minus its sums, then wave 1 subtracts
// its own, so the order of the additions is fixed.  Then the block's factor
// (factor_diag64, on wave 0) into A and lt_out.  Two waves, not four: the
// serial factor runs on one wave, and six two-wave workgroups fit a CU's LDS
// where four-wave ones would leave fewer slots per CU in that phase.
constexpr int kDT = 128;
constexpr int kDW = kDT / 64;

template <typename T>
__device__ __forceinline__ void diag64_sub(Diag64<T>& d, int r, int c, T v) {
    if (r < kNB)
        d.D11[r][c] -= v;
    else if (c < kNB)
        d.D21[r - kNB][c] -= v;
    else
        d.D22[r - kNB][c - kNB] -= v;
}

template <typename T>
__global__ __launch_bounds__(kDT, 2) void k_chol_diag(PrecondArgs a, long long c0, int J0,
                                                      T* __restrict__ scratch,
                                                      int4* __restrict__ meta,
                                                      const int* __restrict__ lvl,
                                                      int* __restrict__ status,
                                                      T* __restrict__ lt_out) {
    __shared__ Diag64<T> s;
    __shared__ double2 xd[kFB];   // coordinates of the block's 64 rows
    const int slot = blockIdx.x;
    const int4 m = meta[slot];
    const int np = m.x;
    if (!m.w || J0 >= np) return;
    const int tid = threadIdx.x, lane = tid & 63, i16 = lane & 15, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    T* A = scratch + (size_t)slot * slot_elems64(a.np_max);
    const int k0 = (np - m.y) / kNB * kNB;
    if (tid < kFB) xd[tid] = a.xy[(size_t)slot * a.np_max + J0 + tid];
    const double shift = sizeof(T) == 4 ? diag_shift(lvl[slot], m.y, a.norm) : 0.0;
    const T* rows[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) rows[x] = A + roff(J0 + 16 * x + i16) + k0 + 4 * g;
    v4<T> acc[10];
#pragma unroll
    for (int t = 0; t < 10; ++t) acc[t] = v4<T>{0, 0, 0, 0};
    auto mma10 = [&](const v4<T>* b) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            int t = 0;
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y <= x; ++y, ++t) acc[t] = mfma(b[x][st], b[y][st], acc[t]);
        }
    };
    const int nchunk = (J0 - k0) / 16;   // even, >= 2
    int ch = 2 * wave;
    if (ch < nchunk) {
        v4<T> p[4], q[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) p[x] = load4(rows[x] + 16 * ch);
        for (; ch < nchunk; ch += 2 * kDW) {
#pragma unroll
            for (int x = 0; x < 4; ++x) q[x] = load4(rows[x] + 16 * (ch + 1));
            mma10(p);
            if (ch + 2 * kDW < nchunk) {
#pragma unroll
                for (int x = 0; x < 4; ++x) p[x] = load4(rows[x] + 16 * (ch + 2 * kDW));
            }
            mma10(q);
        }
    }
    __syncthreads();   // the staged coordinates
    for (int w = 0; w < kDW; ++w) {
        if (wave == w && (w == 0 || 2 * w < nchunk)) {
            int t = 0;
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y <= x; ++y, ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * x + out_row<T>(g, v), c = 16 * y + i16;
                        // rows J0 + r >= 64 lie past the padding (fewer than 64 rows)
                        if (w == 0)
                            diag64_put<T>(s, r, c,
                                          gauss_entry<T>(xd[r], xd[c], r == c, a.mk, a.norm,
                                                         shift) -
                                              acc[t][v]);
                        else
                            diag64_sub<T>(s, r, c, acc[t][v]);
                    }
        }
        __syncthreads();
    }
    const int f = factor_diag64<T>(A, J0, s, lt_out + (size_t)slot * kLtElems);
    if (f && tid == 0) {
        status[c0 + slot] = f;
        meta[slot].w = 0;
    }
}

// Centre rows, forward part: L W = E_C on the trailing block rows; workgroup
// b takes the 64 right-hand sides (b / nslots_pad) of slot b % nslots_pad.
// X(k, col) lives at Zc[col * n_omega + k - p] (padding rows are zero).
template <typename T>
__global__ __launch_bounds__(kT2, 2) void k_z_forward(PrecondArgs a, long long c0, int nslots_pad,
                                                      const T* __restrict__ scratch,
                                                      const int4* __restrict__ meta,
                                                      T* __restrict__ Z) {
    __shared__ ZLds<T> s;
    const int slot = blockIdx.x % nslots_pad, cp = blockIdx.x / nslots_pad;
    const int4 m = meta[slot];
    const int np = m.x, n_omega = m.y, n_c = m.z;
    const int col0 = cp * kZCols;
    if (!m.w || col0 >= n_c) return;
    const int tid = threadIdx.x;
    const int ncol = n_c - col0 < kZCols ? n_c - col0 : kZCols;
    const int p = np - n_omega, q0 = np - n_c, ib = q0 / kNB, nblk = np / kNB;
    const T* A = scratch + (size_t)slot * slot_elems64(a.np_max);
    T* Zc = Z + a.zoff[c0 + slot];
    for (int I = ib; I < nblk; ++I) {
        const int I0 = I * kNB;
        zsolve_forward<T>(A, I0, ib * kNB, I0, Zc, n_omega, p, col0, ncol, q0, s);
        if (tid < ncol) {
            for (int r = 0; r < kNB; ++r) {
                T v = s.acc[r][tid];
                for (int r2 = 0; r2 < r; ++r2) v = fma_t(-s.D[r][r2], s.acc[r2][tid], v);
                s.acc[r][tid] = v * s.invd[r];
            }
            for (int r = 0; r < kNB; ++r)
                if (I0 + r >= p) Zc[(size_t)(col0 + tid) * n_omega + (I0 + r - p)] = s.acc[r][tid];
        }
    }
}

// Centre rows, back solve of block row I: L_II^T X_I = W_I - L[below, I]^T
// X[below]; the slot's block rows are visited from its last one up.  Two waves
// per (slot, 64 right-hand sides): each forms the product for 32 of them (32
// rows x 32 columns, four 16x16 MFMA tiles) with its operands straight from
// memory into registers, the next chunk of 16 k in flight; W_I and the result
// move through LDS with coalesced accesses, and wave 0 runs the 32x32
// triangular solve, one right-hand side per lane, unrolled in registers.
constexpr int kZT = 128;   // threads of the back-solve kernel (two waves)

template <typename T>
struct ZBackLds {
    T T_[kNB][kZCols + 1];   // W_I - product, then X_I
    T L[kNB][kNB + 1];       // L_II
    T invd[kNB];
};

template <typename T>
__device__ __forceinline__ void z_back_block(const T* __restrict__ A, T* __restrict__ Zc, int I,
                                             int np, int n_omega, int p, int ncol, int w_lo,
                                             ZBackLds<T>& s) {
    const int I0 = I * kNB;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // W_I (zero above w_lo and in the padding rows), coalesced along each Z row
    for (int idx = tid; idx < kNB * kZCols; idx += kZT) {
        const int c = idx / kNB, r = idx % kNB;
        const int row = I0 + r;
        s.T_[r][c] = (c < ncol && row >= w_lo && row >= p) ? Zc[(size_t)c * n_omega + row] : T(0);
    }
    for (int idx = tid; idx < kNB * kNB; idx += kZT) {
        const int i = idx / kNB, j = idx % kNB;
        s.L[i][j] = (j <= i) ? A[roff(I0 + i) + I0 + j] : T(0);
    }
    // product over k in [I0 + 32, np); wave w the right-hand sides 32w ..
    const int i16 = lane & 15, g = lane >> 4;
    const int nchunk = (np - I0 - kNB) / 16;   // even
    v4<T> acc[2][2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = v4<T>{0, 0, 0, 0};
    if (nchunk > 0) {
        const T* zr[2];
        bool zv[2];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const int c = 32 * wave + 16 * ct + i16;
            zv[ct] = c < ncol;
            zr[ct] = Zc + (size_t)(zv[ct] ? c : 0) * n_omega;
        }
        struct Buf {
            T a[2][4], b[2][4];
        } q0, q1;
        auto load = [&](Buf& d, int ch) {
            const int k = I0 + kNB + 16 * ch + 4 * g;
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const T* lr = A + roff(k + st) + I0 + i16;
                d.a[0][st] = lr[0];
                d.a[1][st] = lr[16];
            }
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int st = 0; st < 4; ++st) d.b[ct][st] = zv[ct] ? zr[ct][k + st] : T(0);
        };
        auto mma4 = [&](const Buf& d) {
#pragma unroll
            for (int st = 0; st < 4; ++st)
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                    for (int ct = 0; ct < 2; ++ct)
                        acc[rt][ct] = mfma(d.a[rt][st], d.b[ct][st], acc[rt][ct]);
        };
        // two register buffers in turn (nchunk is even)
        load(q0, 0);
        for (int ch = 0; ch < nchunk; ch += 2) {
            load(q1, ch + 1);
            mma4(q0);
            if (ch + 2 < nchunk) load(q0, ch + 2);
            mma4(q1);
        }
    }
    __syncthreads();
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                s.T_[16 * rt + out_row<T>(g, v)][32 * wave + 16 * ct + i16] -= acc[rt][ct][v];
    if (tid < kNB) s.invd[tid] = T(1) / s.L[tid][tid];
    __syncthreads();
    // L_II^T x = t for right-hand side `lane` (wave 0), from the last row up
    if (wave == 0) {
        T x[kNB];
#pragma unroll
        for (int r = 0; r < kNB; ++r) x[r] = s.T_[r][lane];
#pragma unroll
        for (int r = kNB - 1; r >= 0; --r) {
            x[r] *= s.invd[r];
#pragma unroll
            for (int r2 = 0; r2 < r; ++r2) x[r2] = fma_t(-s.L[r][r2], x[r], x[r2]);
        }
#pragma unroll
        for (int r = 0; r < kNB; ++r) s.T_[r][lane] = x[r];
    }
    __syncthreads();
    for (int idx = tid; idx < kNB * kZCols; idx += kZT) {
        const int c = idx / kNB, r = idx % kNB;
        const int row = I0 + r;
        if (c < ncol && row >= p) Zc[(size_t)c * n_omega + row] = s.T_[r][c];
    }
    // the next block rows read these rows back (workgroup-scope release and
    // acquire: the same wave, the same CU)
    __syncthreads();
}

// All block rows of the back solve for one (slot, 64 right-hand sides), from
// the slot's last block row up, in one launch: each block row reuses the rows
// this wave has just solved.
template <typename T>
__global__ __launch_bounds__(kZT, 3) void k_z_back(PrecondArgs a, long long c0, int nslots_pad,
                                                const T* __restrict__ scratch,
                                                const int4* __restrict__ meta,
                                                T* __restrict__ Z) {
    __shared__ ZBackLds<T> s;
    const int slot = blockIdx.x % nslots_pad, cp = blockIdx.x / nslots_pad;
    const int4 m = meta[slot];
    const int np = m.x, n_omega = m.y, n_c = m.z;
    const int col0 = cp * kZCols;
    const int p = np - n_omega;
    if (!m.w || col0 >= n_c) return;
    const int ncol = n_c - col0 < kZCols ? n_c - col0 : kZCols;
    const int w_lo = (np - n_c) / kNB * kNB;   // W is zero above this row
    const T* A = scratch + (size_t)slot * slot_elems64(a.np_max);
    T* Zc = Z + a.zoff[c0 + slot] + (size_t)col0 * n_omega - p;   // Zc[c * n_omega + k]
    for (int I = np / kNB - 1; I >= 0 && I * kNB + kNB > p; --I)
        z_back_block<T>(A, Zc, I, np, n_omega, p, ncol, w_lo, s);
}

}  // namespace

// Batches of nslots cells; every batch runs assembly, the factorisation steps
// and the two solves as one sequence of launches on stream st.  FP32 blocks
// whose factorisation failed are rebuilt with the next diagonal shift (up to
// four times), which needs the batch's status on the host.
template <typename T>
static hipError_t setup_lockstep(const PrecondArgs& a, T* Z, int nslots,
                                 const SetupLane<T>* lanes, int nlanes, int* status,
                                 hipStream_t st, SetupProfile* prof) {
    const int pad = (nslots + 7) / 8 * 8;
    const int ncp = (a.nc_max + kZCols - 1) / kZCols;
    const int attempts = sizeof(T) == 4 ? 5 : 1;
    std::vector<int> hs;
    // every launch goes through here: with a profile, an event pair around it
    hipError_t perr = hipSuccess;
    auto timed = [&](int kind, hipStream_t ls, auto&& launch) {
        SetupProfile::Rec r{kind, nullptr, nullptr};
        if (prof && perr == hipSuccess) {
            perr = hipEventCreate(&r.start);
            if (perr == hipSuccess) perr = hipEventCreate(&r.stop);
            if (perr == hipSuccess) perr = hipEventRecord(r.start, ls);
        }
        launch();
        if (prof && perr == hipSuccess) {
            perr = hipEventRecord(r.stop, ls);
            prof->recs.push_back(r);
        }
    };
    // lanes past the first start after the work already on st and st waits
    // for them at the end
    hipEvent_t join = nullptr;
    if (nlanes > 1) {
        hipError_t e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(join, st);
        for (int l = 1; l < nlanes && e == hipSuccess; ++l) e = hipStreamWaitEvent(lanes[l].st, join, 0);
        if (e != hipSuccess) {
            if (join) (void)hipEventDestroy(join);
            return e;
        }
    }
    const long long nbatch = (a.ncells + nslots - 1) / nslots;
    for (long long b0 = 0; b0 < nbatch; b0 += nlanes) {
        const int nl = (int)(nbatch - b0 < nlanes ? nbatch - b0 : nlanes);
        long long c0[2];
        PrecondArgs al[2];
        for (int l = 0; l < nl; ++l) {
            c0[l] = (b0 + l) * nslots;
            al[l] = a;
            al[l].xy = lanes[l].xy;
        }
        bool run[2] = {true, true};
        for (int att = 0; att < attempts; ++att) {
            if (att > 0) {   // FP32: rebuild only the batches with failed blocks
                bool any = false;
                for (int l = 0; l < nl; ++l) {
                    const int count = (int)(a.ncells - c0[l] < nslots ? a.ncells - c0[l] : nslots);
                    hs.resize(count);
                    hipError_t e = hipMemcpyAsync(hs.data(), status + c0[l], sizeof(int) * count,
                                                  hipMemcpyDeviceToHost, lanes[l].st);
                    if (e == hipSuccess) e = hipStreamSynchronize(lanes[l].st);
                    if (e != hipSuccess) return e;
                    run[l] = false;
                    for (int v : hs) run[l] = run[l] || v > 0;
                    any = any || run[l];
                }
                if (!any) break;
            }
            for (int l = 0; l < nl; ++l)
                if (run[l])
                    timed(RBF_K_ASSEMBLE, lanes[l].st, [&] {
                        k_setup_assemble<T><<<pad, kT2, 0, lanes[l].st>>>(
                            al[l], c0[l], nslots, att > 0, lanes[l].scratch, lanes[l].meta,
                            lanes[l].lvl, status, lanes[l].lt);
                    });
            // the lanes' launches alternate, so one lane's narrow launches (the
            // single-wave diagonal factors, the solves) share the device with the
            // other lane's factorisation steps
            for (int J = 0; J + kFB < a.np_max; J += kFB) {
                const int tiles = (a.np_max - J - kFB + kRows - 1) / kRows;
                const int b = (J / kFB) & 1;
                for (int l = 0; l < nl; ++l)
                    if (run[l])
                        timed(RBF_K_CHOL_STEP, lanes[l].st, [&] {
                            k_chol_step<T><<<pad * tiles, kTS, 0, lanes[l].st>>>(
                                al[l], J, pad, lanes[l].scratch, lanes[l].meta,
                                lanes[l].lt + (size_t)b * pad * kLtElems);
                        });
                for (int l = 0; l < nl; ++l)
                    if (run[l])
                        timed(RBF_K_CHOL_DIAG, lanes[l].st, [&] {
                            k_chol_diag<T><<<pad, kDT, 0, lanes[l].st>>>(
                                al[l], c0[l], J + kFB, lanes[l].scratch, lanes[l].meta,
                                lanes[l].lvl, status, lanes[l].lt + (size_t)(b ^ 1) * pad * kLtElems);
                        });
            }
            if (ncp > 0) {
                for (int l = 0; l < nl; ++l)
                    if (run[l])
                        timed(RBF_K_FORWARD, lanes[l].st, [&] {
                            k_z_forward<T><<<pad * ncp, kT2, 0, lanes[l].st>>>(
                                al[l], c0[l], pad, lanes[l].scratch, lanes[l].meta, Z);
                        });
                for (int l = 0; l < nl; ++l)
                    if (run[l])
                        timed(RBF_K_BACK, lanes[l].st, [&] {
                            k_z_back<T><<<pad * ncp, kZT, 0, lanes[l].st>>>(
                                al[l], c0[l], pad, lanes[l].scratch, lanes[l].meta, Z);
                        });
            }
        }
    }
    hipError_t e = hipGetLastError();
    if (nlanes > 1) {
        for (int l = 1; l < nlanes && e == hipSuccess; ++l) {
            e = hipEventRecord(join, lanes[l].st);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, join, 0);
        }
        (void)hipEventDestroy(join);
    }
    if (perr != hipSuccess) return perr;
    return e;
}

hipError_t launch_precond_setup64(const PrecondArgs& a, double* Z, int nslots,
                                  const SetupLane<double>* lanes, int nlanes, int* status,
                                  hipStream_t st, SetupProfile* prof) {
    return setup_lockstep<double>(a, Z, nslots, lanes, nlanes, status, st, prof);
}

hipError_t launch_precond_setup32(const PrecondArgs& a, float* Z, int nslots,
                                  const SetupLane<float>* lanes, int nlanes, int* status,
                                  hipStream_t st, SetupProfile* prof) {
    return setup_lockstep<float>(a, Z, nslots, lanes, nlanes, status, st, prof);
}

namespace {

// z[c's points] = Z_c v[members of c], one workgroup per cell: the member
// values of v gathered into LDS, then Z_c streamed once from HBM.  Each wave
// takes four rows at a time, a 16-lane group per row (so one load instruction
// reads four row segments), four independent loads per lane in flight, and one
// 16-lane reduction per row.  TZ is Z's storage, TV the precision of v and of
// the sums: FP64 Z with FP64 sums (the FP64 method), FP32 Z with FP32 sums and
// Kahan compensation (the mixed form's inner solves), and FP32 Z widened into
// FP64 sums of the FP64 v (the FP64 method with FP32-stored local inverses: a
// fixed linear operator, so right-preconditioned GMRES is unchanged by it).
template <typename TZ, typename TV>
__device__ __forceinline__ double row_dot(const TZ* __restrict__ zr, const TV* vs, int n_omega,
                                          int ph) {
    if (sizeof(TV) == 8) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int q = ph;
        for (; q + 48 < n_omega; q += 64) {
            const double z0 = (double)zr[q], z1 = (double)zr[q + 16], z2 = (double)zr[q + 32],
                         z3 = (double)zr[q + 48];
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

struct RasmLds {
    double vs[RBF_MAX_BLOCK];   // the member values (as T)
    int rb[kMaxRanges], re[kMaxRanges];
    int nr_s, n_omega_s, n_c_s;
};

template <typename TZ, typename TV>
__device__ __forceinline__ void rasm_cell(PrecondArgs a, const TZ* __restrict__ Z,
                                          const double* __restrict__ v, double* __restrict__ z,
                                          long long c, RasmLds& L) {
    TV* vs = reinterpret_cast<TV*>(L.vs);
    int* rb = L.rb;
    int* re = L.re;
    int& nr_s = L.nr_s;
    int& n_omega_s = L.n_omega_s;
    int& n_c_s = L.n_c_s;
    const int tid = threadIdx.x;
    if (tid == 0) {
        if (a.mem) {
            n_omega_s = (int)(a.moff[c + 1] - a.moff[c]);
            n_c_s = a.nown[c];
            nr_s = 0;
        } else {
            block_ranges(a.cell_start, a.g, a.overlap, c, rb, re, &nr_s, &n_omega_s, &n_c_s);
        }
    }
    __syncthreads();
    const int n_omega = n_omega_s, n_c = n_c_s, nr = nr_s;
    if (n_c == 0) return;
    const int* mlist = a.mem ? a.mem + a.moff[c] : nullptr;
    for (int k = tid; k < n_omega; k += kThreads)
        vs[k] = (TV)v[mlist ? mlist[k] : member_index(rb, re, nr, k)];
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int grp = lane >> 4, ph = lane & 15;
    const TZ* Zc = Z + a.zoff[c];
    const int own = mlist ? 0 : a.cell_start[c];
    for (int r0 = 4 * wave; r0 < n_c; r0 += 4 * (kThreads / 64)) {
        const int r = r0 + grp;
        double sum = 0.0;
        if (r < n_c) sum = row_dot<TZ, TV>(Zc + (size_t)r * n_omega, vs, n_omega, ph);
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) sum += __shfl_xor(sum, o, RBF_WAVE);
        if (ph == 0 && r < n_c) z[mlist ? mlist[n_omega - n_c + r] : own + r] = sum;
    }
}

template <typename TZ, typename TV>
__global__ __launch_bounds__(kThreads) void k_rasm_apply(PrecondArgs a, const TZ* __restrict__ Z,
                                                         const double* __restrict__ v,
                                                         double* __restrict__ z) {
    __shared__ RasmLds L;
    rasm_cell<TZ, TV>(a, Z, v, z, blockIdx.x, L);
}

// Packed form: workgroup b serves subdomain b - block0[j] of job j.
__global__ __launch_bounds__(kThreads) void k_rasm_packed(const RasmJob* __restrict__ jobs,
                                                          const int* __restrict__ block0,
                                                          int njobs) {
    __shared__ RasmLds L;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (block0[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const int j = __builtin_amdgcn_readfirstlane(lo);
    const RasmJob& J = jobs[j];
    const long long c = (long long)blockIdx.x - block0[j];
    if (J.skip) return;
    if (J.prec == 0)
        rasm_cell<double, double>(J.a, static_cast<const double*>(J.Z), J.v, J.z, c, L);
    else if (J.prec == 1)
        rasm_cell<float, float>(J.a, static_cast<const float*>(J.Z), J.v, J.z, c, L);
    else
        rasm_cell<float, double>(J.a, static_cast<const float*>(J.Z), J.v, J.z, c, L);
}

// Members of box b (one wave per box): the candidate cells are those of the
// square of side D around the box's centre, widened by one cell (rounding at
// its edges), scanned row by row, each row's cells one contiguous sorted
// range, so the members come out in sorted order; a first pass takes the
// points inside the square that the box does not own, a second the box's
// own points.  The decisions use the same arithmetic as the oracle's: box
// index floor((x - x0) / B) clamped, centre x0 + (bx + 1/2) B, and
// |x - centre| <= D / 2 along both axes.
__device__ __forceinline__ int box_coord(double v, double v0, double inv, int n) {
    double t = floor((v - v0) * inv);
    if (!(t >= 0.0)) t = 0.0;
    if (t > (double)(n - 1)) t = (double)(n - 1);
    return (int)t;
}

constexpr int kBoxThreads = 256;

template <bool kFill>
__global__ __launch_bounds__(kBoxThreads) void k_box_members(PrecondArgs a, BoxGeometry bg,
                                                            int* __restrict__ n_omega,
                                                            int* __restrict__ n_own,
                                                            const long long* __restrict__ moff,
                                                            int* __restrict__ mem) {
    const int lane = threadIdx.x & 63;
    const long long b = (long long)blockIdx.x * (kBoxThreads / 64) + (threadIdx.x >> 6);
    const long long nbox = (long long)bg.nbx * bg.nby;
    if (b >= nbox) return;
    const int bx = (int)(b % bg.nbx), by = (int)(b / bg.nbx);
    const double cx = bg.x0 + ((double)bx + 0.5) * bg.B;
    const double cy = bg.y0 + ((double)by + 0.5) * bg.B;
    const double h = bg.halfD;
    const Grid& g = a.g;
    int xa = box_coord(cx - h, g.x0, g.invL, g.ncx) - 1, xb = box_coord(cx + h, g.x0, g.invL, g.ncx) + 1;
    int ya = box_coord(cy - h, g.y0, g.invL, g.ncy) - 1, yb = box_coord(cy + h, g.y0, g.invL, g.ncy) + 1;
    xa = xa < 0 ? 0 : xa;
    ya = ya < 0 ? 0 : ya;
    xb = xb > g.ncx - 1 ? g.ncx - 1 : xb;
    yb = yb > g.ncy - 1 ? g.ncy - 1 : yb;
    int* out = kFill ? mem + moff[b] : nullptr;
    int k = 0, kc = 0;
    for (int own = 0; own <= 1; ++own)
        for (int ny = ya; ny <= yb; ++ny) {
            const int j0 = a.cell_start[ny * g.ncx + xa], j1 = a.cell_start[ny * g.ncx + xb + 1];
            for (int jb = j0; jb < j1; jb += 64) {
                const int j = jb + lane;
                bool take = false;
                if (j < j1) {
                    const double x = a.xs[j], y = a.ys[j];
                    const bool mine = box_coord(x, bg.x0, bg.invB, bg.nbx) == bx &&
                                      box_coord(y, bg.y0, bg.invB, bg.nby) == by;
                    const bool inside = fabs(x - cx) <= h && fabs(y - cy) <= h;
                    take = own ? mine : (inside && !mine);
                }
                const unsigned long long m = __ballot(take);
                if (kFill && take) out[k + __popcll(m & ((1ull << lane) - 1ull))] = j;
                const int cnt = __popcll(m);
                k += cnt;
                kc += own ? cnt : 0;
            }
        }
    if (!kFill && lane == 0) {
        n_omega[b] = k;
        n_own[b] = kc;
    }
}

}  // namespace

hipError_t launch_box_members(const PrecondArgs& a, const BoxGeometry& bg, int* n_omega,
                              int* n_own, const long long* moff, int* mem, hipStream_t st) {
    const long long nbox = (long long)bg.nbx * bg.nby;
    const unsigned grid = (unsigned)((nbox + kBoxThreads / 64 - 1) / (kBoxThreads / 64));
    if (nbox == 0) return hipSuccess;
    if (mem)
        k_box_members<true><<<grid, kBoxThreads, 0, st>>>(a, bg, n_omega, n_own, moff, mem);
    else
        k_box_members<false><<<grid, kBoxThreads, 0, st>>>(a, bg, n_omega, n_own, moff, mem);
    return hipGetLastError();
}

hipError_t launch_rasm_packed(const RasmJob* jobs, const int* block0, int njobs, int nblocks,
                              hipStream_t st) {
    if (njobs > 0 && nblocks > 0) k_rasm_packed<<<nblocks, kThreads, 0, st>>>(jobs, block0, njobs);
    return hipGetLastError();
}

hipError_t launch_rasm_apply64(const PrecondArgs& a, const double* Z, const double* v, double* z,
                               hipStream_t st) {
    k_rasm_apply<double, double><<<(unsigned)a.ncells, kThreads, 0, st>>>(a, Z, v, z);
    return hipGetLastError();
}

hipError_t launch_rasm_apply32(const PrecondArgs& a, const float* Z, const double* v, double* z,
                               hipStream_t st) {
    k_rasm_apply<float, float><<<(unsigned)a.ncells, kThreads, 0, st>>>(a, Z, v, z);
    return hipGetLastError();
}

hipError_t launch_rasm_apply32x64(const PrecondArgs& a, const float* Z, const double* v, double* z,
                                  hipStream_t st) {
    k_rasm_apply<float, double><<<(unsigned)a.ncells, kThreads, 0, st>>>(a, Z, v, z);
    return hipGetLastError();
}

}  // namespace rbf
