// krylov.hip -- GMRES vector operations on gfx950 (HBM-bound streaming).
//
// Inner products are reduced in two fixed-order stages (per-block partial sums,
// then one block summing the partials in block order), so every result is
// bit-reproducible run to run.  Several inner products against the same vector
// share one pass over it (classical Gram-Schmidt reads w once for a whole
// column of the Hessenberg matrix).
#include "rbf_device.hpp"
#include "rbf_internal.hpp"

namespace rbf {

namespace {

constexpr int kBlock = 256;
constexpr int kDotChunk = 8;   // inner products per pass over w

template <int NV>
__global__ __launch_bounds__(kBlock) void k_multidot(const double* __restrict__ V, long long ldv,
                                                     const double* __restrict__ w, long long n,
                                                     double* __restrict__ partial, int pstride) {
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        double wi = w[i];
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] = __builtin_fma(V[k * ldv + i], wi, acc[k]);
    }
    __shared__ double sh[kBlock / 64][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double v = wave_sum(acc[k]);
        if (lane == 0) sh[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double v = 0.0;
        for (int q = 0; q < kBlock / 64; ++q) v += sh[q][threadIdx.x];
        partial[(long long)threadIdx.x * pstride + blockIdx.x] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce_partials(const double* __restrict__ partial,
                                                            int nb, int pstride,
                                                            double* __restrict__ out) {
    __shared__ double sh[kBlock];
    const double* p = partial + (long long)blockIdx.x * pstride;
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) v += p[b];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kBlock) void k_multi_axpy(const double* __restrict__ V, long long ldv,
                                                       int nv, const double* __restrict__ h,
                                                       double* __restrict__ w, long long n,
                                                       double sign) {
    __shared__ double hs[64];
    if (threadIdx.x < nv) hs[threadIdx.x] = h[threadIdx.x];
    __syncthreads();
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        double s = 0.0;
        for (int k = 0; k < nv; ++k) s = __builtin_fma(hs[k], V[k * ldv + i], s);
        w[i] = __builtin_fma(sign, s, w[i]);
    }
}

__global__ __launch_bounds__(kBlock) void k_scale_by_inv(const double* __restrict__ src,
                                                         const double* __restrict__ den,
                                                         double* __restrict__ dst, long long n) {
    const double d = __builtin_sqrt(den[0]);   // den holds a squared norm
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        dst[i] = src[i] / d;
}

__global__ __launch_bounds__(kBlock) void k_sub(const double* __restrict__ f,
                                                const double* __restrict__ y,
                                                double* __restrict__ r, long long n) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        r[i] = f[i] - y[i];
}

__global__ __launch_bounds__(kBlock) void k_axpy(double a, const double* __restrict__ z,
                                                 double* __restrict__ x, long long n) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        x[i] = __builtin_fma(a, z[i], x[i]);
}

__global__ __launch_bounds__(kBlock) void k_fill(double* __restrict__ x, double v, long long n) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        x[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_check_finite(const double* __restrict__ x,
                                                         long long n, int* __restrict__ flag) {
    int bad = 0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        bad |= !__builtin_isfinite(x[i]);
    if (bad) atomicOr(flag, 1);
}

// Sum of n non-negative counts into out[0], which the caller zeroes: a
// grid-stride pass, a workgroup reduction, one 64-bit atomic add per
// workgroup (integer sums are exact in any order).
__global__ __launch_bounds__(kBlock) void k_sum_counts(const int* __restrict__ c, long long n,
                                                       unsigned long long* __restrict__ out) {
    __shared__ unsigned long long sh[kBlock];
    unsigned long long v = 0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        v += (unsigned long long)c[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && sh[0] != 0) atomicAdd(out, sh[0]);
}

inline unsigned stream_grid(long long n) {
    long long b = (n + kBlock - 1) / kBlock;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// ---- packed forms: one launch serves the jobs of many problems --------------
// Job j owns workgroups [block0_j, block0_{j+1}); a workgroup finds its job by
// a binary search over the block offsets and runs the single-problem loop with
// its own block index and block count, so every job computes exactly what the
// single-problem launch computes (the same grid-stride decomposition, hence
// bit-identical reductions).
__device__ __forceinline__ int find_job(const int* __restrict__ block0, int njobs, int b) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (block0[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_vec_packed(const VecJob* __restrict__ jobs,
                                                       const int* __restrict__ block0, int njobs) {
    const int j = find_job(block0, njobs, blockIdx.x);
    const VecJob& J = jobs[j];
    const long long nb = block0[j + 1] - block0[j], b = blockIdx.x - block0[j];
    const long long n = J.n;
    const int op = J.op;
    const double* __restrict__ A = J.a;
    double* __restrict__ Y = J.y;
    if (op == VecJob::kNop) return;
    if (op == VecJob::kMultiAxpy) {
        __shared__ double hs[64];
        const int nv = J.nv;
        const long long ld = J.ld;
        if (threadIdx.x < nv) hs[threadIdx.x] = J.coef[threadIdx.x];
        __syncthreads();
        const double sign = J.sign;
        const bool over = J.overwrite != 0;
        for (long long i = b * kBlock + threadIdx.x; i < n; i += nb * kBlock) {
            double s = 0.0;
            for (int k = 0; k < nv; ++k) s = __builtin_fma(hs[k], A[k * ld + i], s);
            Y[i] = __builtin_fma(sign, s, over ? 0.0 : Y[i]);
        }
        return;
    }
    const double* __restrict__ Bv = J.b;
    const double d = op == VecJob::kScaleByInv ? __builtin_sqrt(J.den[0]) : 1.0;
    for (long long i = b * kBlock + threadIdx.x; i < n; i += nb * kBlock) {
        if (op == VecJob::kSub) Y[i] = A[i] - Bv[i];
        else if (op == VecJob::kAxpy) Y[i] = __builtin_fma(1.0, A[i], Y[i]);
        else if (op == VecJob::kAxpyKeep) {
            const double yi = Y[i];
            J.keep[i] = yi;
            Y[i] = __builtin_fma(1.0, A[i], yi);
        }
        else if (op == VecJob::kFill) Y[i] = 0.0;
        else if (op == VecJob::kScaleByInv) Y[i] = A[i] / d;
    }
}

// out partials of <V_k, w>, k < nv, in chunks of 8 as the single-problem
// launches take them (partial[k * kDotBlocks + b])
__global__ __launch_bounds__(kBlock) void k_multidot_packed(const DotJob* __restrict__ jobs,
                                                            const int* __restrict__ block0,
                                                            int njobs) {
    const int j = find_job(block0, njobs, blockIdx.x);
    const DotJob J = jobs[j];   // a few pointers and sizes
    const long long nb = block0[j + 1] - block0[j], b = blockIdx.x - block0[j];
    __shared__ double sh[kBlock / 64][kDotChunk];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k0 = 0; k0 < J.nv; k0 += kDotChunk) {
        const int c = J.nv - k0 < kDotChunk ? J.nv - k0 : kDotChunk;
        const double* Vk = J.V + (long long)k0 * J.ldv;
        double acc[kDotChunk];
#pragma unroll
        for (int k = 0; k < kDotChunk; ++k) acc[k] = 0.0;
        for (long long i = b * kBlock + threadIdx.x; i < J.n; i += nb * kBlock) {
            const double wi = J.w[i];
#pragma unroll
            for (int k = 0; k < kDotChunk; ++k)
                if (k < c) acc[k] = __builtin_fma(Vk[k * J.ldv + i], wi, acc[k]);
        }
#pragma unroll
        for (int k = 0; k < kDotChunk; ++k) {
            const double v = wave_sum(acc[k]);
            if (lane == 0) sh[wave][k] = v;
        }
        __syncthreads();
        if (threadIdx.x < c) {
            double v = 0.0;
            for (int q = 0; q < kBlock / 64; ++q) v += sh[q][threadIdx.x];
            J.partial[(long long)(k0 + threadIdx.x) * kDotBlocks + b] = v;
        }
        __syncthreads();
    }
}

// out[k] = sum of the nb partials of k, one workgroup per (job, k), as
// k_reduce_partials
__global__ __launch_bounds__(kBlock) void k_reduce_packed(const DotJob* __restrict__ jobs,
                                                          const int* __restrict__ block0,
                                                          int njobs) {
    const int j = find_job(block0, njobs, blockIdx.x);
    const DotJob J = jobs[j];
    const int k = blockIdx.x - block0[j];
    if (k >= J.nv) return;
    __shared__ double sh[kBlock];
    const double* p = J.partial + (long long)k * kDotBlocks;
    double v = 0.0;
    for (int b = threadIdx.x; b < J.nb; b += kBlock) v += p[b];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) J.out[k] = sh[0];
}

}  // namespace

int dot_blocks(long long n) {
    long long nb64 = (n + kBlock - 1) / kBlock;
    int nb = (int)(nb64 < kDotBlocks ? nb64 : kDotBlocks);
    return nb < 1 ? 1 : nb;
}

int vec_blocks(long long n) { return (int)stream_grid(n); }

hipError_t launch_vec_packed(const VecJob* jobs, const int* block0, int njobs, int nblocks,
                             hipStream_t st) {
    if (njobs > 0 && nblocks > 0) k_vec_packed<<<nblocks, kBlock, 0, st>>>(jobs, block0, njobs);
    return hipGetLastError();
}

hipError_t launch_multidot_packed(const DotJob* jobs, const int* block0, int njobs, int nblocks,
                                  hipStream_t st) {
    if (njobs > 0 && nblocks > 0) k_multidot_packed<<<nblocks, kBlock, 0, st>>>(jobs, block0, njobs);
    return hipGetLastError();
}

hipError_t launch_reduce_packed(const DotJob* jobs, const int* block0, int njobs, int nblocks,
                                hipStream_t st) {
    if (njobs > 0 && nblocks > 0) k_reduce_packed<<<nblocks, kBlock, 0, st>>>(jobs, block0, njobs);
    return hipGetLastError();
}

hipError_t launch_multidot(const double* V, long long ldv, int nv, const double* w, long long n,
                           double* partial, double* out, hipStream_t st) {
    long long nb64 = (n + kBlock - 1) / kBlock;
    int nb = (int)(nb64 < kDotBlocks ? nb64 : kDotBlocks);
    if (nb < 1) nb = 1;
    for (int k0 = 0; k0 < nv; k0 += kDotChunk) {
        int c = nv - k0 < kDotChunk ? nv - k0 : kDotChunk;
        const double* Vk = V + (long long)k0 * ldv;
        double* pk = partial + (long long)k0 * kDotBlocks;
        switch (c) {
            case 1: k_multidot<1><<<nb, kBlock, 0, st>>>(Vk, ldv, w, n, pk, kDotBlocks); break;
            case 2: k_multidot<2><<<nb, kBlock, 0, st>>>(Vk, ldv, w, n, pk, kDotBlocks); break;
            case 3: k_multidot<3><<<nb, kBlock, 0, st>>>(Vk, ldv, w, n, pk, kDotBlocks); break;
            case 4: k_multidot<4><<<nb, kBlock, 0, st>>>(Vk, ldv, w, n, pk, kDotBlocks); break;
            case 5: k_multidot<5><<<nb, kBlock, 0, st>>>(Vk, ldv, w, n, pk, kDotBlocks); break;
            case 6: k_multidot<6><<<nb, kBlock, 0, st>>>(Vk, ldv, w, n, pk, kDotBlocks); break;
            case 7: k_multidot<7><<<nb, kBlock, 0, st>>>(Vk, ldv, w, n, pk, kDotBlocks); break;
            default: k_multidot<8><<<nb, kBlock, 0, st>>>(Vk, ldv, w, n, pk, kDotBlocks); break;
        }
    }
    k_reduce_partials<<<nv, kBlock, 0, st>>>(partial, nb, kDotBlocks, out);
    return hipGetLastError();
}

hipError_t launch_multi_axpy(const double* V, long long ldv, int nv, const double* h, double* w,
                             long long n, double sign, hipStream_t st) {
    if (nv > 64) return hipErrorInvalidValue;
    k_multi_axpy<<<stream_grid(n), kBlock, 0, st>>>(V, ldv, nv, h, w, n, sign);
    return hipGetLastError();
}

hipError_t launch_scale_by_inv(const double* src, const double* den, double* dst, long long n,
                               hipStream_t st) {
    k_scale_by_inv<<<stream_grid(n), kBlock, 0, st>>>(src, den, dst, n);
    return hipGetLastError();
}

hipError_t launch_sub(const double* f, const double* y, double* r, long long n, hipStream_t st) {
    k_sub<<<stream_grid(n), kBlock, 0, st>>>(f, y, r, n);
    return hipGetLastError();
}

hipError_t launch_axpy(double a, const double* z, double* x, long long n, hipStream_t st) {
    k_axpy<<<stream_grid(n), kBlock, 0, st>>>(a, z, x, n);
    return hipGetLastError();
}

hipError_t launch_fill(double* x, double v, long long n, hipStream_t st) {
    k_fill<<<stream_grid(n), kBlock, 0, st>>>(x, v, n);
    return hipGetLastError();
}

hipError_t launch_check_finite(const double* x, long long n, int* flag, hipStream_t st) {
    k_check_finite<<<stream_grid(n), kBlock, 0, st>>>(x, n, flag);
    return hipGetLastError();
}

hipError_t launch_sum_counts(const int* nnb, long long n, long long* out, hipStream_t st) {
    hipError_t e = hipMemsetAsync(out, 0, sizeof(long long), st);
    if (e != hipSuccess) return e;
    k_sum_counts<<<stream_grid(n), kBlock, 0, st>>>(nnb, n,
                                                   reinterpret_cast<unsigned long long*>(out));
    return hipGetLastError();
}

}  // namespace rbf
