// rbf_device.hpp -- device-side helpers shared by the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define RBF_WAVE 64

namespace rbf {

// ---------------------------------------------------------------------------
// exp(x) for x <= 0 in FP64, written from the standard Cody-Waite argument
// reduction: x = n ln2 + r with n = rint(x / ln2) and |r| <= ln2/2, then
// exp(x) = 2^n exp(r).  exp(r) is the degree-12 Taylor polynomial
// sum_{k<=12} r^k / k!, whose truncation error is below r^13/13! < 1.8e-16
// relative on |r| <= 0.3466.  ln2 is split into a 32-bit head (exact products
// n*LN2_HI for |n| < 2^20) and its remainder.  The rounding to an integer uses
// the 1.5*2^52 shift: after the fused multiply-add the low 32 bits of the sum
// hold n in two's complement.  Valid for -700 < x <= 0 (no overflow, no
// subnormal results); the cutoff keeps the matvec's arguments in [-18, 0].
// The constants are derived in exact arithmetic by gen_constants.py.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double exp_neg(double x) {
    const double kLog2e = 0x1.71547652b82fep+0;        // 1/ln2 rounded
    const double kShift = 0x1.8p52;                   // 1.5 * 2^52
    const double kLn2Hi = 0x1.62e42ff000000p-1;       // ln2 to 32 significant bits
    const double kLn2Lo = -0x1.718432a1b0e26p-35;     // ln2 - kLn2Hi, rounded
    double t = __builtin_fma(x, kLog2e, kShift);
    double nf = t - kShift;
    int n = (int)__double2loint(t);
    double r = __builtin_fma(nf, -kLn2Hi, x);
    r = __builtin_fma(nf, -kLn2Lo, r);
    double p = 0x1.1eed8eff8d898p-29;                  // 1/12!
    p = __builtin_fma(p, r, 0x1.ae64567f544e4p-26);     // 1/11!
    p = __builtin_fma(p, r, 0x1.27e4fb7789f5cp-22);     // 1/10!
    p = __builtin_fma(p, r, 0x1.71de3a556c734p-19);     // 1/9!
    p = __builtin_fma(p, r, 0x1.a01a01a01a01ap-16);     // 1/8!
    p = __builtin_fma(p, r, 0x1.a01a01a01a01ap-13);     // 1/7!
    p = __builtin_fma(p, r, 0x1.6c16c16c16c17p-10);     // 1/6!
    p = __builtin_fma(p, r, 0x1.1111111111111p-7);      // 1/5!
    p = __builtin_fma(p, r, 0x1.5555555555555p-5);      // 1/4!
    p = __builtin_fma(p, r, 0x1.5555555555555p-3);      // 1/3!
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_amdgcn_ldexp(p, n);
}

// ---------------------------------------------------------------------------
// exp(x) for -(ntab-1)/128 <= x <= 0 from a table T[n] = e^{-n/128} (correctly
// rounded, n = 0..ntab-1, held in LDS by the caller): with n = rint(-128 x) and
// r = x + n/128 (|r| <= 1/256, formed exactly up to one rounding),
// exp(x) = T[n] exp(r), exp(r) by its degree-5 Taylor polynomial (truncation
// below r^6/720 < 5e-18).  The rounding to an integer uses the 1.5*2^52 shift.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double exp_neg_tab(double x, const double* __restrict__ T) {
    const double kShift = 0x1.8p52;
    const double t = __builtin_fma(x, -128.0, kShift);
    const double nf = t - kShift;
    const int n = (int)__double2loint(t);
    const double r = __builtin_fma(nf, 0x1p-7, x);
    double p = 0x1.1111111111111p-7;                 // 1/5!
    p = __builtin_fma(p, r, 0x1.5555555555555p-5);   // 1/4!
    p = __builtin_fma(p, r, 0x1.5555555555555p-3);   // 1/3!
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return T[n] * p;
}

// ---------------------------------------------------------------------------
// exp(x) for -700 < x <= 0 by Tang's table-driven method (P. T. P. Tang,
// "Table-driven implementation of the exponential function in IEEE
// floating-point arithmetic", ACM TOMS 15(2), 1989) with a 32-entry table
// T[j] = 2^(j/32) (correctly rounded, held in LDS by the caller; 256 bytes, so
// lanes never conflict on a bank): with k = rint(32 x / ln2) = 32 n + j (0 <= j < 32) and
// r = x - k ln2 / 32 (|r| <= ln2/64, ln2/32 split exactly as above),
// exp(x) = 2^n T[j] exp(r), exp(r) by its degree-6 Taylor polynomial
// (truncation below r^7/7! < 3.5e-18).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double exp_neg_t32(double x, const double* T) {
    const double kLog2e32 = 0x1.71547652b82fep+5;     // 32/ln2 rounded
    const double kShift = 0x1.8p52;
    const double kLn2Hi32 = 0x1.62e42ff000000p-6;     // ln2 head / 32 (exact)
    const double kLn2Lo32 = -0x1.718432a1b0e26p-40;   // ln2 tail / 32 (exact)
    const double t = __builtin_fma(x, kLog2e32, kShift);
    const double kf = t - kShift;
    const int k = (int)__double2loint(t);
    double r = __builtin_fma(kf, -kLn2Hi32, x);
    r = __builtin_fma(kf, -kLn2Lo32, r);
    double p = 0x1.6c16c16c16c17p-10;                 // 1/6!
    p = __builtin_fma(p, r, 0x1.1111111111111p-7);    // 1/5!
    p = __builtin_fma(p, r, 0x1.5555555555555p-5);    // 1/4!
    p = __builtin_fma(p, r, 0x1.5555555555555p-3);    // 1/3!
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_amdgcn_ldexp(T[k & 31] * p, k >> 5);
}

// ---------------------------------------------------------------------------
// 2^(y/32) for y = d2 * beta <= 0, where beta folds the Gaussian's -1/(2 sigma^2)
// and 32/ln2 (so 2^(y/32) = exp(-d2 / (2 sigma^2))), by Tang's table-driven
// method (ACM TOMS 15(2), 1989) from a 32-entry table
// T[j] = 2^(j/32) (correctly rounded, in LDS, as for exp_neg_t32).
// k = rint(y) = 32 n + j is read from the fused product against the 1.5*2^52
// shift; f = y - k comes from a second fused multiply-add of the same exact
// product (one rounding, |f| <= 1/2), so no split constant is needed: the
// reduction's only error is beta's own rounding.  2^(f/32) = exp(f ln2/32) is
// the degree-5 polynomial interpolating it at the six Chebyshev points of
// [-1/2, 1/2] (coefficients solved and rounded by gen_constants.py, which
// checks in exact arithmetic that the rounded polynomial stays within
// 1.41e-16 relative of exp there): one multiply-add fewer than the degree-6
// Taylor polynomial, for an exponential within 5.2e-16 relative instead of
// 4e-16 (table entry and three roundings included).
// Valid for -700*32/ln2 < y <= 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double exp2_scaled_t32(double d2, double beta, const double* T) {
    const double kShift = 0x1.8p52;
    const double t = __builtin_fma(d2, beta, kShift);
    const double kf = t - kShift;
    const int k = (int)__double2loint(t);
    const double f = __builtin_fma(d2, beta, -kf);
    double p = 0x1.5d885e6ef14a6p-35;
    p = __builtin_fma(p, f, 0x1.3b2b301f1eb9cp-27);
    p = __builtin_fma(p, f, 0x1.c6b08d70380ddp-20);
    p = __builtin_fma(p, f, 0x1.ebfbdff7feebap-13);
    p = __builtin_fma(p, f, 0x1.62e42fefa39efp-6);
    p = __builtin_fma(p, f, 1.0);
    // the byte offset 8 (k mod 32) of T[k mod 32] in one instruction: a shift
    // by 3 whose result keeps only its low byte (SDWA destination select), where
    // a mask and a shift would take two
    unsigned off;
    asm("v_lshlrev_b32_sdwa %0, 3, %1 dst_sel:BYTE_0 dst_unused:UNUSED_PAD src0_sel:DWORD "
        "src1_sel:DWORD"
        : "=v"(off)
        : "v"(k));
    const double tj = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(T) + off);
    return __builtin_amdgcn_ldexp(tj * p, k >> 5);
}

// 2^x in FP32 on the hardware transcendental unit (v_exp_f32).
__device__ __forceinline__ float exp2_f32(float x) { return __builtin_amdgcn_exp2f(x); }

// Wave-wide sum of a double (64 lanes), butterfly over lanes; every lane gets it.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, RBF_WAVE);
    return v;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, RBF_WAVE);
    return v;
}

// Kahan-compensated FP32 accumulator.
struct Kahan32 {
    float s = 0.f, c = 0.f;
    __device__ __forceinline__ void add(float v) {
        float y = v - c;
        float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};

}  // namespace rbf
