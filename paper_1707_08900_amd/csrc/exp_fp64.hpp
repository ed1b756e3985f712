// e^x in FP64 for the global diagnostics (mass and kinetic energy sum
// e^lnrho), written out so that it costs the fused sweep few instructions:
//
//   x = k ln2 + r,  k = rint(x / ln2),  |r| <= ln2 / 2,   e^x = 2^k e^r,
//
// the reduction in two fused multiply-adds with ln2 split into a high part of
// 32 significant bits (k * hi is exact for |k| < 2^21) and the FP64
// remainder (Cody and Waite's method), e^r by its Taylor series to degree 13
// (truncation below 4e-18 relative for |r| <= ln2 / 2) evaluated by Horner's
// rule in fused multiply-adds, and 2^k applied exactly by ldexp, which also yields 0 or infinity
// past the FP64 range.  x is clamped to [-1000, 1000] first, where e^x is
// already 0 or infinity in FP64 and k stays small; a NaN x therefore gives a
// number, so callers count non-finite inputs themselves.  Accuracy: within
// 2 ulp of the correctly rounded value over the FP64 range.
#pragma once

#include <hip/hip_runtime.h>

namespace fd6 {

// The arithmetic, with the fused multiply-add supplied by the caller (the
// device form below, or a host fma for checking it on the CPU).
template <typename Fma>
__host__ __device__ inline double exp_fp64_with(double x, Fma fma) {
    constexpr double kInvLn2 = 0x1.71547652b82fep+0;  // 1 / ln2
    constexpr double kLn2Hi = 0x1.62e42fee00000p-1;   // ln2, 32 significant bits
    constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;  // ln2 - kLn2Hi
    x = __builtin_fmin(__builtin_fmax(x, -1000.0), 1000.0);
    const double k = __builtin_rint(x * kInvLn2);
    double r = fma(-k, kLn2Hi, x);
    r = fma(-k, kLn2Lo, r);
    // sum_{n=0}^{13} r^n / n!, innermost term first
    double p = 1.0 / 6227020800.0;  // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return __builtin_ldexp(p, (int)k);
}

// a * b + c as one three-operand instruction.  With the plain builtin the
// compiler forms the two-operand accumulate, which overwrites the addend, and
// so copies each constant of a Horner chain into a fresh register first (one
// extra move per step).
struct FmaVop3 {
    __device__ __forceinline__ double operator()(double a, double b, double c) const {
        double d;
        asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
        return d;
    }
};

__device__ __forceinline__ double exp_fp64(double x) { return exp_fp64_with(x, FmaVop3{}); }

}  // namespace fd6
