// rsv_exp.h -- exponentials for the leapfrog force (the e^{-h_t} y_t^2 term).
//
// The force needs e^{-h} once per site-update; it dominates the instruction
// count of the trajectory kernel.  These versions drop the library's explicit
// overflow / underflow range checks: v_ldexp saturates to +inf / 0 by itself,
// which gives the same results for finite inputs beyond the range; a NaN input
// gives NaN.  (For |x| so large that the reduction itself overflows -- far
// beyond any state a trajectory can accept -- the result is NaN instead of
// inf, and the trajectory is rejected either way.)
#pragma once

#include <hip/hip_runtime.h>

namespace rsv {

// e^x in FP64: x = n ln2 + r, |r| <= ln2/2, e^x = 2^n P(r).  ln2 is split into
// its FP64 value and the rounding remainder so that r carries ~1 ulp.  P is the
// degree-11 minimax polynomial for e^r (relative error 1.7e-17 after rounding
// the coefficients; gen_exp_poly.py).
__device__ __forceinline__ double exp_fast(double x) {
    const double log2e = 0x1.71547652b82fep+0;
    const double ln2_hi = 0x1.62e42fefa39efp-1;
    const double ln2_lo = 0x1.abc9e3b39803fp-56;
    const double n = __builtin_rint(x * log2e);
    double r = __builtin_fma(-n, ln2_hi, x);
    r = __builtin_fma(-n, ln2_lo, r);
    double p = 2.4995873031469468e-08;
    p = __builtin_fma(p, r, 2.7632471742635444e-07);
    p = __builtin_fma(p, r, 2.7557617915243222e-06);
    p = __builtin_fma(p, r, 2.4801485990990488e-05);
    p = __builtin_fma(p, r, 0.00019841269437402027);
    p = __builtin_fma(p, r, 0.0013888888951775489);
    p = __builtin_fma(p, r, 0.00833333333355733);
    p = __builtin_fma(p, r, 0.04166666666649043);
    p = __builtin_fma(p, r, 0.16666666666666172);
    p = __builtin_fma(p, r, 0.5000000000000018);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_amdgcn_ldexp(p, static_cast<int>(n));
}

// e^x in FP32: 2^h with h = x log2 e rounded, times e^r for the residual
// r = x - h ln2 (formed exactly by one FMA), using 1 + r since |r| < 2^-20 |x|.
__device__ __forceinline__ float exp_fast(float x) {
    const float log2e = 0x1.715476p+0f;
    const float ln2 = 0x1.62e430p-1f;
    const float h = x * log2e;
    const float r = __builtin_fmaf(-h, ln2, x);
    const float e2 = __builtin_amdgcn_exp2f(h);
    return __builtin_fmaf(e2, r, e2);
}

}  // namespace rsv
