// rsv_exp.h -- elementary functions of the trajectory kernel.
//
// The force needs e^{-h} once per site-update; it dominates the instruction
// count of the trajectory kernel.  The per-trajectory parts (momentum draw,
// dH terms) use the same kind of short, branch-free versions instead of the
// library's functions, which carry range checks and large-argument paths
// that the arguments here never need.  None of these functions raises or
// branches on its argument; a NaN argument gives NaN (and a NaN dH rejects
// the trajectory).  A leapfrog is volume preserving and reversible for any
// force that is a function of position alone, so the few-ulp differences
// from the library change nothing about the exactness of the chain.
#pragma once

#include <hip/hip_runtime.h>

namespace rsv {

// e^x in FP64: x = n ln2 + r, |r| <= ln2/2, e^x = 2^n P(r).  n is rounded by
// adding 1.5 * 2^52 (the sum's low word then holds n as an integer), ln2 is
// split into its FP64 value and the rounding remainder so that r carries
// ~1 ulp, P is the degree-10 minimax polynomial for e^r (relative error
// 3.3e-16 after rounding the coefficients; gen_exp_poly.py), and 2^n is
// applied by adding n to the exponent field.  n is clamped to [-1022, 1023],
// so 708 < |x| < 745 gives a finite tiny or huge value of the right side;
// beyond that the result saturates explicitly: +inf above ln(DBL_MAX), 0
// below ln of the smallest subnormal, NaN for NaN.  (Without the saturation,
// arguments past the range of the reduction -- |x| > 2^51, which only a
// diverged trajectory produces -- would add a meaningless n to the exponent
// of an infinite polynomial value and return an arbitrary finite number,
// and dH must be +inf or NaN there so that the proposal is rejected.)
// Worst relative error on |x| <= 700: 4.7e-16 (4 ulp).  exp_fast<false>
// leaves out the clamp and the saturation, which change nothing for
// |x| <= 708: for callers that have checked the range of their arguments.
template <bool SATURATE = true>
__device__ __forceinline__ double exp_fast(double x) {
    const double log2e = 0x1.71547652b82fep+0;
    const double ln2_hi = 0x1.62e42fefa39efp-1;
    const double ln2_lo = 0x1.abc9e3b39803fp-56;
    const double shift = 0x1.8p52;
    const double t = __builtin_fma(x, log2e, shift);
    const double n = t - shift;
    double r = __builtin_fma(-n, ln2_hi, x);
    r = __builtin_fma(-n, ln2_lo, r);
    double p = 2.749029984051582e-07;
    p = __builtin_fma(p, r, 2.763997818821441e-06);
    p = __builtin_fma(p, r, 2.480191277326453e-05);
    p = __builtin_fma(p, r, 0.00019841170822930575);
    p = __builtin_fma(p, r, 0.0013888888503440534);
    p = __builtin_fma(p, r, 0.008333333385165677);
    p = __builtin_fma(p, r, 0.04166666666841235);
    p = __builtin_fma(p, r, 0.16666666666556093);
    p = __builtin_fma(p, r, 0.49999999999997297);
    p = __builtin_fma(p, r, 1.0000000000000067);
    p = __builtin_fma(p, r, 1.0);
    int ni = __double2loint(t);
    if constexpr (!SATURATE)
        return __hiloint2double(__double2hiint(p) + (ni << 20), __double2loint(p));
    ni = ni < -1022 ? -1022 : (ni > 1023 ? 1023 : ni);
    const double e = __hiloint2double(__double2hiint(p) + (ni << 20), __double2loint(p));
    // x * inf is +inf for x > 0 and NaN for a NaN x
    const double hi = x <= 709.782712893384 ? e : x * __builtin_inf();
    return x < -745.1332191019412 ? 0.0 : hi;
}

// exp_fast with the clamp and saturation behind a branch on `sat`, which is
// uniform over the wavefront (a real branch: the common case skips them).
__device__ __forceinline__ double exp_dh(double x, bool sat) {
    const double e = exp_fast<false>(x);
    if (!sat) return e;
    asm volatile("" ::: "memory");
    return exp_fast<true>(x);
}

// e^x in FP64 for the leapfrog force only, shorter than exp_fast: ln2 is
// taken as its FP64 value alone (n ln2 then carries |n| * 2.3e-17 of error),
// P is the degree-9 minimax polynomial (relative error 1.4e-14), and n is
// not clamped, so the value is e^x only for |x| <= 708; beyond that (a
// trajectory that has already diverged) it is some other number, still a
// function of x alone.  The force may be any function of position without
// affecting the exactness of the chain (the leapfrog stays reversible and
// volume preserving, and dH is formed with the saturating exp_fast); at
// |x| <= 30 the relative error stays below 1.5e-14, which moves h after a
// trajectory by orders of magnitude less than 1e-12 of its scale.
__device__ __forceinline__ double exp_force(double x) {
    const double log2e = 0x1.71547652b82fep+0;
    const double ln2 = 0x1.62e42fefa39efp-1;
    const double shift = 0x1.8p52;
    const double t = __builtin_fma(x, log2e, shift);
    const double n = t - shift;
    const double r = __builtin_fma(-n, ln2, x);
    double p = 2.748420005832407e-06;
    p = __builtin_fma(p, r, 2.4884235753499622e-05);
    p = __builtin_fma(p, r, 0.00019841591661598775);
    p = __builtin_fma(p, r, 0.0013888802292674836);
    p = __builtin_fma(p, r, 0.008333333006269941);
    p = __builtin_fma(p, r, 0.04166666703643907);
    p = __builtin_fma(p, r, 0.1666666666781916);
    p = __builtin_fma(p, r, 0.4999999999944855);
    p = __builtin_fma(p, r, 0.999999999999893);
    p = __builtin_fma(p, r, 1.000000000000013);
    const int ni = __double2loint(t);
    return __hiloint2double(__double2hiint(p) + (ni << 20), __double2loint(p));
}

// ln u for u in (0, 1]: u = 2^e m with m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(s), s = (m - 1) / (m + 1), |s| <= 0.1716, by its Taylor
// series through s^19 (truncation < 3e-17 relative).
__device__ __forceinline__ double log_unit(double u) {
    int e = __builtin_amdgcn_frexp_exp(u);
    double m = __builtin_amdgcn_frexp_mant(u);  // [0.5, 1)
    if (m < 0x1.6a09e667f3bcdp-1) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    double q = 2.0 / 19.0;
    q = __builtin_fma(q, s2, 2.0 / 17.0);
    q = __builtin_fma(q, s2, 2.0 / 15.0);
    q = __builtin_fma(q, s2, 2.0 / 13.0);
    q = __builtin_fma(q, s2, 2.0 / 11.0);
    q = __builtin_fma(q, s2, 2.0 / 9.0);
    q = __builtin_fma(q, s2, 2.0 / 7.0);
    q = __builtin_fma(q, s2, 2.0 / 5.0);
    q = __builtin_fma(q, s2, 2.0 / 3.0);
    const double ln2_hi = 0x1.62e42fefa39efp-1;
    const double ln2_lo = 0x1.abc9e3b39803fp-56;
    const double de = static_cast<double>(e);
    // ln m = 2s + s^3 q
    const double lnm = __builtin_fma(s * s2, q, 2.0 * s);
    return __builtin_fma(de, ln2_hi, __builtin_fma(de, ln2_lo, lnm));
}

// sin and cos of 2 pi u for u in [0, 1]: 4u = k + r exactly (k integer,
// |r| <= 1/2), angle th = r pi/2 in [-pi/4, pi/4] from a two-part pi/2,
// Taylor series through th^17 (sin) and th^16 (cos), then the quadrant k.
__device__ __forceinline__ void sincos_2pi(double u, double& sn, double& cs) {
    const double x4 = 4.0 * u;
    const double k = __builtin_rint(x4);
    const double r = x4 - k;
    const double pio2_hi = 0x1.921fb54442d18p+0;
    const double pio2_lo = 0x1.1a62633145c07p-54;
    const double th = __builtin_fma(r, pio2_hi, r * pio2_lo);
    const double t2 = th * th;
    double ps = 1.0 / 355687428096000.0;           // 1/17!
    ps = __builtin_fma(ps, t2, -1.0 / 1307674368000.0);
    ps = __builtin_fma(ps, t2, 1.0 / 6227020800.0);
    ps = __builtin_fma(ps, t2, -1.0 / 39916800.0);
    ps = __builtin_fma(ps, t2, 1.0 / 362880.0);
    ps = __builtin_fma(ps, t2, -1.0 / 5040.0);
    ps = __builtin_fma(ps, t2, 1.0 / 120.0);
    ps = __builtin_fma(ps, t2, -1.0 / 6.0);
    const double s = __builtin_fma(th * t2, ps, th);
    double pc = 1.0 / 20922789888000.0;            // 1/16!
    pc = __builtin_fma(pc, t2, -1.0 / 87178291200.0);
    pc = __builtin_fma(pc, t2, 1.0 / 479001600.0);
    pc = __builtin_fma(pc, t2, -1.0 / 3628800.0);
    pc = __builtin_fma(pc, t2, 1.0 / 40320.0);
    pc = __builtin_fma(pc, t2, -1.0 / 720.0);
    pc = __builtin_fma(pc, t2, 1.0 / 24.0);
    pc = __builtin_fma(pc, t2, -0.5);
    const double c = __builtin_fma(t2, pc, 1.0);
    const int q = static_cast<int>(k) & 3;
    const double s_sel = (q & 1) ? c : s;
    const double c_sel = (q & 1) ? s : c;
    sn = (q & 2) ? -s_sel : s_sel;
    cs = ((q + 1) & 2) ? -c_sel : c_sel;
}

// sin and cos of 2 pi u in FP32 for u in [0, 1]: 4u = k + r exactly, angle
// th = r pi/2 in [-pi/4, pi/4], Taylor series through th^9 (sin) and th^10
// (cos) (truncation below 2e-9), then the quadrant k.
__device__ __forceinline__ void sincos_2pi_f32(float u, float& sn, float& cs) {
    const float x4 = 4.0f * u;
    const float k = __builtin_rintf(x4);
    const float th = (x4 - k) * 1.57079632679489662f;
    const float t2 = th * th;
    float ps = 1.0f / 362880.0f;
    ps = __builtin_fmaf(ps, t2, -1.0f / 5040.0f);
    ps = __builtin_fmaf(ps, t2, 1.0f / 120.0f);
    ps = __builtin_fmaf(ps, t2, -1.0f / 6.0f);
    const float s = __builtin_fmaf(th * t2, ps, th);
    float pc = -1.0f / 3628800.0f;
    pc = __builtin_fmaf(pc, t2, 1.0f / 40320.0f);
    pc = __builtin_fmaf(pc, t2, -1.0f / 720.0f);
    pc = __builtin_fmaf(pc, t2, 1.0f / 24.0f);
    pc = __builtin_fmaf(pc, t2, -0.5f);
    const float c = __builtin_fmaf(t2, pc, 1.0f);
    const int q = static_cast<int>(k) & 3;
    const float s_sel = (q & 1) ? c : s;
    const float c_sel = (q & 1) ? s : c;
    sn = (q & 2) ? -s_sel : s_sel;
    cs = ((q + 1) & 2) ? -c_sel : c_sel;
}

// e^x in FP32 for the leapfrog force: 2^(x log2 e) by the hardware base-2
// exponential.  Rounding x log2 e to FP32 changes the value by a relative
// |x| 2^-24 or so, the same as rounding h itself to FP32 does; the force may
// be any function of position (the chain stays exact, dH is formed in FP64).
__device__ __forceinline__ float exp_force(float x) {
    return __builtin_amdgcn_exp2f(x * 0x1.715476p+0f);
}

}  // namespace rsv
