// rsv_device.h -- device building blocks of the RSV HMC library (gfx950).
//
// Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11),
// Box-Muller normals, wavefront neighbour shifts by DPP, and wavefront
// reductions.  Written for 64-lane wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsv_exp.h"

namespace rsv {

constexpr int kWave = 64;

// Stream tags (word 3 of the Philox counter): one stream per use.
enum : uint64_t { kTagMomentum = 0, kTagAccept = 1, kTagTheta = 2, kTagStep = 3, kTagMove = 4 };

// ---------------------------------------------------------------------------
// Philox4x64-10: ten rounds; each round multiplies words 0 and 2 by the two
// round multipliers (full 128-bit products), swaps and xors with the key;
// the key advances by the two Weyl constants after every round.
// ---------------------------------------------------------------------------
// Full 128-bit product m * x as (hi, lo) from four 32 x 32 -> 64 products,
// each with a 32-bit addend that cannot overflow it (one v_mad_u64_u32
// apiece): m x = xh mh 2^64 + (xh ml + xl mh) 2^32 + xl ml.
__device__ __forceinline__ void mulhilo64(uint64_t m, uint64_t x, uint64_t& hi, uint64_t& lo) {
    const uint32_t ml = static_cast<uint32_t>(m), mh = static_cast<uint32_t>(m >> 32);
    const uint32_t xl = static_cast<uint32_t>(x), xh = static_cast<uint32_t>(x >> 32);
    const uint64_t t = static_cast<uint64_t>(xl) * ml;
    const uint64_t u = static_cast<uint64_t>(xl) * mh + (t >> 32);
    const uint64_t v = static_cast<uint64_t>(xh) * ml + static_cast<uint32_t>(u);
    const uint64_t w = static_cast<uint64_t>(xh) * mh + (u >> 32);
    hi = w + (v >> 32);
    lo = (v << 32) | static_cast<uint32_t>(t);
}

struct Philox4x64 {
    uint64_t w[4];

    __device__ static Philox4x64 encrypt(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                         uint64_t k0, uint64_t k1) {
        const uint64_t mul_a = 0xD2E7470EE14C6C93ull;
        const uint64_t mul_b = 0xCA5A826395121157ull;
        const uint64_t weyl_a = 0x9E3779B97F4A7C15ull;
        const uint64_t weyl_b = 0xBB67AE8584CAA73Bull;
#pragma unroll
        for (int round = 0; round < 10; ++round) {
            uint64_t hi_a, lo_a, hi_b, lo_b;
            mulhilo64(mul_a, c0, hi_a, lo_a);
            mulhilo64(mul_b, c2, hi_b, lo_b);
            const uint64_t n0 = hi_b ^ c1 ^ k0;
            const uint64_t n2 = hi_a ^ c3 ^ k1;
            c0 = n0;
            c1 = lo_b;
            c2 = n2;
            c3 = lo_a;
            k0 += weyl_a;
            k1 += weyl_b;
        }
        Philox4x64 r;
        r.w[0] = c0; r.w[1] = c1; r.w[2] = c2; r.w[3] = c3;
        return r;
    }
};

// Top 52 bits of a word, centred in their cell: exact, strictly inside (0,1).
__device__ inline double unit_open(uint64_t bits) {
    return (static_cast<double>(bits >> 12) + 0.5) * 0x1p-52;
}

// Four uniforms of block `idx` of stream (sweep, chain, tag) under key (seed, 0).
__device__ inline void uniforms4(uint64_t seed, uint64_t idx, uint64_t sweep, uint64_t chain,
                                 uint64_t tag, double u[4]) {
    const Philox4x64 x = Philox4x64::encrypt(idx, sweep, chain, tag, seed, 0ull);
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = unit_open(x.w[i]);
}

// Box-Muller on one pair: radius sqrt(-2 ln u0), angle 2 pi u1.
__device__ inline void gauss_pair(double u0, double u1, double& z0, double& z1) {
    const double radius = sqrt(-2.0 * log_unit(u0));
    double s, c;
    sincos_2pi(u1, s, c);
    z0 = radius * c;
    z1 = radius * s;
}

// Box-Muller in FP32 on one pair of uniforms: the radius from the hardware
// base-2 logarithm and square root (sqrt(-2 ln2 log2 u0)), the angle by
// sincos_2pi_f32.
__device__ inline void gauss_pair_f32(float u0, float u1, float& z0, float& z1) {
    const float l2 = __builtin_amdgcn_logf(u0);
    const float radius = __builtin_amdgcn_sqrtf(-1.38629436112f * l2);
    float s, c;
    sincos_2pi_f32(u1, s, c);
    z0 = radius * c;
    z1 = radius * s;
}

// Momentum normals of one Philox block of a chain's momentum stream, in the
// path's precision.  FP64: block idx holds sites 4 idx .. 4 idx + 3, the
// normals of gauss_pair on the block's four 52-bit uniforms.  FP32-mixed:
// block idx holds sites 8 idx .. 8 idx + 7; word q gives sites 8 idx + 2q
// and + 2q + 1 by Box-Muller in FP32 on u0 from its top 40 bits and u1 from
// its low 24 (each centred in its cell, u0 rounded to FP32).  The trajectory
// kernel and rsv_hmc_momenta both draw here.
template <typename R>
constexpr int kMomentumBlock = sizeof(R) == sizeof(double) ? 4 : 8;

template <typename R>
__device__ inline void momentum_normals(uint64_t seed, uint64_t idx, uint64_t sweep,
                                        uint64_t chain, R (&z)[kMomentumBlock<R>]) {
    if constexpr (sizeof(R) == sizeof(double)) {
        double u[4];
        uniforms4(seed, idx, sweep, chain, kTagMomentum, u);
        gauss_pair(u[0], u[1], z[0], z[1]);
        gauss_pair(u[2], u[3], z[2], z[3]);
    } else {
        const Philox4x64 x = Philox4x64::encrypt(idx, sweep, chain, kTagMomentum, seed, 0ull);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t w = x.w[q];
            const uint32_t top = static_cast<uint32_t>(w >> 32);
            const uint32_t mid = static_cast<uint32_t>(w >> 24) & 0xFFu;
            const uint32_t low = static_cast<uint32_t>(w) & 0xFFFFFFu;
            // ((w >> 24) + 1/2) 2^-40 and ((w & 0xFFFFFF) + 1/2) 2^-24
            const float u0 = __builtin_fmaf(static_cast<float>(top), 0x1p-32f,
                                            __builtin_fmaf(static_cast<float>(mid), 0x1p-40f,
                                                           0x1p-41f));
            const float u1 = __builtin_fmaf(static_cast<float>(low), 0x1p-24f, 0x1p-25f);
            gauss_pair_f32(u0, u1, z[2 * q], z[2 * q + 1]);
        }
    }
}

// ---------------------------------------------------------------------------
// Whole-wavefront lane shifts (DPP wave_shr:1 / wave_shl:1).  The lane at the
// end that has no source receives 0 through the bound control bit, so the
// destination needs no initial value.
// ---------------------------------------------------------------------------
__device__ inline int dpp_from_lower(int v) {  // lane l <- lane l-1
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true);
}
__device__ inline int dpp_from_upper(int v) {  // lane l <- lane l+1
    return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true);
}

__device__ inline float from_lower(float v) {
    return __builtin_bit_cast(float, dpp_from_lower(__builtin_bit_cast(int, v)));
}
__device__ inline float from_upper(float v) {
    return __builtin_bit_cast(float, dpp_from_upper(__builtin_bit_cast(int, v)));
}
__device__ inline double from_lower(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = static_cast<uint32_t>(dpp_from_lower(static_cast<int>(b)));
    const uint32_t hi = static_cast<uint32_t>(dpp_from_lower(static_cast<int>(b >> 32)));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}
__device__ inline double from_upper(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = static_cast<uint32_t>(dpp_from_upper(static_cast<int>(b)));
    const uint32_t hi = static_cast<uint32_t>(dpp_from_upper(static_cast<int>(b >> 32)));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// ---------------------------------------------------------------------------
// Values that are equal on every active lane of the wavefront (per-tile
// constants), moved to scalar registers: the loop then reads them as scalar
// operands instead of holding a copy in every lane.
// ---------------------------------------------------------------------------
__device__ inline int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline float wave_uniform(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ inline double wave_uniform(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(b)));
    const uint32_t hi =
        static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(b >> 32)));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// ---------------------------------------------------------------------------
// Compensated accumulation: (sum, error) pairs, merged by Knuth's TwoSum so
// the merge is exact up to the final rounding and independent of magnitude
// order.
// ---------------------------------------------------------------------------
struct Comp {
    double s, c;
};

__device__ inline void comp_add(Comp& a, double x) {
#pragma clang fp contract(off)
    const double t = a.s + x;
    const double bp = t - a.s;
    const double err = (a.s - (t - bp)) + (x - bp);
    a.s = t;
    a.c += err;
}

__device__ inline Comp comp_merge(Comp a, Comp b) {
#pragma clang fp contract(off)
    const double t = a.s + b.s;
    const double bp = t - a.s;
    const double err = (a.s - (t - bp)) + (b.s - bp);
    Comp r;
    r.s = t;
    r.c = a.c + b.c + err;
    return r;
}

// Compensated butterfly sums of N quantities over the 64 lanes (their merges
// interleave), over the levels off = top, top/2, ..., 1; each pair is
// ordered by lane so both partners compute the same merge, and with the full
// butterfly (top = 32) every lane ends with the same totals.  With values
// only in lanes [0, 2 top), the levels above top would merge every such lane
// with zeros, which leaves it unchanged (up to the sign of an exact zero),
// so lane 0 ends with the same totals as the full butterfly.
template <int N>
__device__ inline void wave_comp_sum_n(Comp (&v)[N], int top = kWave / 2) {
    for (int off = top; off >= 1; off >>= 1) {
        const bool low = (threadIdx.x & off) == 0;
#pragma unroll
        for (int q = 0; q < N; ++q) {
            Comp o;
            o.s = __shfl_xor(v[q].s, off, kWave);
            o.c = __shfl_xor(v[q].c, off, kWave);
            v[q] = low ? comp_merge(v[q], o) : comp_merge(o, v[q]);
        }
    }
}

// wave_sum of N quantities at once: the butterflies interleave, each
// quantity's additions are those of wave_sum.
template <int N>
__device__ inline void wave_sum_n(double (&v)[N]) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const bool low = (threadIdx.x & off) == 0;
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const double o = __shfl_xor(v[q], off, kWave);
            v[q] = low ? (v[q] + o) : (o + v[q]);
        }
    }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(v, off, kWave);
        const bool low = (threadIdx.x & off) == 0;
        v = low ? (v + o) : (o + v);
    }
    return v;
}

}  // namespace rsv
