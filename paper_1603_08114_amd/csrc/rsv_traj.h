// rsv_traj.h -- device code of the trajectory, finalize and resident
// kernels, shared by the translation units that instantiate them (one per
// precision and mass variant, so that they compile in parallel).
//
// Paper: T. Takaishi, arXiv:1603.08114.  The leapfrog of Sec. 3, eqs. (6)-(8)
// (mapped to per-site GPU kernels in Sec. 5, eqs. (9)-(11)) is fused here into
// one trajectory kernel that is blocked in time: each wavefront owns a tile
// of one chain, holds h, p and the per-site constants of its tile in
// registers (S contiguous sites per lane), exchanges the two boundary sites
// of each lane with its neighbours by DPP lane shifts, and runs all k steps
// without touching HBM.  Sites within k+1 of a tile's cut are recomputed by
// the neighbouring tile (halo), so every exact site is produced once.
#pragma once

#include <type_traits>

#include "rsv_device.h"
#include "rsv_exp.h"
#include "rsv_internal.h"

#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wunused-function"

namespace rsv {

namespace {
template <typename R>
__device__ inline R ghost_neighbour(R h, R mu, R phi) {
    // Substituting a_{-1} = phi a_0 (and a_{T} = phi a_{T-1}) into the interior
    // AR(1) force reproduces the end-point forces of the stationary model.
    return mu + phi * (h - mu);
}

template <typename R>
__device__ inline R exp_neg(R x);
template <>
__device__ inline double exp_neg<double>(double x) { return exp_force(-x); }
template <>
__device__ inline float exp_neg<float>(float x) { return exp_force(-x); }

// Value of the current state at a site: the stored entry plus the chain's
// pending level shift (0 unless level moves are on), rounded to the state's
// precision.  Every reader of the current state goes through this.
template <typename R>
__device__ __forceinline__ R state_at(const R* hc, int64_t t, double shift) {
    return static_cast<R>(static_cast<double>(hc[t]) + shift);
}

// Step size of one trajectory: dtau scaled by 1 + j (2u - 1), u the first
// uniform of block 0 of the step stream (every tile of a chain draws the same
// u).  Rounded step by step, without contraction, so the value is exact to
// the last bit for any caller that evaluates the same three operations.
__device__ inline double step_size(uint64_t seed, uint64_t sweep, uint64_t chain, double dtau,
                                   double jitter) {
#pragma clang fp contract(off)
    if (!(jitter > 0.0)) return dtau;
    double u[4];
    uniforms4(seed, 0, sweep, chain, kTagStep, u);
    const double w = 2.0 * u[0] - 1.0;
    const double f = 1.0 + jitter * w;
    return dtau * f;
}

// ---------------------------------------------------------------------------
// Per-site arithmetic shared by the trajectory kernel and the resident
// kernel (so that both produce bitwise the same results).
// ---------------------------------------------------------------------------

// One site of a momentum step (kick) p += dk g(h) of eqs. (6)-(8): with the
// per-site constants dc = -dk (c_base - r/sigma_u^2) and ds = dk y^2 / 2 and
// the per-chain mda = -dk alpha, db = dk beta, the force term is
// dc + mda h + db (h_l + h_r) + ds e^{-h}.
template <typename R, bool RET>
__device__ __forceinline__ R kick_site(R p, R dc, R ds, R mda, R db, R h, R hl, R hr) {
    R acc = p + dc;
    acc += mda * h;
    acc += db * (hl + hr);
    if constexpr (RET) acc += ds * exp_neg<R>(h);
    return acc;
}

// A kick with the constants of a step of dt, scaled by the kick's factor kf
// (Forest-Ruth's unequal kicks).
template <typename R, bool RET>
__device__ __forceinline__ R kick_site_scaled(R p, R kf, R dc, R ds, R mda, R db, R h, R hl,
                                              R hr) {
    R acc = dc + mda * h;
    acc += db * (hl + hr);
    if constexpr (RET) acc += ds * exp_neg<R>(h);
    return p + kf * acc;
}

// Per-lane sums of the dH pass: dH, the statistics {B, B2, BB, D1, D2} of
// h' (s1) and of h (s0), and S = sum y^2 e^{-h} of h' and h.
struct DhSums {
    double dH, s1[5], s0[5], sy1, sy0;
};

// Adds exact site t to the sums: the per-site difference of H(h', p') -
// H(h, p) (kinetic term, y and ln RV terms, the bond to site t+1 when
// has_next, the stationary prior of site 0 when first) and the site's
// statistics.  h1 = h'_t, h0 = h_t, pj = p'_t, im = 1/m_t, yy = y_t^2,
// rr = ln RV_t, h1n / h0n the next site's values.  Returns h1 - mu, h0 - mu.
// sat (uniform over the wavefront) selects the saturating exponential;
// without it the caller has checked |h0| <= 700 and |h0 - h1| <= 700, where
// both give the same values.
template <bool RET>
__device__ __forceinline__ void dh_site(DhSums& D, double h1, double h0, double pj, double im,
                                        double yy, double rr, bool rv, bool has_next, double h1n,
                                        double h0n, bool first, double mu, double phi, double xi,
                                        double inv_se, double inv_su, bool sat, double& a1,
                                        double& a0) {
    double d = 0.5 * pj * pj * im;
    if (RET) {
        const double ye0 = yy * exp_dh(-h0, sat);
        const double x10 = exp_dh(h0 - h1, sat);  // e^{-h1} / e^{-h0}
        d += 0.5 * (h1 - h0) + 0.5 * ye0 * (x10 - 1.0);
        D.sy1 += ye0 * x10;
        D.sy0 += ye0;
    }
    if (rv) {
        const double c = rr - xi;
        const double e1 = c - h1, e0 = c - h0;
        d += (e1 - e0) * (e1 + e0) * (0.5 * inv_su);
    }
    a1 = h1 - mu;
    a0 = h0 - mu;
    if (has_next) {
        const double d1 = (h1n - mu) - phi * a1;
        const double d0 = (h0n - mu) - phi * a0;
        d += (d1 - d0) * (d1 + d0) * (0.5 * inv_se);
        D.s1[2] += a1 * (h1n - mu);
        D.s0[2] += a0 * (h0n - mu);
    }
    if (first) d += (1.0 - phi * phi) * (a1 - a0) * (a1 + a0) * (0.5 * inv_se);
    D.dH += d;
    const double e1 = rr - h1 - xi, e0 = rr - h0 - xi;
    D.s1[0] += a1; D.s1[1] += a1 * a1; D.s1[3] += e1; D.s1[4] += e1 * e1;
    D.s0[0] += a0; D.s0[1] += a0 * a0; D.s0[3] += e0; D.s0[4] += e0 * e0;
}

// ---------------------------------------------------------------------------
// Trajectory kernel: momentum refresh, k leapfrog steps, per-site dH terms and
// sufficient statistics of h' and h, for one tile per group of NW wavefronts.
// Lane g = 64*wave + lane of a tile holds sites [la + g*S, la + (g+1)*S).
// Within a wavefront the end sites of each lane move by DPP lane shifts;
// between the NW wavefronts of a tile they pass through LDS (one barrier per
// leapfrog step, slots double-buffered by step parity).
// ---------------------------------------------------------------------------
template <typename R, int NW>
struct TileShared {
    R left[2][NW];   // h of the first site of each wavefront
    R right[2][NW];  // h of the last site of each wavefront
    double red[NW][kNQ];
    double up1[NW], up0[NW];
};

// The tile's starting h, y^2 and ln RV pass through LDS (laid out
// [quantity][site j][lane], rows padded by one element): the wavefront reads
// its block of 64 S sites from memory in coalesced rounds (round r: site
// base + 64 r + lane) and scatters them to their owners' slots, and each lane
// then reads its S sites.  Reading each lane's S neighbouring sites directly
// puts addresses S elements apart across the lanes of one load, which costs
// the memory pipeline several times more per element.  FP64 tiles keep the
// values there for the dH pass after the leapfrog loop (so it does not
// re-read them: the tiles in flight on one XCD hold more than its L2); the
// FP32 dH pass reads h0 from there and the FP64 data from memory.  On for
// every FP32 shape (at most 50 KB per block) and for FP64 while a block's
// copy stays under 51 KB (S * NW * tiles per block <= 32).
template <typename R, int S, int NW, int TPB>
struct Stage {
    static constexpr bool on = sizeof(R) == sizeof(float) || S * NW * TPB <= 32;
    static constexpr int row = 64 * NW + 1;  // a quantity's row of one site j
    static constexpr int n = on ? 3 * S * row : 1;
};

// Orders a wavefront's LDS writes before its reads of other lanes' slots
// (the slots written and read belong to this wavefront only).
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1/m_t from the stored sqrt(m_t), in FP64 with a correctly rounded division:
// the momentum is drawn as z sqrt(m_t), so the kinetic term p^2 / (2 m_t)
// formed from this value is the one of the law the momentum follows (to
// FP64 rounding), and the same value serves both ends of the trajectory.
template <typename R>
__device__ __forceinline__ double inv_mass(R sqrt_m) {
    const double s = static_cast<double>(sqrt_m);
    return 1.0 / (s * s);
}

template <typename R, int S, int NW, bool MASS, bool EDGE, bool RET, bool STAGE>
__device__ __forceinline__ void traj_tile(const TrajArgs<R>& A, TileShared<R, NW>& sh,
                                          const int tile_id, const int wv, const int lane,
                                          R* stage) {
    const TileDesc td = A.tiles[tile_id];
    const ChainDesc cd = A.chains[td.chain];
    const rsv_theta th = A.theta[td.chain];

    const int T = cd.T;
    const int t0 = td.la + (wv * kWave + lane) * S;
    const bool rv = (A.terms & RSV_TERM_RV) != 0;
    const double phi = th.phi, mu = th.mu, xi = th.xi;
    const double inv_se = 1.0 / th.sig2_eta;
    const double inv_su = rv ? 1.0 / th.sig2_u : 0.0;
    const double dt = step_size(A.seed, A.sweep, static_cast<uint64_t>(td.chain), cd.dtau, A.jitter);
    // momentum steps: dt (leapfrog), dt/2 (Omelyan: two per step), or dt
    // times a per-kick factor (Forest-Ruth: three per step)
    const double dk = A.integrator == kIntOmelyan ? 0.5 * dt : dt;
    // force g_t = c_t + alpha h_t - beta (h_{t-1} + h_{t+1}) - s_t e^{-h_t} / 2
    const double alpha = (1.0 + phi * phi) * inv_se + inv_su;
    const double beta = phi * inv_se;
    const double c_base = (RET ? 0.5 : 0.0) + xi * inv_su - mu * (1.0 - phi) * (1.0 - phi) * inv_se;
    const R mda = static_cast<R>(-dk * alpha);
    const R db = static_cast<R>(dk * beta);
    const R mu_r = static_cast<R>(mu), phi_r = static_cast<R>(phi);

    // The loads of the tile's inputs are issued first and consumed after the
    // momentum draw, which needs none of them, so that their latency overlaps
    // it: the state h, the data (y^2, ln RV), with a diagonal mass sqrt(m_t)
    // (kept for the dH pass), and the batch-means accumulators.
    R h[S], p[S], dc[S], ds[S], dtm[MASS ? S : 1], msq[MASS ? S : 1];
    R y_in[S], r_in[S];
    R acc_h[S];
    float acc_s[S], acc_q[S];
    double kin0 = 0.0;  // kinetic energy of the exact sites at the start

    const bool in_b = A.state_sel[td.chain] != 0;
    const R* hc = (in_b ? A.h_b : A.h_a) + cd.h_off;
    const double shift = A.shift ? A.shift[td.chain] : 0.0;
    R* hp = (in_b ? const_cast<R*>(A.h_a) : A.h_b) + cd.h_off;
    const R* y2 = A.y2 + cd.d_off;
    const R* lr = A.lrv + cd.d_off;
    const R* msq_tab = MASS ? A.mass_sqrt + cd.d_off : nullptr;
    constexpr int ROW = Stage<R, S, NW, (NW == 1 ? 4 : 1)>::row;
    const int g = wv * kWave + lane;
    const int wbase = td.la + wv * kWave * S;  // the wavefront's block of 64 S sites
    if constexpr (STAGE) {
        // coalesced rounds; the values go to their owners through LDS below
#pragma unroll
        for (int r = 0; r < S; ++r) {
            const int t = wbase + r * kWave + lane;
            const bool live = t < T;
            h[r] = live ? state_at(hc, t, shift) : R(0);
            y_in[r] = live ? y2[t] : R(0);
            r_in[r] = live ? lr[t] : R(0);
        }
    } else {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int t = t0 + j;
            const bool live = t < T;
            h[j] = live ? state_at(hc, t, shift) : R(0);
            y_in[j] = live ? y2[t] : R(0);
            r_in[j] = live ? lr[t] : R(0);
        }
    }
    if constexpr (MASS) {
#pragma unroll
        for (int j = 0; j < S; ++j) msq[j] = (t0 + j < T) ? msq_tab[t0 + j] : R(1);
    }
    // batch-means accumulators of the starting state (the previous sweep's
    // result) and the trace row of the previous sweep, on the exact sites,
    // read here and written back below, in the same coalesced rounds (they
    // need no per-lane order; without the stage the state is read again)
    const bool acc_on = A.acc_sum || A.acc_sq || A.h_prev_out;
    if (acc_on) {
#pragma unroll
        for (int r = 0; r < S; ++r) {
            const int t = wbase + r * kWave + lane;
            const int64_t i = cd.h_off + t;
            const bool ex = t >= td.a && t < td.b;
            if constexpr (STAGE)
                acc_h[r] = h[r];
            else
                acc_h[r] = ex ? state_at(hc, t, shift) : R(0);
            acc_s[r] = (ex && A.acc_sum) ? A.acc_sum[i] : 0.0f;
            acc_q[r] = (ex && A.acc_sq) ? A.acc_sq[i] : 0.0f;
        }
    }

    // momentum refresh p ~ N(0, m): site t takes normal t%NB of block t/NB
    // (NB = 4 in FP64, 8 in FP32; tiles start at multiples of 8); the factor
    // sqrt(m_t) is applied below, once the table has arrived
    if (A.p0) {
        const double* p0 = A.p0 + cd.h_off;
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int t = t0 + j;
            p[j] = (t < T) ? static_cast<R>(p0[t]) : R(0);
        }
    } else {
        constexpr int NB = kMomentumBlock<R>;
        static_assert(S % NB == 0, "lanes hold whole Philox blocks");
#pragma unroll
        for (int g = 0; g < S / NB; ++g) {
            R z[NB];
            momentum_normals<R>(A.seed, static_cast<uint64_t>(t0 / NB + g), A.sweep,
                                static_cast<uint64_t>(td.chain), z);
#pragma unroll
            for (int q = 0; q < NB; ++q) p[NB * g + q] = z[q];
        }
#pragma unroll
        for (int j = 0; j < S; ++j) {
            R pm = p[j];
            if constexpr (MASS) pm *= msq[MASS ? j : 0];
            p[j] = (t0 + j < T) ? pm : R(0);
        }
    }

    if constexpr (STAGE) {
        // round r, lane l held site offset o = 64 r + l of the wavefront's
        // block: lane o / S's site o % S
#pragma unroll
        for (int r = 0; r < S; ++r) {
            const int o = r * kWave + lane;
            const int slot = (o % S) * ROW + wv * kWave + o / S;
            stage[0 * S * ROW + slot] = h[r];
            stage[1 * S * ROW + slot] = y_in[r];
            stage[2 * S * ROW + slot] = r_in[r];
        }
        wave_sync_lds();
#pragma unroll
        for (int j = 0; j < S; ++j) {
            h[j] = stage[(0 * S + j) * ROW + g];
            y_in[j] = stage[(1 * S + j) * ROW + g];
            r_in[j] = stage[(2 * S + j) * ROW + g];
        }
    }
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const double yy = static_cast<double>(y_in[j]);
        const double rr = static_cast<double>(r_in[j]);
        dc[j] = static_cast<R>(-dk * (c_base - rr * inv_su));
        ds[j] = RET ? static_cast<R>(0.5 * dk * yy) : R(0);
    }
    // a non-finite value in the current state (written by the caller, since
    // accepted proposals always have a finite dH) or in theta is flagged for
    // the host, which reports it at its next call; the trajectory still runs
    // and is rejected (its dH is not finite), so the state does not change
    {
        bool bad = !(isfinite(phi) && isfinite(mu) && isfinite(xi) && isfinite(inv_se));
#pragma unroll
        for (int j = 0; j < S; ++j) bad = bad || !isfinite(static_cast<double>(h[j]));
        const uint64_t any_bad = __ballot(bad);
        if (any_bad != 0 && lane == 0) atomicOr(&A.counters[kCntNonfiniteState], 1u);
    }
    // the accumulators and the trace row of the previous sweep (the same values)
    if (acc_on) {
#pragma unroll
        for (int r = 0; r < S; ++r) {
            const int t = wbase + r * kWave + lane;
            if (t >= td.a && t < td.b) {
                const float v = static_cast<float>(acc_h[r]);
                const int64_t i = cd.h_off + t;
                if (A.acc_sum) A.acc_sum[i] = acc_s[r] + v;
                if (A.acc_sq) A.acc_sq[i] = __builtin_fmaf(v, v, acc_q[r]);
                if (A.h_prev_out) A.h_prev_out[i] = acc_h[r];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int t = t0 + j;
        const double im = MASS ? inv_mass(msq[MASS ? j : 0]) : 1.0;
        if constexpr (MASS) dtm[j] = static_cast<R>(dt * im);
        if (t >= td.a && t < td.b) {
            const double pj = static_cast<double>(p[j]);
            kin0 += 0.5 * pj * pj * im;
        }
    }

    // ---- integrator: the leapfrog of eqs. (6)-(8), Omelyan's or Forest-Ruth's ----
    // Both are a chain of momentum steps (kicks) p += dk * force(h), all
    // alike, with position steps (drifts) h += c dt p / m between them:
    //   leapfrog, k kicks:  c = 1/2, then 1 between kicks, 1/2 at the end
    //                       (adjacent half steps of consecutive steps merged);
    //   Omelyan, 2k kicks:  c = lambda, then 1 - 2 lambda and 2 lambda in
    //                       turn, lambda at the end;
    //   Forest-Ruth, 3k kicks of theta, 1 - 2 theta, theta (times dt):
    //                       c = theta/2, then (1 - theta)/2, (1 - theta)/2,
    //                       theta in turn, theta/2 at the end.
    // Per-tile constants live in scalar registers.
    const R s_mda = wave_uniform(mda), s_db = wave_uniform(db);
    const R s_mu = wave_uniform(mu_r), s_phi = wave_uniform(phi_r);
    const int n_steps = wave_uniform(cd.n_steps);
    const bool lane_first = (t0 == 0);
    const bool lane_last = (t0 + S == T);
    // only the wavefronts that hold a chain end substitute a neighbour
    const bool wave_end = __ballot(lane_first || lane_last) != 0;
    // p += dk * force(h); `par` selects the LDS slots of this kick, which
    // alternate with the kick index (a wavefront one kick ahead writes the
    // other slot while its neighbours still read this one)
    // With `scaled`, the constants are for a step of dt and the force is
    // added times the kick's factor `kf` (the same five operations per site).
    auto kick = [&](auto par_c, auto scaled_c, R kf) {
        constexpr int par = decltype(par_c)::value;
        constexpr bool scaled = decltype(scaled_c)::value;
        R hl0 = from_lower(h[S - 1]);
        R hrS = from_upper(h[0]);
        if constexpr (NW > 1) {
            if (lane == 0) sh.left[par][wv] = h[0];
            if (lane == kWave - 1) sh.right[par][wv] = h[S - 1];
            __syncthreads();
            if (lane == 0 && wv > 0) hl0 = sh.right[par][wv - 1];
            if (lane == kWave - 1 && wv < NW - 1) hrS = sh.left[par][wv + 1];
        }
        if (wave_end) {
            // a real branch: without the barrier the compiler computes the
            // substitutes in every wavefront and selects
            asm volatile("" ::: "memory");
            if (lane_first) hl0 = ghost_neighbour(h[0], s_mu, s_phi);
            if (lane_last) hrS = ghost_neighbour(h[S - 1], s_mu, s_phi);
        }
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const R hl = (j == 0) ? hl0 : h[j - 1];
            R hr = (j == S - 1) ? hrS : h[j + 1];
            if constexpr (EDGE) {
                if (j < S - 1 && t0 + j == T - 1) hr = ghost_neighbour(h[j], s_mu, s_phi);
            }
            if constexpr (scaled)
                p[j] = kick_site_scaled<R, RET>(p[j], kf, dc[j], ds[j], s_mda, s_db, h[j], hl, hr);
            else
                p[j] = kick_site<R, RET>(p[j], dc[j], ds[j], s_mda, s_db, h[j], hl, hr);
        }
    };
    using Plain = std::false_type;
    using Even = std::integral_constant<int, 0>;
    using Odd = std::integral_constant<int, 1>;
    auto integrate = [&](auto omelyan_c) {
        constexpr bool OM = decltype(omelyan_c)::value;
        constexpr double kLambda = 0.1931833275037836;
        // drift factors: first, after an even kick, after an odd kick, last
        constexpr double f_first = OM ? kLambda : 0.5;
        constexpr double f_even = OM ? 1.0 - 2.0 * kLambda : 1.0;
        constexpr double f_odd = OM ? 2.0 * kLambda : 1.0;
        const R s_first = wave_uniform(static_cast<R>(f_first * dt));
        const R s_even = wave_uniform(static_cast<R>(f_even * dt));
        const R s_odd = wave_uniform(static_cast<R>(f_odd * dt));
        // h += c p (identity mass: c = f dt; diagonal mass: c = f dt / m_t)
        auto drift = [&](auto which_c) {
            constexpr int which = decltype(which_c)::value;  // 0 first/last, 1 even, 2 odd
            constexpr double f = which == 0 ? f_first : (which == 1 ? f_even : f_odd);
            const R sc = which == 0 ? s_first : (which == 1 ? s_even : s_odd);
#pragma unroll
            for (int j = 0; j < S; ++j) {
                R c;
                if constexpr (MASS)
                    c = f == 1.0 ? dtm[MASS ? j : 0] : static_cast<R>(f) * dtm[MASS ? j : 0];
                else
                    c = sc;
                h[j] += c * p[j];
            }
        };
        using First = std::integral_constant<int, 0>;
        using AfterEven = std::integral_constant<int, 1>;
        using AfterOdd = std::integral_constant<int, 2>;
        const int n_kicks = OM ? 2 * n_steps : n_steps;
        drift(First{});
        int i = 0;
        for (; i + 2 < n_kicks; i += 2) {
            kick(Even{}, Plain{}, R(0));
            drift(AfterEven{});
            kick(Odd{}, Plain{}, R(0));
            drift(AfterOdd{});
        }
        // one or two kicks remain; `i` is even
        kick(Even{}, Plain{}, R(0));
        if (n_kicks - i == 2) {
            drift(AfterEven{});
            kick(Odd{}, Plain{}, R(0));
        }
        drift(First{});  // the last drift has the first one's factor
    };
    // Forest-Ruth: factors change with the kick index modulo 3 (a scalar)
    auto integrate_fr = [&]() {
        constexpr double kTheta = 1.3512071919596578;
        const R kf_outer = wave_uniform(static_cast<R>(kTheta));
        const R kf_mid = wave_uniform(static_cast<R>(1.0 - 2.0 * kTheta));
        const R f_half = wave_uniform(static_cast<R>(0.5 * kTheta));
        const R f_mid = wave_uniform(static_cast<R>(0.5 * (1.0 - kTheta)));
        const R f_full = wave_uniform(static_cast<R>(kTheta));
        const R c_half = wave_uniform(static_cast<R>(0.5 * kTheta * dt));
        const R c_mid = wave_uniform(static_cast<R>(0.5 * (1.0 - kTheta) * dt));
        const R c_full = wave_uniform(static_cast<R>(kTheta * dt));
        // h += c p: c = f dt (identity mass) or f dt / m_t
        auto drift_by = [&](R f, R c) {
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const R cj = MASS ? f * dtm[MASS ? j : 0] : c;
                h[j] += cj * p[j];
            }
        };
        using Scaled = std::true_type;
        const int n_kicks = 3 * n_steps;
        drift_by(f_half, c_half);
        int i = 0, m = 0;  // m = i mod 3
        for (; i + 2 < n_kicks; i += 2) {
            kick(Even{}, Scaled{}, m == 1 ? kf_mid : kf_outer);
            drift_by(m == 2 ? f_full : f_mid, m == 2 ? c_full : c_mid);
            m = m == 2 ? 0 : m + 1;
            kick(Odd{}, Scaled{}, m == 1 ? kf_mid : kf_outer);
            drift_by(m == 2 ? f_full : f_mid, m == 2 ? c_full : c_mid);
            m = m == 2 ? 0 : m + 1;
        }
        kick(Even{}, Scaled{}, m == 1 ? kf_mid : kf_outer);
        if (n_kicks - i == 2) {
            drift_by(m == 2 ? f_full : f_mid, m == 2 ? c_full : c_mid);
            m = m == 2 ? 0 : m + 1;
            kick(Odd{}, Scaled{}, m == 1 ? kf_mid : kf_outer);
        }
        drift_by(f_half, c_half);  // the last kick is the third of a step
    };
    if (A.integrator == kIntOmelyan)
        integrate(std::true_type{});
    else if (A.integrator == kIntForestRuth)
        integrate_fr();
    else
        integrate(std::false_type{});

    // ---- dH = sum over exact sites of per-site differences (FP64), and the
    //      sufficient statistics of the proposal and of the current state ----
    const double* y2d = A.y2_d + cd.d_off;
    const double* lrd = A.lrv_d + cd.d_off;
    // FP64 keeps y^2 and ln RV in the stage; FP32 reads them in FP64 from memory
    constexpr bool STAGE_DATA = STAGE && sizeof(R) == sizeof(double);
    double h0d[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int t = t0 + j;
        if constexpr (STAGE)
            h0d[j] = static_cast<double>(stage[(0 * S + j) * ROW + g]);  // 0 beyond T, as below
        else
            h0d[j] = (t < T) ? static_cast<double>(state_at(hc, t, shift)) : 0.0;
    }
    double h1_up = static_cast<double>(from_upper(h[0]));
    double h0_up = from_upper(h0d[0]);
    if constexpr (NW > 1) {
        if (lane == 0) {
            sh.up1[wv] = static_cast<double>(h[0]);
            sh.up0[wv] = h0d[0];
        }
        __syncthreads();
        if (lane == kWave - 1 && wv < NW - 1) {
            h1_up = sh.up1[wv + 1];
            h0_up = sh.up0[wv + 1];
        }
    }

    DhSums D = {-kin0, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}, 0.0, 0.0};
    double* edge = A.chain_edge + static_cast<int64_t>(td.chain) * kEdge;
    // the exponentials of the pass saturate only where an argument may leave
    // [-700, 700] (a diverged proposal, or NaN): a uniform branch per wavefront
    bool in_range = true;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const double h1j = static_cast<double>(h[j]);
        in_range = in_range && __builtin_fabs(h0d[j]) <= 700.0 && __builtin_fabs(h0d[j] - h1j) <= 700.0;
    }
    const bool sat = __ballot(!in_range) != 0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int t = t0 + j;
        if (t < td.a || t >= td.b) continue;
        const double im = MASS ? inv_mass(msq[MASS ? j : 0]) : 1.0;
        const double rr = STAGE_DATA ? static_cast<double>(stage[(2 * S + j) * ROW + g]) : lrd[t];
        const double yy = RET ? (STAGE_DATA ? static_cast<double>(stage[(1 * S + j) * ROW + g]) : y2d[t]) : 0.0;
        const double h1n = (j == S - 1) ? h1_up : static_cast<double>(h[j + (j < S - 1)]);
        const double h0n = (j == S - 1) ? h0_up : h0d[j + (j < S - 1)];
        double a1, a0;
        dh_site<RET>(D, static_cast<double>(h[j]), h0d[j], static_cast<double>(p[j]), im, yy, rr,
                     rv, t + 1 < T, h1n, h0n, t == 0, mu, phi, xi, inv_se, inv_su, sat, a1, a0);
        if (t == 0) {
            edge[0] = a1;
            edge[2] = a0;
        }
        if (t == T - 1) {
            edge[1] = a1;
            edge[3] = a0;
        }
        hp[t] = h[j];
    }

    double red[kNQ];
    red[kPartDH] = D.dH;
    red[kPartSyProp] = D.sy1;
    red[kPartSyCur] = D.sy0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        red[kPartProp + q] = D.s1[q];
        red[kPartCur + q] = D.s0[q];
    }
    wave_sum_n(red);
    if constexpr (NW > 1) {
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < kNQ; ++q) sh.red[wv][q] = red[q];
        }
        __syncthreads();
        if (wv == 0) {
#pragma unroll
            for (int q = 0; q < kNQ; ++q) {
                double v = sh.red[0][q];
                for (int x = 1; x < NW; ++x) v += sh.red[x][q];
                red[q] = v;
            }
        }
    }
    if (wv == 0 && lane == 0) {
        double* out = A.partials + static_cast<int64_t>(tile_id) * kPart;
#pragma unroll
        for (int q = 0; q < kNQ; ++q) out[q] = red[q];
    }
}

// One launch covers every tile; tiles whose chain ends inside a lane (EDGE)
// take the variant that substitutes the end-point neighbour per site.
template <typename R, int S, int NW, bool MASS, bool RET>
__device__ __forceinline__ void traj_launch_body(const TrajArgs<R>& A) {
    static_assert(S % 4 == 0, "lanes hold whole Philox blocks");
    static_assert(NW == 1 || NW == 2 || NW == 4 || NW == 8, "tile shapes");
    // NW = 1: four independent tiles per 256-thread block (no barriers);
    // NW > 1: one tile per block of NW wavefronts, so a barrier never spans
    // tiles of chains with different k.
    constexpr int kTilesPerBlock = NW == 1 ? 4 : 1;
    using St = Stage<R, S, NW, kTilesPerBlock>;
    __shared__ TileShared<R, NW> sh_all[kTilesPerBlock];
    __shared__ R stage_all[kTilesPerBlock][St::n];
    const int lane = threadIdx.x & (kWave - 1);
    // wavefront index in the block: uniform, so the tile index and everything
    // read through it stay in scalar registers
    const int wv_blk = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int w = blockIdx.x * kTilesPerBlock + wv_blk / NW;
    if (w >= A.n_list) return;  // uniform over the tile's wavefronts
    const int tile_id = A.tile_first + w;
    R* stage = stage_all[wv_blk / NW];
    if (A.tiles[tile_id].edge)
        traj_tile<R, S, NW, MASS, true, RET, St::on>(A, sh_all[wv_blk / NW], tile_id,
                                                     wv_blk % NW, lane, stage);
    else
        traj_tile<R, S, NW, MASS, false, RET, St::on>(A, sh_all[wv_blk / NW], tile_id,
                                                      wv_blk % NW, lane, stage);
}

// Identity mass.
template <typename R, int S, int NW, bool RET>
__global__ __launch_bounds__(NW == 1 ? 256 : 64 * NW)
void k_traj(TrajArgs<R> A) {
    traj_launch_body<R, S, NW, false, RET>(A);
}

// Diagonal mass.  Shapes with 32 bytes of state per lane (FP64 S = 4, FP32
// S = 8) are held to four waves per SIMD (128 registers), which they fit
// without spilling; the larger shapes need more than that in the leapfrog
// loop itself and are left uncapped (two or three waves per SIMD).
template <typename R, int S, int NW, bool RET>
__global__ __launch_bounds__(NW == 1 ? 256 : 64 * NW)
__attribute__((amdgpu_waves_per_eu(S * sizeof(R) <= 32 ? 4 : 1)))
void k_traj_mass(TrajArgs<R> A) {
    traj_launch_body<R, S, NW, true, RET>(A);
}

// ---------------------------------------------------------------------------
// Statistics of the current state over the exact range of each tile.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_stats(const TileDesc* tiles, int32_t n_tiles,
                                               const ChainDesc* chains, const rsv_theta* theta,
                                               const R* h_a, const R* h_b,
                                               const int32_t* state_sel, const double* shift,
                                               const double* y2_d, const double* lrv_d,
                                               double* partials, double* chain_edge) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (w >= n_tiles) return;
    const TileDesc td = tiles[w];
    const ChainDesc cd = chains[td.chain];
    const rsv_theta th = theta[td.chain];
    const R* hc = (state_sel[td.chain] ? h_b : h_a) + cd.h_off;
    const double sft = shift ? shift[td.chain] : 0.0;
    const double* lr = lrv_d + cd.d_off;
    const double* yy = y2_d + cd.d_off;
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int t = td.a + lane; t < td.b; t += kWave) {
        const double hv = static_cast<double>(state_at(hc, t, sft));
        const double b = hv - th.mu;
        const double e = lr[t] - hv - th.xi;
        s[0] += b;
        s[1] += b * b;
        if (t + 1 < cd.T) s[2] += b * (static_cast<double>(state_at(hc, t + 1, sft)) - th.mu);
        s[3] += e;
        s[4] += e * e;
        s[5] += yy[t] * exp_fast(-hv);
        if (t == 0) chain_edge[static_cast<int64_t>(td.chain) * kEdge + 2] = b;
        if (t == cd.T - 1) chain_edge[static_cast<int64_t>(td.chain) * kEdge + 3] = b;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) s[q] = wave_sum(s[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 5; ++q) partials[static_cast<int64_t>(w) * kPart + kPartCur + q] = s[q];
        partials[static_cast<int64_t>(w) * kPart + kPartSyCur] = s[5];
    }
}

// ---------------------------------------------------------------------------
// theta update: Gibbs mu -> phi -> sigma_eta^2 -> xi -> sigma_u^2 from the
// sufficient statistics.  Random numbers come from the theta stream: block 0
// (z_mu, z_phi, u_phi), block 1 (z_xi), blocks 2..33 and 34..65 the Gamma
// attempts of sigma_eta^2 and sigma_u^2 (Marsaglia-Tsang, no squeeze; the
// first accepted attempt is the draw).  None of these depends on the other
// parameters except through the known Gamma shapes a + T/2, so one lane per
// block evaluates them all in parallel; one lane then does the algebra.
// The level move draws from its own stream (tag 4): block 0 (z_c, u_c) and
// the Gamma(T/2) attempts in blocks 1..32; they follow the theta blocks and
// the Metropolis uniform in the draw index.
// ---------------------------------------------------------------------------
constexpr int kGammaTries = 32;
constexpr int kGammaEtaBlock = 2, kGammaUBlock = 2 + kGammaTries;
constexpr int kThetaBlocks = 2 + 2 * kGammaTries;
constexpr int kAcceptBlock = kThetaBlocks;
constexpr int kMoveBlock = kThetaBlocks + 1;            // block 0 of the move stream
constexpr int kMoveGammaBlock = kMoveBlock + 1;         // its Gamma attempts
constexpr int kDrawBlocks = kMoveGammaBlock + kGammaTries;
// Gamma attempts evaluated in parallel; the rest only when all of these are
// rejected (Marsaglia-Tsang accepts > 99% of attempts for shapes >= 1.5).
// (A build-time knob: the draws do not depend on it, only how many attempts
// are evaluated before the serial continuation.)
#ifndef RSV_GAMMA_PARALLEL
#define RSV_GAMMA_PARALLEL 4
#endif
constexpr int kGammaParallel = RSV_GAMMA_PARALLEL;

__device__ inline bool gamma_block(int b) {
    return (b >= kGammaEtaBlock && b < kThetaBlocks) || b >= kMoveGammaBlock;
}
__device__ inline int gamma_index(int b) {  // attempt number within its Gamma draw
    if (b >= kMoveGammaBlock) return b - kMoveGammaBlock;
    return b < kGammaUBlock ? b - kGammaEtaBlock : b - kGammaUBlock;
}

struct ThetaDraws {
    double z_mu, z_phi, u_phi, z_xi, log_u_accept, z_c, u_c;
    double g_val[kDrawBlocks];    // d v^3 of each Gamma attempt
    int g_ok[kDrawBlocks];        // attempt accepted
};

__device__ void gamma_attempt(int b, ThetaDraws& D, const double u[4], double z0, double shape) {
#pragma clang fp contract(off)
    const double d = shape - 1.0 / 3.0;
    const double cc = 1.0 / sqrt(9.0 * d);
    double v = 1.0 + cc * z0;
    int ok = 0;
    if (v > 0.0) {
        v = v * v * v;
        ok = log(u[2]) < 0.5 * z0 * z0 + d - d * v + d * log(v);
    }
    D.g_ok[b] = ok;
    D.g_val[b] = ok ? d * v : d;
}

// Draw block b for chain c: theta stream blocks, the Metropolis uniform, the
// level move's blocks.
__device__ void theta_draw_block(int b, ThetaDraws& D, uint64_t seed, uint64_t sweep, uint64_t c,
                                 double shape_eta, double shape_u, double shape_level) {
#pragma clang fp contract(off)
    double u[4];
    if (b == kAcceptBlock) {
        uniforms4(seed, 0, sweep, c, kTagAccept, u);
        D.log_u_accept = log(u[0]);
        return;
    }
    if (b >= kMoveBlock) {
        uniforms4(seed, static_cast<uint64_t>(b - kMoveBlock), sweep, c, kTagMove, u);
        double z0, z1;
        gauss_pair(u[0], u[1], z0, z1);
        if (b == kMoveBlock) {
            D.z_c = z0;
            D.u_c = u[2];
        } else {
            gamma_attempt(b, D, u, z0, shape_level);
        }
        return;
    }
    uniforms4(seed, static_cast<uint64_t>(b), sweep, c, kTagTheta, u);
    double z0, z1;
    gauss_pair(u[0], u[1], z0, z1);
    if (b == 0) {
        D.z_mu = z0;
        D.z_phi = z1;
        D.u_phi = u[2];
    } else if (b == 1) {
        D.z_xi = z0;
    } else {
        gamma_attempt(b, D, u, z0, b < kGammaUBlock ? shape_eta : shape_u);
    }
}

__device__ double first_gamma(const ThetaDraws& D, int first, bool& ran_out) {
    for (int i = 0; i < kGammaTries; ++i)
        if (D.g_ok[first + i]) return D.g_val[first + i];
    ran_out = true;
    return D.g_val[first];  // d, the attempt's fallback
}

// Level move along h -> h + c, mu -> mu + c (xi -> xi - c with the RV term):
// the return term gives e^{-c} ~ Gamma(T/2, rate S/2) with S = sum y^2 e^{-h},
// and the prior ratio of mu (and xi) is the Metropolis test; without the
// return term c is drawn from the Gaussian prior factors.  Returns the c
// applied (0 when rejected) and moves cur.mu / cur.xi.
__device__ double level_move(rsv_theta& cur, double S, const rsv_prior& pr, int terms,
                             const ThetaDraws& D, bool& ran_out) {
#pragma clang fp contract(off)
    const bool rv = (terms & RSV_TERM_RV) != 0;
    double c;
    bool accept;
    if (terms & RSV_TERM_RETURN) {
        const double g = first_gamma(D, kMoveGammaBlock, ran_out);
        c = -log(2.0 * g / S);
        const double dm0 = cur.mu - pr.mu_mean, dm1 = cur.mu + c - pr.mu_mean;
        double log_a = -0.5 * dm1 * dm1 / pr.mu_var - (-0.5 * dm0 * dm0 / pr.mu_var);
        if (rv) {
            const double dx0 = cur.xi - pr.xi_mean, dx1 = cur.xi - c - pr.xi_mean;
            log_a += -0.5 * dx1 * dx1 / pr.xi_var - (-0.5 * dx0 * dx0 / pr.xi_var);
        }
        accept = isfinite(c) && log(D.u_c) < log_a;
    } else {
        const double prec = 1.0 / pr.mu_var + (rv ? 1.0 / pr.xi_var : 0.0);
        const double lin = (pr.mu_mean - cur.mu) / pr.mu_var
                         + (rv ? (cur.xi - pr.xi_mean) / pr.xi_var : 0.0);
        c = lin / prec + D.z_c / sqrt(prec);
        accept = true;
    }
    if (!accept) return 0.0;
    cur.mu += c;
    if (rv) cur.xi -= c;
    return c;
}


__device__ rsv_theta gibbs_theta(const double st[7], double n, rsv_theta cur,
                                 const rsv_prior& pr, int terms, const ThetaDraws& D,
                                 bool& ran_out) {
#pragma clang fp contract(off)
    const double B = st[0], B2 = st[1], BB = st[2], D1 = st[3], D2 = st[4];
    const double bf = st[5], bl = st[6];
    rsv_theta nxt = cur;

    // mu: Gaussian; precision from the stationary start and T-1 transitions
    {
        const double one_m_phi = 1.0 - cur.phi;
        const double prec = 1.0 / pr.mu_var
                          + ((1.0 - cur.phi * cur.phi) + (n - 1.0) * one_m_phi * one_m_phi)
                                / cur.sig2_eta;
        const double lin = (pr.mu_mean - cur.mu) / pr.mu_var
                         + ((1.0 - cur.phi * cur.phi) * bf
                            + one_m_phi * ((B - bf) - cur.phi * (B - bl))) / cur.sig2_eta;
        nxt.mu = cur.mu + lin / prec + D.z_mu / sqrt(prec);
    }
    const double eps = nxt.mu - cur.mu;
    // a_t = b_t - eps;  Q(phi) = sum a^2 - 2 phi sum a_t a_{t+1} + phi^2 sum_{interior} a^2
    const double sum_aa = B2 - 2.0 * eps * B + n * eps * eps;
    const double lag = BB - eps * (2.0 * B - bf - bl) + (n - 1.0) * eps * eps;
    const double inner = (B2 - bf * bf - bl * bl) - 2.0 * eps * (B - bf - bl) + (n - 2.0) * eps * eps;
    // phi: independence proposal from the Gaussian factor, corrected by sqrt(1-phi^2)
    {
        const double cand = lag / inner + D.z_phi * sqrt(cur.sig2_eta / inner);
        if (fabs(cand) < 1.0) {
            const double ratio = (1.0 - cand * cand) / (1.0 - cur.phi * cur.phi);
            if (D.u_phi * D.u_phi < ratio) nxt.phi = cand;
        }
    }
    {
        const double q = sum_aa - 2.0 * nxt.phi * lag + nxt.phi * nxt.phi * inner;
        nxt.sig2_eta = (pr.eta_scale + 0.5 * q) / first_gamma(D, kGammaEtaBlock, ran_out);
    }
    if (terms & RSV_TERM_RV) {
        const double prec = 1.0 / pr.xi_var + n / cur.sig2_u;
        const double lin = (pr.xi_mean - cur.xi) / pr.xi_var + D1 / cur.sig2_u;
        nxt.xi = cur.xi + lin / prec + D.z_xi / sqrt(prec);
        const double f = nxt.xi - cur.xi;
        const double ss = D2 - 2.0 * f * D1 + n * f * f;
        nxt.sig2_u = (pr.u_scale + 0.5 * ss) / first_gamma(D, kGammaUBlock, ran_out);
    }
    return nxt;
}

// ---------------------------------------------------------------------------
// Per-chain finalize: reduce tile partials (compensated, fixed order), the
// Metropolis test, the choice of statistics, and the theta update.
// ---------------------------------------------------------------------------

// Random numbers of chain c's Metropolis test, level move and theta update,
// by `nt` lanes (lane `tid` evaluates blocks tid, tid + nt, ...); the Gamma
// attempts beyond the first kGammaParallel wait for finalize_decide.
__device__ void finalize_draws(const FinalizeArgs& A, const int c, const int T, const int tid,
                               const int nt, ThetaDraws& draws) {
    const double n = static_cast<double>(T);
    const bool need_theta = A.do_theta != 0;
    const bool need_accept = A.do_metropolis && !A.log_u;
    const bool need_move = A.do_theta && A.level_move;
    for (int b = tid; b < kDrawBlocks; b += nt) {
        const bool need = b < kThetaBlocks ? need_theta
                                           : (b == kAcceptBlock ? need_accept : need_move);
        if (need && !(gamma_block(b) && gamma_index(b) >= kGammaParallel))
            theta_draw_block(b, draws, A.seed, A.sweep, static_cast<uint64_t>(c),
                             A.prior.eta_shape + 0.5 * n, A.prior.u_shape + 0.5 * n, 0.5 * n);
    }
}

// What the finalize decided for one chain.
struct Decision {
    bool accepted;
    double shift;   // the chain's pending level shift after this sweep
};

// What the decision reads of chain c besides its totals: the edge values,
// the pending level shift of the current state, the caller's ln u (if given)
// and theta.  Loaded by the deciding lane before the reductions, so that
// their memory latency overlaps them.
struct ChainIn {
    double edge[kEdge];
    double shift;
    double log_u;
    rsv_theta th;
};

__device__ __forceinline__ ChainIn load_chain_in(const FinalizeArgs& A, const int c) {
    ChainIn in;
    const double* ce = A.chain_edge + static_cast<int64_t>(c) * kEdge;
#pragma unroll
    for (int q = 0; q < kEdge; ++q) in.edge[q] = ce[q];
    in.shift = A.shift ? A.shift[c] : 0.0;
    in.log_u = A.log_u ? A.log_u[c] : 0.0;
    in.th = A.theta[c];
    return in;
}

// Metropolis test, statistics and theta update of chain c from its totals
// tot[kNQ] (dH, statistics of h' and h, S of h' and h) and what load_chain_in
// read, by one lane.  Writes theta, the per-chain outputs and counters of A.
__device__ Decision finalize_decide(const FinalizeArgs& A, const int c, const int T,
                                    const double (&tot)[kNQ], const ChainIn& in,
                                    ThetaDraws& draws) {
    const double (&edge)[kEdge] = in.edge;
    const double shift_in = in.shift;
    // a Gamma draw whose parallel attempts were all rejected continues serially
    // up to its first accepted attempt, so the first accepted attempt is the
    // same one a fully parallel evaluation would find
    {
        const double n = static_cast<double>(T);
        const int firsts[3] = {kGammaEtaBlock, kGammaUBlock, kMoveGammaBlock};
        const bool needed[3] = {A.do_theta != 0, A.do_theta != 0,
                                A.do_theta && A.level_move != 0};
        for (int gi = 0; gi < 3; ++gi) {
            if (!needed[gi]) continue;
            bool found = false;
            for (int i = 0; i < kGammaParallel; ++i) found = found || draws.g_ok[firsts[gi] + i];
            for (int i = kGammaParallel; i < kGammaTries && !found; ++i) {
                theta_draw_block(firsts[gi] + i, draws, A.seed, A.sweep, static_cast<uint64_t>(c),
                                 A.prior.eta_shape + 0.5 * n, A.prior.u_shape + 0.5 * n, 0.5 * n);
                found = draws.g_ok[firsts[gi] + i];
            }
        }
    }
    const rsv_theta th = in.th;
    bool use_prop = false;
    if (A.do_metropolis) {
#pragma clang fp contract(off)
        const double dH = tot[kPartDH];
        const double lu = A.log_u ? in.log_u : draws.log_u_accept;
        const bool finite = isfinite(dH);
        const bool accept = finite && (lu < -dH);
        if (!finite) atomicAdd(&A.counters[kCntNonfiniteDH], 1u);
        use_prop = accept;
        if (A.delta_h_out) A.delta_h_out[c] = dH;
        if (A.accepted_out) A.accepted_out[c] = accept ? 1 : 0;
    }
    const int base = use_prop ? kPartProp : kPartCur;
    double st[7];
#pragma unroll
    for (int q = 0; q < 5; ++q) st[q] = tot[base + q];
    st[5] = use_prop ? edge[0] : edge[2];
    st[6] = use_prop ? edge[1] : edge[3];
    if (A.stats_out) {
#pragma unroll
        for (int q = 0; q < 7; ++q) A.stats_out[static_cast<int64_t>(c) * 7 + q] = st[q];
    }
    rsv_theta out = th;
    // the pending level shift belongs to the buffer that held the current state
    double shift = use_prop ? 0.0 : shift_in;
    if (A.do_theta) {
        bool ran_out = false;
        rsv_theta cur = th;
        if (A.level_move) {
            // h - mu and r - xi - h are unchanged by the move, so the statistics are too
            const double S = tot[use_prop ? kPartSyProp : kPartSyCur];
            shift += level_move(cur, S, A.prior, A.terms, draws, ran_out);
        }
        out = gibbs_theta(st, static_cast<double>(T), cur, A.prior, A.terms, draws, ran_out);
        if (ran_out) atomicAdd(&A.counters[kCntGammaExhausted], 1u);
        if (!(isfinite(out.phi) && isfinite(out.mu) && isfinite(out.xi) &&
              isfinite(out.sig2_eta) && isfinite(out.sig2_u))) {
            // statistics of a non-finite state: keep theta and the level, flag it
            atomicOr(&A.counters[kCntNonfiniteState], 1u);
            out = th;
            shift = use_prop ? 0.0 : shift_in;
        }
        A.theta[c] = out;
    }
    if (A.theta_trace) A.theta_trace[c] = out;
    return Decision{use_prop, shift};
}

// Synchronises the lanes of one wavefront through LDS.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Chain c's decision from its totals, by one lane: finalize_decide, then the
// state selector and the shift.
__device__ __forceinline__ void finalize_commit(const FinalizeArgs& A, const int c, const int T,
                                                const double (&tot)[kNQ], const ChainIn& in,
                                                ThetaDraws& draws) {
    const Decision d = finalize_decide(A, c, T, tot, in, draws);
    if (d.accepted) A.state_sel[c] ^= 1;
    if (A.shift) A.shift[c] = d.shift;
}

// Everything the finalize does for chain c, by NT threads (tid = 0..NT-1;
// NT = 64: one wavefront, which may be one of several in its block) with
// shared scratch passed in; returns in every thread.  With OWN_DRAWS false
// (NT = 64) another wavefront of the block fills `draws` meanwhile, and the
// wavefront meets it at a block barrier before the decision.
template <int NT, bool OWN_DRAWS = true>
__device__ void finalize_chain(const FinalizeArgs& A, const int c, Comp (&part)[NT / kWave][kNQ],
                               ThetaDraws& draws, const int tid) {
    static_assert(OWN_DRAWS || NT == kWave, "split draws: one reducing wavefront");
    constexpr int NW = NT / kWave;
    constexpr int NQ = kNQ;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const ChainDesc cd = A.chains[c];
    ChainIn in;
    if (tid == 0) in = load_chain_in(A, c);

    const double* chain_parts = A.partials + static_cast<int64_t>(cd.tile_begin) * kPart;
    if constexpr (NT == kWave) {
        // one wavefront, chains of at most 64 body tiles: each lane's tile
        // (and lane 0's edge tile) is loaded before the random draws, so the
        // loads' latency overlaps with them; then one quantity at a time (the
        // same additions as the general path below)
        if (cd.tile_count <= NT) {
            const bool has = tid < cd.tile_count;
            const bool has_edge = tid == 0 && cd.edge_tile >= 0;
            const double* pt = chain_parts + static_cast<int64_t>(has ? tid : 0) * kPart;
            const double* pe = A.partials + static_cast<int64_t>(has_edge ? cd.edge_tile : 0) * kPart;
            double v[NQ], ve[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                v[q] = has ? pt[q] : 0.0;
                ve[q] = has_edge ? pe[q] : 0.0;
            }
            if constexpr (OWN_DRAWS) finalize_draws(A, c, cd.T, tid, NT, draws);
            Comp acc[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                acc[q] = Comp{0.0, 0.0};
                if (has) comp_add(acc[q], v[q]);
                if (has_edge) comp_add(acc[q], ve[q]);
            }
            // tiles in lanes [0, tile_count): the butterfly from the first
            // level that pairs two of them
            int top = 0;
            if (cd.tile_count > 1) {
                top = 1;
                while (2 * top < cd.tile_count) top *= 2;
            }
            wave_comp_sum_n(acc, top);
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) part[0][q] = acc[q];
            }
        } else {
            if constexpr (OWN_DRAWS) finalize_draws(A, c, cd.T, tid, NT, draws);
            Comp acc[NQ];
            for (int q = 0; q < NQ; ++q) {
                acc[q] = Comp{0.0, 0.0};
                for (int i = tid; i < cd.tile_count; i += NT)
                    comp_add(acc[q], chain_parts[static_cast<int64_t>(i) * kPart + q]);
                if (tid == 0 && cd.edge_tile >= 0)
                    comp_add(acc[q], A.partials[static_cast<int64_t>(cd.edge_tile) * kPart + q]);
            }
            wave_comp_sum_n(acc);
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) part[0][q] = acc[q];
            }
        }
    } else {
        if constexpr (OWN_DRAWS) finalize_draws(A, c, cd.T, tid, NT, draws);
        Comp acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = Comp{0.0, 0.0};
        int i = tid;
        if constexpr (NT >= 256) {
            // chains of thousands of tiles: the partials of four tiles are
            // loaded before any is added, so their memory latencies overlap
            // (same order of additions as one tile at a time)
            for (; i + 3 * NT < cd.tile_count; i += 4 * NT) {
                double v[4][NQ];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        v[u][q] = chain_parts[static_cast<int64_t>(i + u * NT) * kPart + q];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int q = 0; q < NQ; ++q) comp_add(acc[q], v[u][q]);
            }
        }
        for (; i < cd.tile_count; i += NT) {
            const double* pp = chain_parts + static_cast<int64_t>(i) * kPart;
#pragma unroll
            for (int q = 0; q < NQ; ++q) comp_add(acc[q], pp[q]);
        }
        if (tid == 0 && cd.edge_tile >= 0) {
            const double* pp = A.partials + static_cast<int64_t>(cd.edge_tile) * kPart;
#pragma unroll
            for (int q = 0; q < NQ; ++q) comp_add(acc[q], pp[q]);
        }
        wave_comp_sum_n(acc);
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) part[wv][q] = acc[q];
        }
    }
    if constexpr (NT == kWave && OWN_DRAWS)
        wave_sync();
    else
        __syncthreads();
    if (tid != 0) return;
    double tot[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        Comp r = part[0][q];
        for (int w = 1; w < NW; ++w) r = comp_merge(r, part[w][q]);
        tot[q] = r.s + r.c;
    }
    finalize_commit(A, c, cd.T, tot, in, draws);
}

// The split finalize of chains of many tiles: block (s, c) adds slice s
// (kSliceTiles tiles) of chain c's partials, read coalesced -- thread t holds
// quantity t % 16 of tiles t / 16 + 16 j -- and stores the slice's compensated
// sums; the last block of the chain to finish (a per-chain arrival count)
// merges the slices in order and adds the edge tile (first wavefront) while
// its other wavefronts draw the chain's random numbers, then runs
// finalize_commit.  One block per slice spreads the reads of
// a long chain's partials over many compute units.
template <int NT>
__global__ __launch_bounds__(NT) void k_finalize_split(FinalizeArgs A) {
    static_assert(NT == 256 && kSliceTiles * kPart % NT == 0, "slice layout");
    constexpr int kLoads = kSliceTiles * kPart / NT;
    constexpr int kMergeChunk = 32;  // slices per chunk of the final merge
    constexpr int kMergeLoads = (kMergeChunk * 2 * kNQ + kWave - 1) / kWave;
    __shared__ Comp part[NT / kWave][kNQ];
    __shared__ double merge_buf[kMergeLoads * kWave];
    __shared__ ThetaDraws draws;
    __shared__ int last;
    const int c = A.chain_first + static_cast<int>(blockIdx.y);
    const int sl = blockIdx.x;
    const ChainDesc cd = A.chains[c];
    const int n_sl = (cd.tile_count + kSliceTiles - 1) / kSliceTiles;
    if (sl >= n_sl) return;  // uniform over the block
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const int q = tid & (kPart - 1);
    const int t_lo = sl * kSliceTiles;
    const int n_here = min(kSliceTiles, cd.tile_count - t_lo);
    const double* base = A.partials + static_cast<int64_t>(cd.tile_begin + t_lo) * kPart;
    Comp acc[2] = {Comp{0.0, 0.0}, Comp{0.0, 0.0}};
    {
        double v[kLoads];
#pragma unroll
        for (int j = 0; j < kLoads; ++j) {
            const int tile = tid / kPart + (NT / kPart) * j;
            v[j] = (q < kNQ && tile < n_here) ? base[tid + NT * j] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kLoads; ++j) comp_add(acc[j & 1], v[j]);
    }
    Comp r = comp_merge(acc[0], acc[1]);
    // lanes l, l ^ 16, l ^ 32, l ^ 48 of a wavefront hold the same quantity
#pragma unroll
    for (int off = kWave / 2; off >= kPart; off >>= 1) {
        Comp o;
        o.s = __shfl_xor(r.s, off, kWave);
        o.c = __shfl_xor(r.c, off, kWave);
        r = (tid & off) == 0 ? comp_merge(r, o) : comp_merge(o, r);
    }
    if (lane < kNQ) part[wv][lane] = r;
    __syncthreads();
    double* mine = A.slices + (static_cast<int64_t>(c) + cd.tile_begin / kSliceTiles + sl) * (2 * kNQ);
    if (tid < kNQ) {
        Comp m = part[0][tid];
#pragma unroll
        for (int w = 1; w < NT / kWave; ++w) m = comp_merge(m, part[w][tid]);
        mine[2 * tid] = m.s;
        mine[2 * tid + 1] = m.c;
    }
    // publish the slice, then count it; the block that counts the last slice
    // continues with the whole chain
    __threadfence();
    __syncthreads();
    if (tid == 0) last = atomicAdd(&A.arrive[c], 1u) == static_cast<uint32_t>(n_sl - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    ChainIn in;
    if (tid == 0) {
        A.arrive[c] = 0u;  // for the next launch
        in = load_chain_in(A, c);
    }
    const double* first = A.slices + (static_cast<int64_t>(c) + cd.tile_begin / kSliceTiles) * (2 * kNQ);
    if (tid < kWave) {
        // the first wavefront loads the slices kMergeChunk at a time (all of
        // a chunk's loads in flight together) into LDS, then lanes 0..kNQ-1
        // merge them in slice order
        const bool has_edge = tid < kNQ && cd.edge_tile >= 0;
        const double e = has_edge ? A.partials[static_cast<int64_t>(cd.edge_tile) * kPart + tid] : 0.0;
        Comp m{0.0, 0.0};
        for (int s0 = 0; s0 < n_sl; s0 += kMergeChunk) {
            const int ns = min(kMergeChunk, n_sl - s0);
            const double* src = first + static_cast<int64_t>(s0) * (2 * kNQ);
            double v[kMergeLoads];
#pragma unroll
            for (int j = 0; j < kMergeLoads; ++j) {
                const int i = tid + kWave * j;
                v[j] = i < ns * 2 * kNQ ? src[i] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < kMergeLoads; ++j) merge_buf[tid + kWave * j] = v[j];
            wave_sync_lds();
            if (tid < kNQ) {
                for (int s = 0; s < ns; ++s) {
                    const Comp x{merge_buf[s * 2 * kNQ + 2 * tid], merge_buf[s * 2 * kNQ + 2 * tid + 1]};
                    m = s0 + s == 0 ? x : comp_merge(m, x);
                }
            }
            wave_sync_lds();
        }
        if (has_edge) comp_add(m, e);
        if (tid < kNQ) part[0][tid] = m;
    }
    // the random numbers by the other wavefronts, while the first merges
    if (tid >= kWave) finalize_draws(A, c, cd.T, tid - kWave, NT - kWave, draws);
    __syncthreads();
    if (tid != 0) return;
    double tot[kNQ];
#pragma unroll
    for (int k = 0; k < kNQ; ++k) tot[k] = part[0][k].s + part[0][k].c;
    finalize_commit(A, c, cd.T, tot, in, draws);
}

// One chain per block of two wavefronts: the first loads and adds the tile
// partials while the second evaluates the chain's random numbers (the two
// are independent), then the first wavefront's lane 0 decides.
__global__ __launch_bounds__(2 * kWave) void k_finalize(FinalizeArgs A) {
    __shared__ Comp part[1][kNQ];
    __shared__ ThetaDraws draws;
    const int c = A.chain_first + static_cast<int>(blockIdx.x);
    if (threadIdx.x >= kWave) {
        finalize_draws(A, c, A.chains[c].T, threadIdx.x - kWave, kWave, draws);
        __syncthreads();  // meets the first wavefront's barrier before the decision
        return;
    }
    finalize_chain<kWave, false>(A, c, part, draws, threadIdx.x);
}

}  // namespace

}  // namespace rsv

#pragma clang diagnostic pop
