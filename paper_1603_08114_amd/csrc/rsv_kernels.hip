// rsv_kernels.hip -- HIP kernels (gfx950) of the RSV-model HMC update.
//
// Paper: T. Takaishi, arXiv:1603.08114.  The leapfrog of Sec. 3, eqs. (6)-(8)
// (mapped to per-site GPU kernels in Sec. 5, eqs. (9)-(11)) is fused here into
// one trajectory kernel that is blocked in time: each wavefront owns a tile
// of one chain, holds h, p and the per-site constants of its tile in
// registers (S contiguous sites per lane), exchanges the two boundary sites
// of each lane with its neighbours by DPP lane shifts, and runs all k steps
// without touching HBM.  Sites within k+1 of a tile's cut are recomputed by
// the neighbouring tile (halo), so every exact site is produced once.
#include "rsv_device.h"
#include "rsv_internal.h"

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
__device__ inline double exp_neg<double>(double x) { return exp(-x); }
template <>
__device__ inline float exp_neg<float>(float x) { return expf(-x); }

// ---------------------------------------------------------------------------
// Trajectory kernel: momentum refresh, k leapfrog steps, per-site dH terms and
// sufficient statistics of h' and h, all for one tile per wavefront.
// ---------------------------------------------------------------------------
template <typename R, int S, bool MASS, bool EDGE, bool RET>
__global__ __launch_bounds__(256) void k_traj(TrajArgs<R> A) {
    static_assert(S % 4 == 0, "lanes hold whole Philox blocks");
    const int lane = threadIdx.x & (kWave - 1);
    const int w = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (w >= A.n_list) return;  // uniform over the wavefront
    const int tile_id = A.tile_first + w;
    const TileDesc td = A.tiles[tile_id];
    const ChainDesc cd = A.chains[td.chain];
    const rsv_theta th = A.theta[td.chain];

    const int T = cd.T;
    const int t0 = td.la + lane * S;
    const bool rv = (A.terms & RSV_TERM_RV) != 0;
    const double phi = th.phi, mu = th.mu, xi = th.xi;
    const double inv_se = 1.0 / th.sig2_eta;
    const double inv_su = rv ? 1.0 / th.sig2_u : 0.0;
    const double dt = cd.dtau;
    // force g_t = c_t + alpha h_t - beta (h_{t-1} + h_{t+1}) - s_t e^{-h_t} / 2
    const double alpha = (1.0 + phi * phi) * inv_se + inv_su;
    const double beta = phi * inv_se;
    const double c_base = (RET ? 0.5 : 0.0) + xi * inv_su - mu * (1.0 - phi) * (1.0 - phi) * inv_se;
    const R mda = static_cast<R>(-dt * alpha);
    const R db = static_cast<R>(dt * beta);
    const R mu_r = static_cast<R>(mu), phi_r = static_cast<R>(phi);

    R h[S], p[S], dc[S], ds[S], dtm[MASS ? S : 1];
    double kin0 = 0.0;  // kinetic energy of the exact sites at the start

    const R* hc = A.h_cur + cd.h_off;
    const R* y2 = A.y2 + cd.d_off;
    const R* lr = A.lrv + cd.d_off;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int t = t0 + j;
        const bool live = t < T;
        h[j] = live ? hc[t] : R(0);
        const double yy = live ? static_cast<double>(y2[t]) : 0.0;
        const double rr = live ? static_cast<double>(lr[t]) : 0.0;
        dc[j] = static_cast<R>(-dt * (c_base - rr * inv_su));
        ds[j] = RET ? static_cast<R>(0.5 * dt * yy) : R(0);
    }

    // momentum refresh p ~ N(0, m): site t takes normal t%4 of block t/4
    const float* lm = MASS ? A.log_mass + cd.d_off : nullptr;
    if constexpr (MASS) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int t = t0 + j;
            const double l = (t < T) ? static_cast<double>(lm[t]) : 0.0;
            dtm[j] = static_cast<R>(dt * exp(-l));
        }
    }
    if (A.p0) {
        const double* p0 = A.p0 + cd.h_off;
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int t = t0 + j;
            p[j] = (t < T) ? static_cast<R>(p0[t]) : R(0);
        }
    } else {
#pragma unroll
        for (int g = 0; g < S / 4; ++g) {
            double u[4], z[4];
            uniforms4(A.seed, static_cast<uint64_t>((t0 >> 2) + g), A.sweep,
                      static_cast<uint64_t>(td.chain), kTagMomentum, u);
            gauss_pair(u[0], u[1], z[0], z[1]);
            gauss_pair(u[2], u[3], z[2], z[3]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = 4 * g + q;
                const int t = t0 + j;
                double pm = z[q];
                if constexpr (MASS) pm *= exp(0.5 * ((t < T) ? static_cast<double>(lm[t]) : 0.0));
                p[j] = (t < T) ? static_cast<R>(pm) : R(0);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int t = t0 + j;
        if (t >= td.a && t < td.b) {
            const double pj = static_cast<double>(p[j]);
            const double im = MASS ? exp(-static_cast<double>(lm[t])) : 1.0;
            kin0 += 0.5 * pj * pj * im;
        }
    }

    // ---- leapfrog, eqs. (6)-(8); adjacent h half steps of consecutive
    //      steps are merged into one full step ----
    const R dt_r = static_cast<R>(dt);
    const R half_r = static_cast<R>(0.5 * dt);
#pragma unroll
    for (int j = 0; j < S; ++j)
        h[j] += (MASS ? R(0.5) * dtm[MASS ? j : 0] : half_r) * p[j];

    const bool lane_first = (t0 == 0);
    const bool lane_last = (t0 + S == T);
    for (int step = 0; step < cd.n_steps; ++step) {
        R hl0 = from_lower(h[S - 1]);
        R hrS = from_upper(h[0]);
        if (lane_first) hl0 = ghost_neighbour(h[0], mu_r, phi_r);
        if (lane_last) hrS = ghost_neighbour(h[S - 1], mu_r, phi_r);
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const R hl = (j == 0) ? hl0 : h[j - 1];
            R hr = (j == S - 1) ? hrS : h[j + 1];
            if constexpr (EDGE) {
                if (j < S - 1 && t0 + j == T - 1) hr = ghost_neighbour(h[j], mu_r, phi_r);
            }
            R acc = p[j] + dc[j];
            acc += mda * h[j];
            acc += db * (hl + hr);
            if constexpr (RET) acc += ds[j] * exp_neg<R>(h[j]);
            p[j] = acc;
        }
        const bool last = (step + 1 == cd.n_steps);
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const R c = MASS ? (last ? R(0.5) * dtm[MASS ? j : 0] : dtm[MASS ? j : 0])
                             : (last ? half_r : dt_r);
            h[j] += c * p[j];
        }
    }

    // ---- dH = sum over exact sites of per-site differences (FP64), and the
    //      sufficient statistics of the proposal and of the current state ----
    const double* y2d = A.y2_d + cd.d_off;
    const double* lrd = A.lrv_d + cd.d_off;
    double h0d[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int t = t0 + j;
        h0d[j] = (t < T) ? static_cast<double>(hc[t]) : 0.0;
    }
    const double h1_up = static_cast<double>(from_upper(h[0]));
    const double h0_up = from_upper(h0d[0]);

    double dH = -kin0;
    double s1[5] = {0, 0, 0, 0, 0}, s0[5] = {0, 0, 0, 0, 0};
    double* edge = A.chain_edge + static_cast<int64_t>(td.chain) * kEdge;
    R* hp = A.h_prop + cd.h_off;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int t = t0 + j;
        if (t < td.a || t >= td.b) continue;
        const double h1 = static_cast<double>(h[j]);
        const double h0 = h0d[j];
        const double pj = static_cast<double>(p[j]);
        const double im = MASS ? exp(-static_cast<double>(lm[t])) : 1.0;
        const double rr = lrd[t];
        double d = 0.5 * pj * pj * im;
        if (RET) d += 0.5 * (h1 - h0) + 0.5 * y2d[t] * exp(-h0) * expm1(h0 - h1);
        if (rv) {
            const double c = rr - xi;
            const double e1 = c - h1, e0 = c - h0;
            d += (e1 - e0) * (e1 + e0) * (0.5 * inv_su);
        }
        const double a1 = h1 - mu, a0 = h0 - mu;
        if (t + 1 < T) {
            const double h1n = (j == S - 1) ? h1_up : static_cast<double>(h[j + 1]);
            const double h0n = (j == S - 1) ? h0_up : h0d[j + 1];
            const double d1 = (h1n - mu) - phi * a1;
            const double d0 = (h0n - mu) - phi * a0;
            d += (d1 - d0) * (d1 + d0) * (0.5 * inv_se);
            s1[2] += a1 * (h1n - mu);
            s0[2] += a0 * (h0n - mu);
        }
        if (t == 0) {
            d += (1.0 - phi * phi) * (a1 - a0) * (a1 + a0) * (0.5 * inv_se);
            edge[0] = a1;
            edge[2] = a0;
        }
        if (t == T - 1) {
            edge[1] = a1;
            edge[3] = a0;
        }
        dH += d;
        const double e1 = rr - h1 - xi, e0 = rr - h0 - xi;
        s1[0] += a1; s1[1] += a1 * a1; s1[3] += e1; s1[4] += e1 * e1;
        s0[0] += a0; s0[1] += a0 * a0; s0[3] += e0; s0[4] += e0 * e0;
        hp[t] = h[j];
    }

    dH = wave_sum(dH);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        s1[q] = wave_sum(s1[q]);
        s0[q] = wave_sum(s0[q]);
    }
    if (lane == 0) {
        double* out = A.partials + static_cast<int64_t>(tile_id) * kPart;
        out[kPartDH] = dH;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            out[kPartProp + q] = s1[q];
            out[kPartCur + q] = s0[q];
        }
    }
}

// ---------------------------------------------------------------------------
// Statistics of the current state over the exact range of each tile.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_stats(const TileDesc* tiles, int32_t n_tiles,
                                               const ChainDesc* chains, const rsv_theta* theta,
                                               const R* h, const double* lrv_d,
                                               double* partials, double* chain_edge) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (w >= n_tiles) return;
    const TileDesc td = tiles[w];
    const ChainDesc cd = chains[td.chain];
    const rsv_theta th = theta[td.chain];
    const R* hc = h + cd.h_off;
    const double* lr = lrv_d + cd.d_off;
    double s[5] = {0, 0, 0, 0, 0};
    for (int t = td.a + lane; t < td.b; t += kWave) {
        const double b = static_cast<double>(hc[t]) - th.mu;
        const double e = lr[t] - static_cast<double>(hc[t]) - th.xi;
        s[0] += b;
        s[1] += b * b;
        if (t + 1 < cd.T) s[2] += b * (static_cast<double>(hc[t + 1]) - th.mu);
        s[3] += e;
        s[4] += e * e;
        if (t == 0) chain_edge[static_cast<int64_t>(td.chain) * kEdge + 2] = b;
        if (t == cd.T - 1) chain_edge[static_cast<int64_t>(td.chain) * kEdge + 3] = b;
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) s[q] = wave_sum(s[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 5; ++q) partials[static_cast<int64_t>(w) * kPart + kPartCur + q] = s[q];
    }
}

// ---------------------------------------------------------------------------
// theta update (one lane per chain): Gibbs mu -> phi -> sigma_eta^2 -> xi ->
// sigma_u^2 from the sufficient statistics; random numbers from the theta
// stream: block 0 (z_mu, z_phi, u_phi), block 1 (z_xi), blocks 2.. and 34..
// the Gamma attempts of sigma_eta^2 and sigma_u^2.
// ---------------------------------------------------------------------------
constexpr int kGammaTries = 32;
constexpr uint64_t kGammaEtaBlock = 2, kGammaUBlock = 2 + kGammaTries;

struct ThetaStream {
    uint64_t seed, sweep, chain;
    __device__ void block(uint64_t idx, double u[4]) const {
        uniforms4(seed, idx, sweep, chain, kTagTheta, u);
    }
    // Gamma(shape, 1), shape >= 1, by Marsaglia-Tsang squeeze-free acceptance.
    __device__ double gamma(double shape, uint64_t first_block, bool& ran_out) const {
#pragma clang fp contract(off)
        const double d = shape - 1.0 / 3.0;
        const double c = 1.0 / sqrt(9.0 * d);
        for (int i = 0; i < kGammaTries; ++i) {
            double u[4], x, unused;
            block(first_block + static_cast<uint64_t>(i), u);
            gauss_pair(u[0], u[1], x, unused);
            double v = 1.0 + c * x;
            if (v <= 0.0) continue;
            v = v * v * v;
            if (log(u[2]) < 0.5 * x * x + d - d * v + d * log(v)) return d * v;
        }
        ran_out = true;
        return d;
    }
};

__device__ rsv_theta gibbs_theta(const double st[7], double n, rsv_theta cur,
                                 const rsv_prior& pr, int terms, const ThetaStream& rs,
                                 bool& ran_out) {
#pragma clang fp contract(off)
    const double B = st[0], B2 = st[1], BB = st[2], D1 = st[3], D2 = st[4];
    const double bf = st[5], bl = st[6];
    rsv_theta nxt = cur;

    double u0[4], z_mu, z_phi;
    rs.block(0, u0);
    gauss_pair(u0[0], u0[1], z_mu, z_phi);

    // mu: Gaussian; precision from the stationary start and T-1 transitions
    {
        const double one_m_phi = 1.0 - cur.phi;
        const double prec = 1.0 / pr.mu_var
                          + ((1.0 - cur.phi * cur.phi) + (n - 1.0) * one_m_phi * one_m_phi)
                                / cur.sig2_eta;
        const double lin = (pr.mu_mean - cur.mu) / pr.mu_var
                         + ((1.0 - cur.phi * cur.phi) * bf
                            + one_m_phi * ((B - bf) - cur.phi * (B - bl))) / cur.sig2_eta;
        nxt.mu = cur.mu + lin / prec + z_mu / sqrt(prec);
    }
    const double eps = nxt.mu - cur.mu;
    // a_t = b_t - eps;  Q(phi) = sum a^2 - 2 phi sum a_t a_{t+1} + phi^2 sum_{interior} a^2
    const double sum_aa = B2 - 2.0 * eps * B + n * eps * eps;
    const double lag = BB - eps * (2.0 * B - bf - bl) + (n - 1.0) * eps * eps;
    const double inner = (B2 - bf * bf - bl * bl) - 2.0 * eps * (B - bf - bl) + (n - 2.0) * eps * eps;
    // phi: independence proposal from the Gaussian factor, corrected by sqrt(1-phi^2)
    {
        const double cand = lag / inner + z_phi * sqrt(cur.sig2_eta / inner);
        if (fabs(cand) < 1.0) {
            const double ratio = (1.0 - cand * cand) / (1.0 - cur.phi * cur.phi);
            if (u0[2] * u0[2] < ratio) nxt.phi = cand;
        }
    }
    {
        const double q = sum_aa - 2.0 * nxt.phi * lag + nxt.phi * nxt.phi * inner;
        const double g = rs.gamma(pr.eta_shape + 0.5 * n, kGammaEtaBlock, ran_out);
        nxt.sig2_eta = (pr.eta_scale + 0.5 * q) / g;
    }
    if (terms & RSV_TERM_RV) {
        double u1[4], z_xi, unused;
        rs.block(1, u1);
        gauss_pair(u1[0], u1[1], z_xi, unused);
        const double prec = 1.0 / pr.xi_var + n / cur.sig2_u;
        const double lin = (pr.xi_mean - cur.xi) / pr.xi_var + D1 / cur.sig2_u;
        nxt.xi = cur.xi + lin / prec + z_xi / sqrt(prec);
        const double f = nxt.xi - cur.xi;
        const double ss = D2 - 2.0 * f * D1 + n * f * f;
        const double g = rs.gamma(pr.u_shape + 0.5 * n, kGammaUBlock, ran_out);
        nxt.sig2_u = (pr.u_scale + 0.5 * ss) / g;
    }
    return nxt;
}

// ---------------------------------------------------------------------------
// Per-chain finalize: reduce tile partials (compensated, fixed order), the
// Metropolis test, the choice of statistics, and the theta update.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_finalize(FinalizeArgs A) {
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    const ChainDesc cd = A.chains[c];
    constexpr int NQ = 11;
    Comp acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = Comp{0.0, 0.0};
    for (int i = lane; i < cd.tile_count; i += kWave) {
        const double* pp = A.partials + static_cast<int64_t>(cd.tile_begin + i) * kPart;
#pragma unroll
        for (int q = 0; q < NQ; ++q) comp_add(acc[q], pp[q]);
    }
    if (lane == 0 && cd.edge_tile >= 0) {
        const double* pp = A.partials + static_cast<int64_t>(cd.edge_tile) * kPart;
#pragma unroll
        for (int q = 0; q < NQ; ++q) comp_add(acc[q], pp[q]);
    }
    double tot[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const Comp r = wave_comp_sum(acc[q]);
        tot[q] = r.s + r.c;
    }
    if (lane != 0) return;

    const rsv_theta th = A.theta[c];
    bool use_prop = false;
    if (A.do_metropolis) {
#pragma clang fp contract(off)
        const double dH = tot[kPartDH];
        double lu;
        if (A.log_u) {
            lu = A.log_u[c];
        } else {
            double u[4];
            uniforms4(A.seed, 0, A.sweep, static_cast<uint64_t>(c), kTagAccept, u);
            lu = log(u[0]);
        }
        const bool finite = isfinite(dH);
        const bool accept = finite && (lu < -dH);
        if (!finite) atomicAdd(&A.counters[kCntNonfiniteDH], 1u);
        use_prop = accept;
        A.accept_ws[c] = accept ? 1 : 0;
        if (A.delta_h_out) A.delta_h_out[c] = dH;
        if (A.accepted_out) A.accepted_out[c] = accept ? 1 : 0;
    }
    const int base = use_prop ? kPartProp : kPartCur;
    const double* edge = A.chain_edge + static_cast<int64_t>(c) * kEdge;
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
    if (A.do_theta) {
        bool ran_out = false;
        const ThetaStream rs{A.seed, A.sweep, static_cast<uint64_t>(c)};
        out = gibbs_theta(st, static_cast<double>(cd.T), th, A.prior, A.terms, rs, ran_out);
        if (ran_out) atomicAdd(&A.counters[kCntGammaExhausted], 1u);
        A.theta[c] = out;
    }
    if (A.theta_trace) A.theta_trace[c] = out;
}

// ---------------------------------------------------------------------------
// Commit accepted proposals into the state (and copy h to a trace).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_commit(const ChainDesc* chains, const int32_t* acc,
                                                const R* h_prop, R* h_cur, R* h_trace) {
    const int c = blockIdx.y;
    const ChainDesc cd = chains[c];
    const bool take = acc[c] != 0;
    if (!take && !h_trace) return;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < cd.T;
         t += stride) {
        const int64_t i = cd.h_off + t;
        const R v = take ? h_prop[i] : h_cur[i];
        if (take) h_cur[i] = v;
        if (h_trace) h_trace[i] = v;
    }
}

// ---------------------------------------------------------------------------
// Standalone momentum refresh (same streams as the trajectory kernel).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_momenta(const ChainDesc* chains, const float* log_mass,
                                                 uint64_t seed, uint64_t sweep, double* p_out) {
    const int c = blockIdx.y;
    const ChainDesc cd = chains[c];
    const int n_blocks = (cd.T + 3) / 4;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n_blocks;
         g += gridDim.x * blockDim.x) {
        double u[4], z[4];
        uniforms4(seed, static_cast<uint64_t>(g), sweep, static_cast<uint64_t>(c), kTagMomentum, u);
        gauss_pair(u[0], u[1], z[0], z[1]);
        gauss_pair(u[2], u[3], z[2], z[3]);
        for (int q = 0; q < 4; ++q) {
            const int t = 4 * g + q;
            if (t >= cd.T) break;
            const double sm = log_mass ? exp(0.5 * static_cast<double>(log_mass[cd.d_off + t])) : 1.0;
            p_out[cd.h_off + t] = z[q] * sm;
        }
    }
}

// ---------------------------------------------------------------------------
// Data preparation and validation.
// ---------------------------------------------------------------------------
__global__ void k_prepare(const double* y, const double* lrv, int64_t n, double* y2_d,
                          float* y2_f, float* lrv_f) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double yy = y[i] * y[i];
        y2_d[i] = yy;
        if (y2_f) y2_f[i] = static_cast<float>(yy);
        if (lrv_f) lrv_f[i] = static_cast<float>(lrv[i]);
    }
}

template <typename R>
__global__ void k_count_nonfinite(const R* x, int64_t n, uint32_t* counter) {
    uint32_t bad = 0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        bad += isfinite(static_cast<double>(x[i])) ? 0u : 1u;
    if (bad) atomicAdd(counter, bad);
}

inline int grid_for(int64_t n, int block, int cap) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return static_cast<int>(g > cap ? cap : g);
}

template <typename R, int S>
hipError_t launch_traj_t(hipStream_t st, bool mass, bool edge, bool ret, const TrajArgs<R>& a) {
    if (a.n_list <= 0) return hipSuccess;
    const dim3 grid((a.n_list + 3) / 4), block(256);
#define RSV_TRAJ(M, E, RT) hipLaunchKernelGGL((k_traj<R, S, M, E, RT>), grid, block, 0, st, a)
    if (ret) {
        if (mass) { if (edge) RSV_TRAJ(true, true, true); else RSV_TRAJ(true, false, true); }
        else      { if (edge) RSV_TRAJ(false, true, true); else RSV_TRAJ(false, false, true); }
    } else {
        if (mass) { if (edge) RSV_TRAJ(true, true, false); else RSV_TRAJ(true, false, false); }
        else      { if (edge) RSV_TRAJ(false, true, false); else RSV_TRAJ(false, false, false); }
    }
#undef RSV_TRAJ
    return hipGetLastError();
}

}  // namespace

// Sites per lane of the trajectory kernel: the compiled choices per
// precision, the first being the default.
int traj_sites_per_lane(int precision, int requested) {
    if (precision == RSV_F64) {
        if (requested == 0) return 8;
        return (requested == 8 || requested == 16) ? requested : -1;
    }
    if (requested == 0) return 16;
    return (requested == 16 || requested == 32) ? requested : -1;
}

hipError_t launch_traj(hipStream_t st, int precision, int S, bool mass, bool edge,
                       const void* args) {
    if (precision == RSV_F64) {
        const auto& a = *static_cast<const TrajArgs<double>*>(args);
        const bool ret = (a.terms & RSV_TERM_RETURN) != 0;
        if (S == 8) return launch_traj_t<double, 8>(st, mass, edge, ret, a);
        if (S == 16) return launch_traj_t<double, 16>(st, mass, edge, ret, a);
    } else {
        const auto& a = *static_cast<const TrajArgs<float>*>(args);
        const bool ret = (a.terms & RSV_TERM_RETURN) != 0;
        if (S == 16) return launch_traj_t<float, 16>(st, mass, edge, ret, a);
        if (S == 32) return launch_traj_t<float, 32>(st, mass, edge, ret, a);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_prepare(hipStream_t st, const double* y, const double* lrv, int64_t n,
                          double* y2_d, float* y2_f, float* lrv_f) {
    hipLaunchKernelGGL(k_prepare, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, y, lrv, n,
                       y2_d, y2_f, lrv_f);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(hipStream_t st, const void* h, int64_t n, int precision,
                                  uint32_t* counter) {
    const dim3 g(grid_for(n, 256, 4096)), b(256);
    if (precision == RSV_F64)
        hipLaunchKernelGGL(k_count_nonfinite<double>, g, b, 0, st, static_cast<const double*>(h),
                           n, counter);
    else
        hipLaunchKernelGGL(k_count_nonfinite<float>, g, b, 0, st, static_cast<const float*>(h), n,
                           counter);
    return hipGetLastError();
}

hipError_t launch_validate(hipStream_t st, const double* y, const double* lrv, int64_t n_data,
                           const void* h, int64_t n_state, int precision, uint32_t* counters) {
    const dim3 g(grid_for(n_data, 256, 4096)), b(256);
    hipLaunchKernelGGL(k_count_nonfinite<double>, g, b, 0, st, y, n_data,
                       counters + kCntNonfiniteData);
    hipLaunchKernelGGL(k_count_nonfinite<double>, g, b, 0, st, lrv, n_data,
                       counters + kCntNonfiniteData);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_count_nonfinite(st, h, n_state, precision, counters + kCntNonfiniteState);
}

hipError_t launch_finalize(hipStream_t st, const FinalizeArgs& a) {
    hipLaunchKernelGGL(k_finalize, dim3(a.n_chains), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_commit(hipStream_t st, const ChainDesc* chains, int32_t n_chains, int32_t max_T,
                         const int32_t* accept_ws, const void* h_prop, void* h_cur,
                         void* h_trace, int precision) {
    const dim3 g(grid_for(max_T, 256, 1024), n_chains), b(256);
    if (precision == RSV_F64)
        hipLaunchKernelGGL(k_commit<double>, g, b, 0, st, chains, accept_ws,
                           static_cast<const double*>(h_prop), static_cast<double*>(h_cur),
                           static_cast<double*>(h_trace));
    else
        hipLaunchKernelGGL(k_commit<float>, g, b, 0, st, chains, accept_ws,
                           static_cast<const float*>(h_prop), static_cast<float*>(h_cur),
                           static_cast<float*>(h_trace));
    return hipGetLastError();
}

hipError_t launch_stats(hipStream_t st, const TileDesc* tiles, int32_t n_tiles,
                        const ChainDesc* chains, const rsv_theta* theta, const void* h_cur,
                        const double* lrv_d, double* partials, double* chain_edge,
                        int precision) {
    const dim3 g((n_tiles + 3) / 4), b(256);
    if (precision == RSV_F64)
        hipLaunchKernelGGL(k_stats<double>, g, b, 0, st, tiles, n_tiles, chains, theta,
                           static_cast<const double*>(h_cur), lrv_d, partials, chain_edge);
    else
        hipLaunchKernelGGL(k_stats<float>, g, b, 0, st, tiles, n_tiles, chains, theta,
                           static_cast<const float*>(h_cur), lrv_d, partials, chain_edge);
    return hipGetLastError();
}

hipError_t launch_momenta(hipStream_t st, const ChainDesc* chains, int32_t n_chains,
                          int32_t max_T, const float* log_mass, uint64_t seed, uint64_t sweep,
                          double* p_out) {
    const dim3 g(grid_for((max_T + 3) / 4, 256, 1024), n_chains), b(256);
    hipLaunchKernelGGL(k_momenta, g, b, 0, st, chains, log_mass, seed, sweep, p_out);
    return hipGetLastError();
}

}  // namespace rsv
