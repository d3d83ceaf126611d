/*
 * rsv_oracle.c -- plain, serial, FP64 CPU oracle of the RSV-model HMC
 * volatility update and theta update.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  It shares no
 * code with the HIP library.  Built with -O2 -ffp-contract=off so that the
 * arithmetic is exactly what is written.
 *
 * Follows T. Takaishi, arXiv:1603.08114:
 *   Sec. 2, eqs. (1)-(3)  model                 -> orc_energy, orc_grad
 *   Sec. 3                H = 1/2 sum p^2 - ln f -> orc_hamiltonian
 *   Sec. 3, eqs. (6)-(8)  leapfrog, k steps     -> orc_leapfrog
 *   Sec. 3 (end)          Metropolis, dH        -> orc_delta_h, orc_trajectory
 * The paper leaves ln f, the law of h_1, the momentum law, the priors and
 * the theta sampler unstated; the readings taken here are listed in the
 * header comments of each function and in the design notes.
 */
#include "rsv_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128  */
/* multiplications, Weyl key schedule between rounds.                  */
/* ------------------------------------------------------------------ */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL;
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL;

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        unsigned __int128 prod0 = (unsigned __int128)PHILOX_M0 * x0;
        unsigned __int128 prod1 = (unsigned __int128)PHILOX_M1 * x2;
        uint64_t hi0 = (uint64_t)(prod0 >> 64), lo0 = (uint64_t)prod0;
        uint64_t hi1 = (uint64_t)(prod1 >> 64), lo1 = (uint64_t)prod1;
        uint64_t n0 = hi1 ^ x1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ x3 ^ k1;
        uint64_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Top 52 bits, centred in their cell: exactly representable, in (0,1). */
static double u01_from_bits(uint64_t x)
{
    return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

void orc_uniforms4(uint64_t seed, uint64_t idx, uint64_t sweep, uint64_t chain,
                   uint64_t tag, double u[4])
{
    uint64_t ctr[4] = { idx, sweep, chain, tag };
    uint64_t key[2] = { seed, 0 };
    uint64_t bits[4];
    orc_philox4x64_10(ctr, key, bits);
    for (int i = 0; i < 4; ++i) u[i] = u01_from_bits(bits[i]);
}

/* Box-Muller: (u0,u1) -> sqrt(-2 ln u0) * (cos 2 pi u1, sin 2 pi u1). */
static void box_muller(double u0, double u1, double *z0, double *z1)
{
    double radius = sqrt(-2.0 * log(u0));
    double angle = 6.283185307179586 * u1;
    *z0 = radius * cos(angle);
    *z1 = radius * sin(angle);
}

static void normals4(uint64_t seed, uint64_t idx, uint64_t sweep, uint64_t chain,
                     uint64_t tag, double z[4])
{
    double u[4];
    orc_uniforms4(seed, idx, sweep, chain, tag, u);
    box_muller(u[0], u[1], &z[0], &z[1]);
    box_muller(u[2], u[3], &z[2], &z[3]);
}

void orc_uniform_stream(uint64_t seed, uint64_t sweep, uint64_t chain, uint64_t tag,
                        int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double u[4];
        orc_uniforms4(seed, (uint64_t)(i / 4), sweep, chain, tag, u);
        out[i] = u[i % 4];
    }
}

void orc_normal_stream(uint64_t seed, uint64_t sweep, uint64_t chain, uint64_t tag,
                       int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double z[4];
        normals4(seed, (uint64_t)(i / 4), sweep, chain, tag, z);
        out[i] = z[i % 4];
    }
}

/* ------------------------------------------------------------------ */
/* Compensated summation (Neumaier's variant of Kahan).                */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}

static double nsum_value(const nsum *a) { return a->s + a->c; }

double orc_neumaier_sum(int64_t n, const double *x)
{
    nsum acc = { 0.0, 0.0 };
    for (int64_t i = 0; i < n; ++i) nsum_add(&acc, x[i]);
    return nsum_value(&acc);
}

/* ------------------------------------------------------------------ */
/* Target.  With a_t = h_t - mu and the model of eqs. (1)-(3):         */
/*   y_t | h_t      ~ N(0, exp(h_t))               eq. (1)             */
/*   ln RV_t | h_t  ~ N(xi + h_t, sigma_u^2)       eq. (2)             */
/*   a_{t+1} | a_t  ~ N(phi a_t, sigma_eta^2)      eq. (3)             */
/*   a_1            ~ N(0, sigma_eta^2/(1-phi^2))  (reading: stationary)*/
/* U(h) = -ln f(h | theta, data) up to a constant in h.                */
/* ------------------------------------------------------------------ */
double orc_energy(int64_t T, const double *h, const double *y2, const double *r,
                  const orc_theta *th, int terms)
{
    nsum acc = { 0.0, 0.0 };
    for (int64_t t = 0; t < T; ++t) {
        if (terms & ORC_TERM_RETURN)
            nsum_add(&acc, 0.5 * h[t] + 0.5 * y2[t] * exp(-h[t]));
        if (terms & ORC_TERM_RV) {
            double resid = r[t] - th->xi - h[t];
            nsum_add(&acc, resid * resid / (2.0 * th->sig2_u));
        }
    }
    double a0 = h[0] - th->mu;
    nsum_add(&acc, (1.0 - th->phi * th->phi) * a0 * a0 / (2.0 * th->sig2_eta));
    for (int64_t t = 0; t + 1 < T; ++t) {
        double innov = (h[t + 1] - th->mu) - th->phi * (h[t] - th->mu);
        nsum_add(&acc, innov * innov / (2.0 * th->sig2_eta));
    }
    return nsum_value(&acc);
}

/* dU/dh_t, term by term: each squared residual of U contributes its
 * derivative to the sites it contains. */
void orc_grad(int64_t T, const double *h, const double *y2, const double *r,
              const orc_theta *th, int terms, double *g)
{
    for (int64_t t = 0; t < T; ++t) {
        double gt = 0.0;
        if (terms & ORC_TERM_RETURN) gt += 0.5 - 0.5 * y2[t] * exp(-h[t]);
        if (terms & ORC_TERM_RV) gt -= (r[t] - th->xi - h[t]) / th->sig2_u;
        g[t] = gt;
    }
    double a0 = h[0] - th->mu;
    g[0] += (1.0 - th->phi * th->phi) * a0 / th->sig2_eta;
    for (int64_t t = 0; t + 1 < T; ++t) {
        double innov = (h[t + 1] - th->mu) - th->phi * (h[t] - th->mu);
        g[t + 1] += innov / th->sig2_eta;
        g[t] -= th->phi * innov / th->sig2_eta;
    }
}

double orc_hamiltonian(int64_t T, const double *h, const double *p, const double *log_m,
                       const double *y2, const double *r, const orc_theta *th, int terms)
{
    nsum acc = { 0.0, 0.0 };
    for (int64_t t = 0; t < T; ++t) {
        double inv_m = log_m ? exp(-log_m[t]) : 1.0;
        nsum_add(&acc, 0.5 * p[t] * p[t] * inv_m);
    }
    nsum_add(&acc, orc_energy(T, h, y2, r, th, terms));
    return nsum_value(&acc);
}

/* Eqs. (6)-(8), repeated k times: half step of h with the current p,
 * full step of p with the force at the half-stepped h, half step of h. */
void orc_leapfrog(int64_t T, double *h, double *p, const double *log_m,
                  const double *y2, const double *r, const orc_theta *th, int terms,
                  int32_t k, double dtau)
{
    double *g = (double *)malloc((size_t)T * sizeof(double));
    double *inv_m = (double *)malloc((size_t)T * sizeof(double));
    for (int64_t t = 0; t < T; ++t) inv_m[t] = log_m ? exp(-log_m[t]) : 1.0;
    for (int32_t step = 0; step < k; ++step) {
        for (int64_t t = 0; t < T; ++t) h[t] = h[t] + 0.5 * dtau * p[t] * inv_m[t];
        orc_grad(T, h, y2, r, th, terms, g);
        for (int64_t t = 0; t < T; ++t) p[t] = p[t] - dtau * g[t];
        for (int64_t t = 0; t < T; ++t) h[t] = h[t] + 0.5 * dtau * p[t] * inv_m[t];
    }
    free(inv_m);
    free(g);
}

/* Omelyan's second-order minimum-norm integrator (Omelyan, Mryglod and
 * Folk, Comput. Phys. Commun. 151 (2003) 272; its h-first form is the one
 * Takaishi and de Forcrand tested for HMC, Phys. Rev. E 73 (2006) 036706),
 * a higher-order alternative to the leapfrog that Sec. 3 says may be used.
 * Each of the k steps: h by lambda dtau, p by dtau/2, h by (1 - 2 lambda)
 * dtau, p by dtau/2, h by lambda dtau, with the momentum steps taking the
 * force at the current h.  Two force evaluations per step. */
void orc_omelyan(int64_t T, double *h, double *p, const double *log_m,
                 const double *y2, const double *r, const orc_theta *th, int terms,
                 int32_t k, double dtau)
{
    const double lambda = ORC_OMELYAN_LAMBDA;
    double *g = (double *)malloc((size_t)T * sizeof(double));
    double *inv_m = (double *)malloc((size_t)T * sizeof(double));
    for (int64_t t = 0; t < T; ++t) inv_m[t] = log_m ? exp(-log_m[t]) : 1.0;
    for (int32_t step = 0; step < k; ++step) {
        for (int64_t t = 0; t < T; ++t) h[t] = h[t] + lambda * dtau * p[t] * inv_m[t];
        orc_grad(T, h, y2, r, th, terms, g);
        for (int64_t t = 0; t < T; ++t) p[t] = p[t] - 0.5 * dtau * g[t];
        for (int64_t t = 0; t < T; ++t)
            h[t] = h[t] + (1.0 - 2.0 * lambda) * dtau * p[t] * inv_m[t];
        orc_grad(T, h, y2, r, th, terms, g);
        for (int64_t t = 0; t < T; ++t) p[t] = p[t] - 0.5 * dtau * g[t];
        for (int64_t t = 0; t < T; ++t) h[t] = h[t] + lambda * dtau * p[t] * inv_m[t];
    }
    free(inv_m);
    free(g);
}

/* Forest and Ruth's fourth-order scheme (Physica D 43 (1990) 105), the
 * h-first composition of three leapfrogs of sizes theta, 1 - 2 theta, theta
 * with theta = 1 / (2 - 2^(1/3)): each of the k steps moves h by
 * theta/2 dtau, p by theta dtau, h by (1 - theta)/2 dtau, p by
 * (1 - 2 theta) dtau, h by (1 - theta)/2 dtau, p by theta dtau, h by
 * theta/2 dtau.  Three force evaluations per step. */
void orc_forest_ruth(int64_t T, double *h, double *p, const double *log_m,
                     const double *y2, const double *r, const orc_theta *th, int terms,
                     int32_t k, double dtau)
{
    const double theta = ORC_FOREST_RUTH_THETA;
    const double drift[4] = { 0.5 * theta, 0.5 * (1.0 - theta), 0.5 * (1.0 - theta),
                              0.5 * theta };
    const double kick[3] = { theta, 1.0 - 2.0 * theta, theta };
    double *g = (double *)malloc((size_t)T * sizeof(double));
    double *inv_m = (double *)malloc((size_t)T * sizeof(double));
    for (int64_t t = 0; t < T; ++t) inv_m[t] = log_m ? exp(-log_m[t]) : 1.0;
    for (int32_t step = 0; step < k; ++step) {
        for (int s = 0; s < 3; ++s) {
            for (int64_t t = 0; t < T; ++t) h[t] = h[t] + drift[s] * dtau * p[t] * inv_m[t];
            orc_grad(T, h, y2, r, th, terms, g);
            for (int64_t t = 0; t < T; ++t) p[t] = p[t] - kick[s] * dtau * g[t];
        }
        for (int64_t t = 0; t < T; ++t) h[t] = h[t] + drift[3] * dtau * p[t] * inv_m[t];
    }
    free(inv_m);
    free(g);
}

void orc_integrate(int64_t T, double *h, double *p, const double *log_m,
                   const double *y2, const double *r, const orc_theta *th, int terms,
                   int32_t k, double dtau, int integrator)
{
    if (integrator == ORC_INT_OMELYAN)
        orc_omelyan(T, h, p, log_m, y2, r, th, terms, k, dtau);
    else if (integrator == ORC_INT_FOREST_RUTH)
        orc_forest_ruth(T, h, p, log_m, y2, r, th, terms, k, dtau);
    else
        orc_leapfrog(T, h, p, log_m, y2, r, th, terms, k, dtau);
}

/* dH as a sum of per-site changes, each formed from differences so that
 * nothing of the size of H itself is ever subtracted:
 *   x'^2 - x^2 = (x'-x)(x'+x);  e^{-h'} - e^{-h} = e^{-h} expm1(-(h'-h)). */
double orc_delta_h(int64_t T, const double *h0, const double *p0,
                   const double *h1, const double *p1, const double *log_m,
                   const double *y2, const double *r, const orc_theta *th, int terms)
{
    nsum acc = { 0.0, 0.0 };
    const double phi = th->phi, mu = th->mu;
    for (int64_t t = 0; t < T; ++t) {
        double inv_m = log_m ? exp(-log_m[t]) : 1.0;
        double dt = 0.5 * (p1[t] - p0[t]) * (p1[t] + p0[t]) * inv_m;
        if (terms & ORC_TERM_RETURN)
            dt += 0.5 * (h1[t] - h0[t]) + 0.5 * y2[t] * exp(-h0[t]) * expm1(-(h1[t] - h0[t]));
        if (terms & ORC_TERM_RV) {
            double c = r[t] - th->xi;
            double e1 = c - h1[t], e0 = c - h0[t];
            dt += (e1 - e0) * (e1 + e0) / (2.0 * th->sig2_u);
        }
        if (t + 1 < T) {
            double d1 = (h1[t + 1] - mu) - phi * (h1[t] - mu);
            double d0 = (h0[t + 1] - mu) - phi * (h0[t] - mu);
            dt += (d1 - d0) * (d1 + d0) / (2.0 * th->sig2_eta);
        }
        if (t == 0) {
            double a1 = h1[0] - mu, a0 = h0[0] - mu;
            dt += (1.0 - phi * phi) * (a1 - a0) * (a1 + a0) / (2.0 * th->sig2_eta);
        }
        nsum_add(&acc, dt);
    }
    return nsum_value(&acc);
}

/* Momentum refresh (reading: the Gibbs draw implied by the kinetic term):
 * site t takes normal t%4 of Philox block t/4 of the momentum stream. */
void orc_momenta(uint64_t seed, uint64_t sweep, uint64_t chain, int64_t T,
                 const double *log_m, double *p)
{
    for (int64_t t = 0; t < T; ++t) {
        double z[4];
        normals4(seed, (uint64_t)(t / 4), sweep, chain, ORC_TAG_MOMENTUM, z);
        p[t] = z[t % 4] * (log_m ? exp(0.5 * log_m[t]) : 1.0);
    }
}

/* Momentum refresh of the FP32-mixed path (the library's own stream layout
 * for that precision): site t takes normal t%8 of Philox block t/8 of the
 * momentum stream; word q of the block gives sites 2q and 2q+1 of the block
 * by Box-Muller on u0 = (top 40 bits + 1/2) 2^-40 and u1 = (low 24 bits +
 * 1/2) 2^-24.  Computed here in FP64; the library forms it in FP32. */
void orc_momenta_f32(uint64_t seed, uint64_t sweep, uint64_t chain, int64_t T,
                     const double *log_m, double *p)
{
    for (int64_t t = 0; t < T; ++t) {
        uint64_t ctr[4] = { (uint64_t)(t / 8), sweep, chain, ORC_TAG_MOMENTUM };
        uint64_t key[2] = { seed, 0 };
        uint64_t w[4];
        orc_philox4x64_10(ctr, key, w);
        const int r = (int)(t % 8);
        const uint64_t word = w[r / 2];
        const double u0 = ((double)(word >> 24) + 0.5) * 0x1p-40;
        const double u1 = ((double)(word & 0xFFFFFFu) + 0.5) * 0x1p-24;
        double z0, z1;
        box_muller(u0, u1, &z0, &z1);
        p[t] = ((r & 1) ? z1 : z0) * (log_m ? exp(0.5 * log_m[t]) : 1.0);
    }
}

double orc_log_u(uint64_t seed, uint64_t sweep, uint64_t chain)
{
    double u[4];
    orc_uniforms4(seed, 0, sweep, chain, ORC_TAG_ACCEPT, u);
    return log(u[0]);
}

/* Step-size jitter (an extension of the fixed dtau of Sec. 2): the length
 * k * dtau of every trajectory is scaled by a factor uniform on [1-j, 1+j],
 * drawn independently of the state, which keeps the Markov chain exact and
 * breaks the near-periodic orbits of modes whose period divides k * dtau. */
double orc_step_size(uint64_t seed, uint64_t sweep, uint64_t chain, double dtau, double jitter)
{
    if (!(jitter > 0.0)) return dtau;
    double u[4];
    orc_uniforms4(seed, 0, sweep, chain, ORC_TAG_STEP, u);
    double w = 2.0 * u[0] - 1.0;
    double f = jitter * w;
    f = 1.0 + f;
    return dtau * f;
}

int orc_trajectory(int64_t T, double *h, const double *log_m,
                   const double *y2, const double *r, const orc_theta *th, int terms,
                   int32_t k, double dtau, int integrator, uint64_t seed, uint64_t sweep,
                   uint64_t chain, const double *p0, const double *log_u, double *p_out,
                   double *dH_out)
{
    size_t bytes = (size_t)T * sizeof(double);
    double *h_start = (double *)malloc(bytes);
    double *p_start = (double *)malloc(bytes);
    double *p = (double *)malloc(bytes);
    memcpy(h_start, h, bytes);
    if (p0) memcpy(p_start, p0, bytes);
    else orc_momenta(seed, sweep, chain, T, log_m, p_start);
    memcpy(p, p_start, bytes);
    if (p_out) memcpy(p_out, p_start, bytes);

    orc_integrate(T, h, p, log_m, y2, r, th, terms, k, dtau, integrator);
    double dH = orc_delta_h(T, h_start, p_start, h, p, log_m, y2, r, th, terms);
    double lu = log_u ? *log_u : orc_log_u(seed, sweep, chain);
    /* accept with probability min{1, exp(-dH)}: u < exp(-dH); ties and
     * non-finite dH reject. */
    int accept = isfinite(dH) && (lu < -dH);
    if (!accept) memcpy(h, h_start, bytes);
    if (dH_out) *dH_out = dH;
    free(p);
    free(p_start);
    free(h_start);
    return accept;
}

/* ------------------------------------------------------------------ */
/* Sufficient statistics of h for the theta update (shifted sums).     */
/* ------------------------------------------------------------------ */
void orc_suffstats(int64_t T, const double *h, const double *r, double c_mu, double c_xi,
                   double out[7])
{
    nsum sb = { 0, 0 }, sbb = { 0, 0 }, slag = { 0, 0 }, se = { 0, 0 }, see = { 0, 0 };
    for (int64_t t = 0; t < T; ++t) {
        double b = h[t] - c_mu;
        double e = r[t] - h[t] - c_xi;
        nsum_add(&sb, b);
        nsum_add(&sbb, b * b);
        if (t + 1 < T) nsum_add(&slag, b * (h[t + 1] - c_mu));
        nsum_add(&se, e);
        nsum_add(&see, e * e);
    }
    out[0] = nsum_value(&sb);
    out[1] = nsum_value(&sbb);
    out[2] = nsum_value(&slag);
    out[3] = nsum_value(&se);
    out[4] = nsum_value(&see);
    out[5] = h[0] - c_mu;
    out[6] = h[T - 1] - c_mu;
}

/* ------------------------------------------------------------------ */
/* Theta update (the paper gives none; reading): Gibbs over            */
/* mu | phi,s_eta  ->  phi | mu,s_eta (independence Metropolis)        */
/*  -> s_eta | phi,mu  ->  xi | s_u  ->  s_u | xi,                     */
/* all conditional on the current h through its statistics.            */
/* Stream (tag 2) layout: block 0 -> (z_mu, z_phi, u_phi), block 1 ->  */
/* z_xi, blocks 2..33 -> Gamma attempts of s_eta, 34..65 -> s_u.       */
/* ------------------------------------------------------------------ */
enum { GAMMA_ATTEMPTS = 32, IDX_GAMMA_ETA = 2, IDX_GAMMA_U = 2 + GAMMA_ATTEMPTS };

double orc_gamma(double alpha, uint64_t seed, uint64_t sweep, uint64_t chain, uint64_t tag,
                 uint64_t idx0, int *exhausted)
{
    /* Marsaglia & Tsang (2000), alpha >= 1. */
    double d = alpha - 1.0 / 3.0;
    double c = 1.0 / sqrt(9.0 * d);
    for (int attempt = 0; attempt < GAMMA_ATTEMPTS; ++attempt) {
        double u[4], x, unused;
        orc_uniforms4(seed, idx0 + (uint64_t)attempt, sweep, chain, tag, u);
        box_muller(u[0], u[1], &x, &unused);
        double v = 1.0 + c * x;
        if (v <= 0.0) continue;
        v = v * v * v;
        if (log(u[2]) < 0.5 * x * x + d - d * v + d * log(v)) return d * v;
    }
    if (exhausted) *exhausted = 1;
    return d;
}

/* mu | phi, sigma_eta^2, h: Gaussian.  With b_t = h_t - c_mu and
 * mu = c_mu + eps, the AR(1) part of U is
 *   [(1-phi^2)(b_1-eps)^2 + sum_{t=1}^{T-1} (b_{t+1} - phi b_t - (1-phi) eps)^2] / (2 s_eta). */
double orc_draw_mu(int64_t T, const double st[7], const orc_theta *th, const orc_prior *pr,
                   double z)
{
    double phi = th->phi, s_eta = th->sig2_eta, c_mu = th->mu;
    double B = st[0], b_first = st[5], b_last = st[6];
    double prec = 1.0 / pr->mu_var
                + ((1.0 - phi * phi) + (double)(T - 1) * (1.0 - phi) * (1.0 - phi)) / s_eta;
    double lin = (pr->mu_mean - c_mu) / pr->mu_var
               + ((1.0 - phi * phi) * b_first
                  + (1.0 - phi) * ((B - b_first) - phi * (B - b_last))) / s_eta;
    return c_mu + lin / prec + z / sqrt(prec);
}

/* xi | sigma_u^2, h: Gaussian; e_t = r_t - h_t - c_xi, xi = c_xi + f. */
double orc_draw_xi(int64_t T, const double st[7], const orc_theta *th, const orc_prior *pr,
                   double z)
{
    double s_u = th->sig2_u, c_xi = th->xi;
    double prec = 1.0 / pr->xi_var + (double)T / s_u;
    double lin = (pr->xi_mean - c_xi) / pr->xi_var + st[3] / s_u;
    return c_xi + lin / prec + z / sqrt(prec);
}

int orc_theta_update(int64_t T, const double st[7], const orc_theta *th_in,
                     const orc_prior *pr, int terms, uint64_t seed, uint64_t sweep,
                     uint64_t chain, orc_theta *th_out)
{
    const uint64_t tag = ORC_TAG_THETA;
    int flags = 0, exhausted = 0;
    double B = st[0], B2 = st[1], BB = st[2], D1 = st[3], D2 = st[4];
    double b_first = st[5], b_last = st[6];
    double n = (double)T;
    orc_theta th = *th_in;

    double u0[4], z_mu, z_phi;
    orc_uniforms4(seed, 0, sweep, chain, tag, u0);
    box_muller(u0[0], u0[1], &z_mu, &z_phi);

    /* mu */
    th.mu = orc_draw_mu(T, st, th_in, pr, z_mu);
    double eps = th.mu - th_in->mu;

    /* phi: with a_t = b_t - eps the AR(1) part is Q(phi)/(2 s_eta),
     *   Q(phi) = SA - 2 phi C + phi^2 D,  SA = sum_{t=1}^T a_t^2,
     *   C = sum_{t=1}^{T-1} a_t a_{t+1},  D = sum_{t=2}^{T-1} a_t^2,
     * and the stationary law of a_1 adds a factor sqrt(1-phi^2).
     * Propose from N(C/D, s_eta/D); accept with sqrt((1-phi*^2)/(1-phi^2)). */
    double SA = B2 - 2.0 * eps * B + n * eps * eps;
    double C = BB - eps * (2.0 * B - b_first - b_last) + (n - 1.0) * eps * eps;
    double D = (B2 - b_first * b_first - b_last * b_last)
             - 2.0 * eps * (B - b_first - b_last) + (n - 2.0) * eps * eps;
    double phi_prop = C / D + z_phi * sqrt(th.sig2_eta / D);
    if (fabs(phi_prop) < 1.0) {
        double ratio = (1.0 - phi_prop * phi_prop) / (1.0 - th.phi * th.phi);
        if (u0[2] * u0[2] < ratio) { th.phi = phi_prop; flags |= 1; }
    }

    /* sigma_eta^2 | phi, mu: IG(a + T/2, b + Q/2) */
    double Q = SA - 2.0 * th.phi * C + th.phi * th.phi * D;
    double g_eta = orc_gamma(pr->eta_shape + 0.5 * n, seed, sweep, chain, tag,
                             IDX_GAMMA_ETA, &exhausted);
    th.sig2_eta = (pr->eta_scale + 0.5 * Q) / g_eta;

    if (terms & ORC_TERM_RV) {
        double u1[4], z_xi, unused;
        orc_uniforms4(seed, 1, sweep, chain, tag, u1);
        box_muller(u1[0], u1[1], &z_xi, &unused);
        th.xi = orc_draw_xi(T, st, th_in, pr, z_xi);
        double f = th.xi - th_in->xi;
        /* sigma_u^2 | xi: IG(a + T/2, b + sum (e_t - f)^2 / 2) */
        double SS = D2 - 2.0 * f * D1 + n * f * f;
        double g_u = orc_gamma(pr->u_shape + 0.5 * n, seed, sweep, chain, tag,
                               IDX_GAMMA_U, &exhausted);
        th.sig2_u = (pr->u_scale + 0.5 * SS) / g_u;
    }
    if (exhausted) flags |= 2;
    *th_out = th;
    return flags;
}

/* ------------------------------------------------------------------ */
/* Level move (an extension; see the header).                          */
/* ------------------------------------------------------------------ */
enum { MOVE_IDX_GAMMA = 1 };

static double log_normal_kernel(double x, double mean, double var)
{
    double d = x - mean;
    return -0.5 * d * d / var;
}

int orc_level_move(int64_t T, double *h, orc_theta *th, const double *y2, const orc_prior *pr,
                   int terms, uint64_t seed, uint64_t sweep, uint64_t chain, double *c_out)
{
    const uint64_t tag = ORC_TAG_MOVE;
    const int ret = (terms & ORC_TERM_RETURN) != 0, rv = (terms & ORC_TERM_RV) != 0;
    const double n = (double)T;
    int flags = 0;
    double u[4], z_c, unused;
    (void)unused;
    orc_uniforms4(seed, 0, sweep, chain, tag, u);
    box_muller(u[0], u[1], &z_c, &unused);
    double c_applied = 0.0;
    {
        double c;
        int accept;
        if (ret) {
            nsum sy = { 0, 0 };
            for (int64_t t = 0; t < T; ++t) nsum_add(&sy, y2[t] * exp(-h[t]));
            int exhausted = 0;
            double g = orc_gamma(0.5 * n, seed, sweep, chain, tag, MOVE_IDX_GAMMA, &exhausted);
            if (exhausted) flags |= 4;
            c = -log(2.0 * g / nsum_value(&sy));
            double log_a = log_normal_kernel(th->mu + c, pr->mu_mean, pr->mu_var)
                         - log_normal_kernel(th->mu, pr->mu_mean, pr->mu_var);
            if (rv)
                log_a += log_normal_kernel(th->xi - c, pr->xi_mean, pr->xi_var)
                       - log_normal_kernel(th->xi, pr->xi_mean, pr->xi_var);
            accept = isfinite(c) && log(u[2]) < log_a;
        } else {
            /* Gaussian in c: N(mu + c; m_mu, v_mu) [N(xi - c; m_xi, v_xi)] */
            double prec = 1.0 / pr->mu_var + (rv ? 1.0 / pr->xi_var : 0.0);
            double lin = (pr->mu_mean - th->mu) / pr->mu_var
                       + (rv ? (th->xi - pr->xi_mean) / pr->xi_var : 0.0);
            c = lin / prec + z_c / sqrt(prec);
            accept = 1;
        }
        if (accept) {
            for (int64_t t = 0; t < T; ++t) h[t] += c;
            th->mu += c;
            if (rv) th->xi -= c;
            c_applied = c;
            flags |= 2;
        }
    }
    if (c_out) *c_out = c_applied;
    return flags;
}

int64_t orc_run(int64_t T, double *h, orc_theta *th, const double *log_m,
                const double *y2, const double *r, const orc_prior *pr, int terms,
                int32_t k, double dtau, double jitter, int moves, int integrator,
                uint64_t seed, uint64_t chain, uint64_t first_sweep, int64_t n_sweeps,
                int update_theta, double *dH_trace, int32_t *acc_trace,
                orc_theta *theta_trace, double *h_trace)
{
    int64_t n_acc = 0;
    for (int64_t i = 0; i < n_sweeps; ++i) {
        uint64_t sweep = first_sweep + (uint64_t)i;
        double dH;
        double dt = orc_step_size(seed, sweep, chain, dtau, jitter);
        int acc = orc_trajectory(T, h, log_m, y2, r, th, terms, k, dt, integrator, seed,
                                 sweep, chain, NULL, NULL, NULL, &dH);
        n_acc += acc;
        if (update_theta) {
            if (moves & ORC_MOVE_LEVEL)
                orc_level_move(T, h, th, y2, pr, terms, seed, sweep, chain, NULL);
            double st[7];
            orc_suffstats(T, h, r, th->mu, th->xi, st);
            orc_theta next;
            orc_theta_update(T, st, th, pr, terms, seed, sweep, chain, &next);
            *th = next;
        }
        if (dH_trace) dH_trace[i] = dH;
        if (acc_trace) acc_trace[i] = acc;
        if (theta_trace) theta_trace[i] = *th;
        if (h_trace) memcpy(h_trace + i * T, h, (size_t)T * sizeof(double));
    }
    return n_acc;
}
