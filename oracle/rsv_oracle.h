/*
 * rsv_oracle.h -- plain FP64 CPU oracle of the RSV-model HMC volatility update.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP library under
 * paper_1603_08114_amd/; the two are written independently and compared.
 *
 * Paper: T. Takaishi, "GPU Computing in Bayesian Inference of Realized
 * Stochastic Volatility Model" (arXiv:1603.08114).
 *   Sec. 2, eqs. (1)-(3): the RSV model.
 *   Sec. 3, eqs. (4)-(5): Hamilton's equations; H = 1/2 sum p^2 - ln f(h,theta).
 *   Sec. 3, eqs. (6)-(8): second-order leapfrog in h-p-h order, k steps.
 *   Sec. 3 (end): Metropolis test with probability min{1, exp(-dH)}.
 *
 * Sites are 0-based here (t = 0..T-1 is the paper's t = 1..T).
 * Every array is caller-owned host memory.  Nothing here allocates except
 * the scratch of orc_run, which it frees before returning.
 */
#ifndef RSV_ORACLE_H
#define RSV_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* theta = (phi, mu, xi, sigma_eta^2, sigma_u^2), Sec. 2 */
typedef struct { double phi, mu, xi, sig2_eta, sig2_u; } orc_theta;

/* Priors of the theta update (the paper states none; readings):
 * phi ~ U(-1,1), mu ~ N(mu_mean, mu_var), xi ~ N(xi_mean, xi_var),
 * sigma_eta^2 ~ IG(eta_shape, eta_scale), sigma_u^2 ~ IG(u_shape, u_scale). */
typedef struct {
    double mu_mean, mu_var, xi_mean, xi_var;
    double eta_shape, eta_scale, u_shape, u_scale;
} orc_prior;

/* Model-term switches.  Both on = the RSV model of eqs. (1)-(3).
 * Dropping eq. (1) leaves a linear-Gaussian state-space model (a pin);
 * dropping eq. (2) leaves the plain SV model. */
enum { ORC_TERM_RETURN = 1, ORC_TERM_RV = 2, ORC_TERMS_RSV = 3 };

/* Random-number stream tags (Philox counter word 3). */
enum { ORC_TAG_MOMENTUM = 0, ORC_TAG_ACCEPT = 1, ORC_TAG_THETA = 2, ORC_TAG_STEP = 3,
       ORC_TAG_MOVE = 4 };

/* Moves that orc_run applies before each theta update (bit set). */
enum { ORC_MOVE_LEVEL = 2 };

/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
/* Four uniforms in (0,1) for counter (idx, sweep, chain, tag) and key (seed, 0). */
void orc_uniforms4(uint64_t seed, uint64_t idx, uint64_t sweep, uint64_t chain,
                   uint64_t tag, double u[4]);
/* Fill out[n] with consecutive uniforms / standard normals of one stream
 * (normals: Box-Muller on the pairs (u0,u1), (u2,u3) of each block). */
void orc_uniform_stream(uint64_t seed, uint64_t sweep, uint64_t chain, uint64_t tag,
                        int64_t n, double *out);
void orc_normal_stream(uint64_t seed, uint64_t sweep, uint64_t chain, uint64_t tag,
                       int64_t n, double *out);

/* Negative log conditional posterior U(h) = -ln f(h|theta,data) + const,
 * from eqs. (1)-(3) with a stationary h_1. y2[t] = y_t^2, r[t] = ln RV_t. */
double orc_energy(int64_t T, const double *h, const double *y2, const double *r,
                  const orc_theta *th, int terms);
/* g[t] = dU/dh_t (the force of eq. (7) is -g). */
void orc_grad(int64_t T, const double *h, const double *y2, const double *r,
              const orc_theta *th, int terms, double *g);
/* H(p,h) = sum p_t^2/(2 m_t) + U(h), Sec. 3.  log_m == NULL means m = 1. */
double orc_hamiltonian(int64_t T, const double *h, const double *p, const double *log_m,
                       const double *y2, const double *r, const orc_theta *th, int terms);
/* k leapfrog steps of eqs. (6)-(8), in place. */
void orc_leapfrog(int64_t T, double *h, double *p, const double *log_m,
                  const double *y2, const double *r, const orc_theta *th, int terms,
                  int32_t k, double dtau);
/* Integrators of the trajectory: the paper's leapfrog, Omelyan's
 * second-order minimum-norm scheme (h-first form, lambda below), or Forest
 * and Ruth's fourth-order scheme (h-first form, theta below). */
enum { ORC_INT_LEAPFROG = 0, ORC_INT_OMELYAN = 1, ORC_INT_FOREST_RUTH = 2 };
#define ORC_OMELYAN_LAMBDA 0.1931833275037836
#define ORC_FOREST_RUTH_THETA 1.3512071919596578
/* k steps of the Omelyan scheme, in place (2k force evaluations). */
void orc_omelyan(int64_t T, double *h, double *p, const double *log_m,
                 const double *y2, const double *r, const orc_theta *th, int terms,
                 int32_t k, double dtau);
/* k steps of the Forest-Ruth scheme, in place (3k force evaluations). */
void orc_forest_ruth(int64_t T, double *h, double *p, const double *log_m,
                     const double *y2, const double *r, const orc_theta *th, int terms,
                     int32_t k, double dtau);
/* k steps of the integrator `integrator` (ORC_INT_*), in place. */
void orc_integrate(int64_t T, double *h, double *p, const double *log_m,
                   const double *y2, const double *r, const orc_theta *th, int terms,
                   int32_t k, double dtau, int integrator);
/* dH = H(h1,p1) - H(h0,p0) as a compensated sum of per-site differences. */
double orc_delta_h(int64_t T, const double *h0, const double *p0,
                   const double *h1, const double *p1, const double *log_m,
                   const double *y2, const double *r, const orc_theta *th, int terms);
/* Momentum refresh p_t ~ N(0, m_t) for (seed, sweep, chain). */
void orc_momenta(uint64_t seed, uint64_t sweep, uint64_t chain, int64_t T,
                 const double *log_m, double *p);
/* The same on the FP32-mixed path's stream layout (8 sites per block). */
void orc_momenta_f32(uint64_t seed, uint64_t sweep, uint64_t chain, int64_t T,
                     const double *log_m, double *p);
/* log u of the Metropolis test of (seed, sweep, chain). */
double orc_log_u(uint64_t seed, uint64_t sweep, uint64_t chain);

/* Step size of sweep (seed, sweep, chain) under step-size jitter j in [0,1):
 * dtau * (1 + j (2u - 1)) with u the first uniform of block 0 of stream tag 3
 * (an extension: the paper's dtau is fixed; j = 0 returns dtau). */
double orc_step_size(uint64_t seed, uint64_t sweep, uint64_t chain, double dtau, double jitter);

/* One HMC trajectory on h (in place: left at h' if accepted, else at h0)
 * with k steps of the integrator `integrator` (ORC_INT_*).
 * p0 / log_u may be NULL (then drawn from the streams).  p_out (may be NULL)
 * receives the momenta used.  Returns 1 if accepted, 0 if rejected. */
int orc_trajectory(int64_t T, double *h, const double *log_m,
                   const double *y2, const double *r, const orc_theta *th, int terms,
                   int32_t k, double dtau, int integrator, uint64_t seed, uint64_t sweep,
                   uint64_t chain, const double *p0, const double *log_u, double *p_out,
                   double *dH_out);

/* Sufficient statistics of h for the theta update with shifts c_mu, c_xi:
 * out = {B, B2, BB, D1, D2, b_first, b_last}. */
void orc_suffstats(int64_t T, const double *h, const double *r, double c_mu, double c_xi,
                   double out[7]);

/* One theta update mu -> phi -> sigma_eta^2 -> xi -> sigma_u^2 from the
 * statistics of h (shifts = th_in->mu, th_in->xi).  Returns a bit set:
 * 1 = phi proposal accepted, 2 = a Gamma draw ran out of attempts. */
int orc_theta_update(int64_t T, const double stats[7], const orc_theta *th_in,
                     const orc_prior *pr, int terms, uint64_t seed, uint64_t sweep,
                     uint64_t chain, orc_theta *th_out);

/* Single conditional draws (each from the stats of h and the current theta),
 * exposed so each conditional can be checked on its own. */
double orc_draw_mu(int64_t T, const double stats[7], const orc_theta *th, const orc_prior *pr,
                   double z);
double orc_draw_xi(int64_t T, const double stats[7], const orc_theta *th, const orc_prior *pr,
                   double z);
/* Gamma(alpha, 1) by Marsaglia-Tsang over attempts idx0.. of stream (seed,sweep,chain,tag);
 * *exhausted set to 1 when no attempt is accepted. */
double orc_gamma(double alpha, uint64_t seed, uint64_t sweep, uint64_t chain, uint64_t tag,
                 uint64_t idx0, int *exhausted);

/* Compensated (Neumaier) sum. */
double orc_neumaier_sum(int64_t n, const double *x);

/* Level move of the whole state (an extension: the paper updates h only,
 * and the Gibbs theta step alone moves slowly along this direction, on
 * which ln RV pins xi + h_t):  h_t -> h_t + c, mu -> mu + c and, with the RV
 * term, xi -> xi - c.  The AR(1) part and the RV residuals are unchanged, so
 * along this orbit the posterior is the return term times the priors of mu
 * and xi.  With the return term, e^{-c} is drawn from its exact law given
 * the return term, Gamma(T/2, rate S/2) with S = sum y_t^2 e^{-h_t}, and the
 * prior ratio of mu (and xi) decides a Metropolis test (an independence
 * sampler along the orbit); without it, c is drawn from the Gaussian prior
 * part.  Applied on h in place and *th.  Random
 * numbers: stream tag 4, block 0 = (u0, u1 -> z by Box-Muller, u2 = test);
 * Gamma attempts from block 1 on.  *c_out (may be NULL) receives the c
 * applied (0 when rejected).  Returns a bit set: 2 = accepted, 4 = the Gamma
 * draw ran out of attempts. */
int orc_level_move(int64_t T, double *h, orc_theta *th, const double *y2, const orc_prior *pr,
                   int terms, uint64_t seed, uint64_t sweep, uint64_t chain, double *c_out);

/* n sweeps (trajectory, then optional theta update) of one chain; the step
 * size of each sweep is orc_step_size(seed, sweep, chain, dtau, jitter);
 * with update_theta the moves `moves` (ORC_MOVE_LEVEL) run between the
 * trajectory and the Gibbs theta update.
 * Traces (each may be NULL): dH[n], acc[n], theta[n] (after the sweep),
 * h_trace[n*T] (h after each sweep).  Returns the number accepted. */
int64_t orc_run(int64_t T, double *h, orc_theta *th, const double *log_m,
                const double *y2, const double *r, const orc_prior *pr, int terms,
                int32_t k, double dtau, double jitter, int moves, int integrator,
                uint64_t seed, uint64_t chain, uint64_t first_sweep, int64_t n_sweeps,
                int update_theta, double *dH_trace, int32_t *acc_trace,
                orc_theta *theta_trace, double *h_trace);

#ifdef __cplusplus
}
#endif
#endif
