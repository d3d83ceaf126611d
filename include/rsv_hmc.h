/*
 * rsv_hmc.h -- C ABI of the MI355X (gfx950) HIP library for the Hybrid Monte
 * Carlo volatility update of the realized stochastic volatility (RSV) model.
 *
 * Paper: T. Takaishi, "GPU Computing in Bayesian Inference of Realized
 * Stochastic Volatility Model", arXiv:1603.08114.
 *   Sec. 2, eqs. (1)-(3)  the RSV model: y_t = exp(h_t/2) eps_t,
 *                         ln RV_t = xi + h_t + u_t,
 *                         h_{t+1} = mu + phi (h_t - mu) + eta_t;
 *                         theta = (phi, mu, xi, sigma_eta^2, sigma_u^2).
 *   Sec. 3, eqs. (4)-(5)  Hamilton's equations, H = 1/2 sum p^2 - ln f(h,theta).
 *   Sec. 3, eqs. (6)-(8)  second-order leapfrog (h half step, p full step,
 *                         h half step), repeated k times, l = k dtau.
 *   Sec. 3 (end)          Metropolis test, accept with min{1, exp(-dH)}.
 *   Sec. 5, eqs. (9)-(11) the same step applied to all sites i = 1..T in
 *                         parallel (here fused, and blocked in time).
 *
 * Conventions for every entry point
 *   - Sites are 0-based: site t here is the paper's t+1.
 *   - "device" pointers are HIP device memory owned by the caller (the
 *     Python binding passes torch tensors).  The library never allocates or
 *     frees device memory; it works inside the caller's workspace.
 *   - "host" pointers are read during the call only.
 *   - All work is enqueued on the stream given to rsv_hmc_init.  Init and
 *     rsv_hmc_check synchronise; rsv_hmc_momenta, rsv_hmc_trajectory,
 *     rsv_theta_update and rsv_hmc_sweep first wait for the work already on
 *     the stream and read the non-finite flag (below), then only enqueue.
 *     A context of rsv_hmc_init with two or more chains also owns a side
 *     stream (default priority) and two events, made at init and destroyed
 *     by rsv_hmc_destroy: rsv_hmc_sweep runs about half of the chains there,
 *     forked from the given stream by an event at the start of the call and
 *     joined back into it by another at its end, so the call's work is
 *     ordered on the given stream as a whole.  Results are the same as on
 *     one stream, bit for bit.
 *   - A non-OK status leaves the context usable; rsv_last_error() returns a
 *     thread-local message describing the most recent failure.
 *   - Non-finite state.  The trajectory kernel flags a non-finite value in
 *     the current state h or in theta (accepted proposals always have a
 *     finite dH, so only a caller's write puts one there), and the theta
 *     update keeps theta unchanged and flags it when its draw would not be
 *     finite.  rsv_hmc_momenta, rsv_hmc_trajectory, rsv_theta_update and
 *     rsv_hmc_sweep return RSV_ENONFINITE, enqueuing nothing, while that flag
 *     is set, so the call after the one whose kernels set it returns it.
 *     The chains stay at their last accepted state (a trajectory from a
 *     non-finite state is rejected).  rsv_hmc_check clears the flag once the
 *     state is finite again.
 *   - One context per stream; a context is not thread-safe.
 *
 * Data layout (HBM)
 *   Series s = 0..S-1 has T_s = offsets[s+1] - offsets[s] sites; its data
 *   y, log_rv occupy [offsets[s], offsets[s+1]) of the data arrays.
 *   Chain c = s*C + j (j = 0..C-1) has its state h at
 *   [C*offsets[s] + j*T_s, C*offsets[s] + (j+1)*T_s) of the state array:
 *   every chain is one contiguous run of sites, chains of a series adjacent.
 *   theta is one rsv_theta per chain (array of structs, 40 bytes each).
 */
#ifndef RSV_HMC_H
#define RSV_HMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rsv_status;
enum {
    RSV_OK = 0,
    RSV_EINVAL = -1,     /* an argument or the problem is invalid           */
    RSV_EDEVICE = -2,    /* a HIP call failed                               */
    RSV_ENOMEM = -3,     /* the workspace is too small                      */
    RSV_ESTATE = -4,     /* call out of order (e.g. context not initialised) */
    RSV_ENONFINITE = -5  /* non-finite state or data was detected           */
};

/* Arithmetic of the leapfrog.  RSV_F64: everything in FP64.
 * RSV_F32_MIXED: h, p and the force in FP32; dH, the Metropolis log-ratio,
 * the sufficient statistics and theta in FP64. */
typedef enum { RSV_F64 = 0, RSV_F32_MIXED = 1 } rsv_precision;

/* Model terms of -ln f.  Both on = the RSV model of eqs. (1)-(3).  Without
 * RSV_TERM_RETURN (eq. (1)) the model is linear-Gaussian; without
 * RSV_TERM_RV (eq. (2)) it is the plain SV model and xi, sigma_u^2 are not
 * updated. */
enum { RSV_TERM_RETURN = 1, RSV_TERM_RV = 2, RSV_TERMS_RSV = 3 };

/* Flags.
 * RSV_FLAG_RESIDENT: rsv_hmc_sweep runs every sweep of a call in a single
 *   launch (when the tile shape has one or four wavefronts and no chain has
 *   more than 64 tiles): whole chains are packed into bins, one block per
 *   bin, which integrates its tiles, then runs one finalize (dH total,
 *   Metropolis test, theta update) per chain on one of its wavefronts, with
 *   a block barrier between, for every sweep.  Without the flag each sweep
 *   is one launch of the trajectory kernel and one of the finalize kernel,
 *   which measures faster on MI355X at every problem size tried (the fused
 *   kernel needs more registers and its blocks wait for their serial
 *   finalize).  Results are identical either way, bit for bit.
 * RSV_FLAG_LEVEL_MOVE: every theta update (rsv_hmc_sweep with update_theta,
 *   rsv_theta_update) first moves the whole state along h_t -> h_t + c,
 *   mu -> mu + c, xi -> xi - c (xi only with RSV_TERM_RV).  That direction
 *   leaves the AR(1) part and the RV residuals unchanged; with the return
 *   term e^{-c} is drawn from Gamma(T/2, rate S/2), S = sum_t y_t^2 e^{-h_t},
 *   and the prior ratio of mu (and xi) is the Metropolis test; without it c
 *   is drawn from the Gaussian prior factors.  Random numbers: Philox stream
 *   tag 4, block 0 (Box-Muller z from u0, u1; u2 the test), Gamma attempts
 *   in blocks 1..32.  An extension: the paper's method updates h only, and
 *   the Gibbs theta step alone mixes slowly along this direction (xi + h_t is
 *   pinned by ln RV_t).  Off by default.
 * RSV_FLAG_OMELYAN: the trajectory integrates with Omelyan's second-order
 *   minimum-norm scheme instead of the leapfrog of eqs. (6)-(8) (Sec. 3
 *   allows higher-order integrators): each of the n_steps steps moves h by
 *   lambda dtau, p by dtau/2, h by (1 - 2 lambda) dtau, p by dtau/2, h by
 *   lambda dtau (lambda = 0.1931833275037836; Omelyan, Mryglod and Folk,
 *   Comput. Phys. Commun. 151 (2003) 272).  Two force evaluations per step,
 *   so a step costs about twice a leapfrog step and the halo of a tile is
 *   sized for 2 n_steps (max_steps is checked against that).  Off by
 *   default.
 * RSV_FLAG_FOREST_RUTH: Forest and Ruth's fourth-order scheme (Physica D 43
 *   (1990) 105) instead: each step moves h by theta/2 dtau, p by theta dtau,
 *   h by (1 - theta)/2 dtau, p by (1 - 2 theta) dtau, h by (1 - theta)/2
 *   dtau, p by theta dtau, h by theta/2 dtau, theta = 1/(2 - 2^(1/3)).
 *   Three force evaluations per step; the halo is sized for 3 n_steps.  At
 *   most one of RSV_FLAG_OMELYAN and RSV_FLAG_FOREST_RUTH (EINVAL if both).
 *   Off by default. */
enum {
    RSV_FLAG_RESIDENT = 1,
    RSV_FLAG_LEVEL_MOVE = 2,
    RSV_FLAG_OMELYAN = 4,
    RSV_FLAG_FOREST_RUTH = 8
};

/* theta of Sec. 2. */
typedef struct { double phi, mu, xi, sig2_eta, sig2_u; } rsv_theta;

/* Priors of the theta update.  The paper states none; the reading taken is
 * phi ~ U(-1,1), mu ~ N(mu_mean, mu_var), xi ~ N(xi_mean, xi_var),
 * sigma_eta^2 ~ IG(eta_shape, eta_scale), sigma_u^2 ~ IG(u_shape, u_scale). */
typedef struct {
    double mu_mean, mu_var, xi_mean, xi_var;
    double eta_shape, eta_scale, u_shape, u_scale;
} rsv_prior;

/* Integrator knobs of Sec. 3: k steps of size dtau (leapfrog steps, or
 * Omelyan / Forest-Ruth steps under their flags). */
typedef struct { int32_t n_steps; int32_t reserved; double dtau; } rsv_leapfrog;

typedef struct {
    int32_t n_series;           /* S >= 1                                      */
    int32_t chains_per_series;  /* C >= 1                                      */
    const int64_t *offsets;     /* host, S+1 entries, offsets[0] = 0,
                                   T_s = offsets[s+1]-offsets[s] >= 3          */
    const double *y;            /* device, offsets[S] daily returns y_t        */
    const double *log_rv;       /* device, offsets[S] values ln RV_t           */
    int32_t precision;          /* rsv_precision                               */
    int32_t terms;              /* RSV_TERM_* bit set, at least one bit        */
    int32_t max_steps;          /* largest k any later call will use (>= 1)    */
    int32_t sites_per_lane;     /* tile shape of the trajectory kernel: sites
                                   held by each lane (0 = library default: 4
                                   for RSV_F64, 8 for RSV_F32_MIXED; compiled:
                                   RSV_F64 4 or 8, RSV_F32_MIXED 8 or 16)       */
    int32_t waves_per_tile;     /* wavefronts per tile (0 = default 4; compiled
                                   (S, NW): F64 S in {4, 8} x NW in {1, 2, 4,
                                   8}; F32 S = 8 x NW in {1, 2, 4, 8} and
                                   S = 16 x NW in {1, 2, 4}).  Resident
                                   sweeps (see RSV_FLAG_RESIDENT) run for
                                   NW in {1, 4}.
                                   A tile spans 64 * waves_per_tile *
                                   sites_per_lane sites, of which all but a
                                   k+1 halo on each cut side are exact          */
    int32_t flags;              /* RSV_FLAG_* bit set (0 = defaults)           */
    uint64_t seed;              /* key of all random streams                   */
    double dtau_jitter;         /* j in [0, 1): the step size of every
                                   trajectory is dtau * (1 + j (2u - 1)), u the
                                   first uniform of Philox block (0, sweep,
                                   chain, tag 3); 0 = the paper's fixed dtau.
                                   An extension: a factor drawn independently
                                   of the state keeps the chain exact and
                                   breaks near-periodic orbits of modes whose
                                   period divides k * dtau                      */
    rsv_prior prior;
} rsv_problem;

/* Per-sweep records written by rsv_hmc_sweep.  Every pointer may be NULL. */
typedef struct {
    double *delta_h;     /* device, n_sweeps * n_chains, dH of each trajectory */
    int32_t *accepted;   /* device, n_sweeps * n_chains, 1 if accepted         */
    rsv_theta *theta;    /* device, n_sweeps * n_chains, theta after the sweep */
    void *h;             /* device, n_sweeps * n_state, h after the sweep, in the
                            state precision (FP64 or FP32)                      */
    /* Moment accumulators for runs too long to store (batch means): after
     * sweep i of the call, h is added to h_batch_sum[(i / batch_len) * n_state
     * + site] and h^2 to h_sq_sum[site] (FP64; the caller zeroes them).  The
     * states of a batch are summed in FP32 in the workspace and the batch
     * total is added to these arrays (relative error ~ batch_len * 6e-8;
     * without h_batch_sum the squares are added every 64 sweeps). */
    double *h_batch_sum; /* device, ceil(n_sweeps / batch_len) * n_state, or NULL */
    double *h_sq_sum;    /* device, n_state, or NULL                            */
    int32_t batch_len;   /* sweeps per batch (>= 1 when h_batch_sum is set)    */
    int32_t reserved;
} rsv_trace;

typedef struct rsv_ctx rsv_ctx;

/* Bytes of device workspace rsv_hmc_init needs for this problem (0 if the
 * problem is invalid; see rsv_last_error): the proposal state buffer, y^2
 * (and FP32 copies on the mixed path), the tile descriptors and per-tile
 * partials, per-chain selectors and level shifts, and one entry of the
 * state's type per data site for the diagonal-mass table (sqrt(m_t), 8 bytes
 * in FP64, 4 in FP32; reserved whether or not a mass is given). */
size_t rsv_hmc_workspace_bytes(const rsv_problem *pb);

/* Number of state entries, C * offsets[S] (0 if invalid). */
int64_t rsv_hmc_state_size(const rsv_problem *pb);

/* Create a context.
 *   h        device, rsv_hmc_state_size entries of double (RSV_F64) or float
 *            (RSV_F32_MIXED): the initial h on entry; the library keeps the
 *            current state of every chain here after each call.
 *   theta    device, S*C rsv_theta, initial values; updated in place.
 *   log_mass device, offsets[S] floats: log of the diagonal mass m_t of each
 *            series-site (shared by the chains of a series), or NULL for
 *            m = 1 (the paper's kinetic term 1/2 sum p^2).  Read once here:
 *            sqrt(m_t) is kept in the workspace in the state's precision
 *            (rounded to FP32 on the mixed path; that value defines the
 *            mass: momenta are drawn as z sqrt(m_t) and the kinetic term
 *            uses 1/m_t formed from it in FP64).  A site whose ln m_t is
 *            not finite or outside [-80, 80] takes m_t = 1 (the identity
 *            mass; the chain stays exact for any fixed positive mass).
 *   workspace, ws_bytes  device scratch of at least rsv_hmc_workspace_bytes.
 *   hip_stream  hipStream_t to enqueue on (NULL = the null stream).
 * Validates the problem on the host and the data, h and theta on the device
 * (one synchronisation): RSV_EINVAL for T_s < 3, non-finite y / log_rv / h,
 * |phi| >= 1, a variance <= 0 or a bad prior; RSV_ENOMEM if ws_bytes is too
 * small.  The pointers are borrowed and must outlive the context. */
rsv_status rsv_hmc_init(rsv_ctx **out, const rsv_problem *pb, void *h, rsv_theta *theta,
                        const float *log_mass, void *workspace, size_t ws_bytes,
                        void *hip_stream);

/* rsv_hmc_init for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same context, but its workspace is a library-owned device array of
 * RSV_STATIC_WORKSPACE_BYTES (32 MiB) on the device current at the call,
 * which that device keeps until the process ends.  Nothing is allocated on
 * the device here or in later calls on the context.  Limit: problems whose
 * rsv_hmc_workspace_bytes exceeds RSV_STATIC_WORKSPACE_BYTES get
 * RSV_ENOMEM (e.g. one FP64 chain of more than about 1 040 000 sites).
 * Sharing: every static context on a device uses that device's one array,
 * and each rsv_hmc_init_static takes it over: calls on an older static
 * context of the device then return RSV_ESTATE.  The array keeps the last
 * context's contents; initialisation clears what must start at zero.  Work
 * of an older static context still running when a new one is created races
 * with it: synchronise that context's stream first.  Other arguments and
 * errors as rsv_hmc_init. */
#define RSV_STATIC_WORKSPACE_BYTES (32u << 20)
rsv_status rsv_hmc_init_static(rsv_ctx **out, const rsv_problem *pb, void *h, rsv_theta *theta,
                               const float *log_mass, void *hip_stream);

/* Momentum refresh of sweep `sweep` (the Gibbs draw p ~ N(0, m) implied by
 * the kinetic term of H, Sec. 3), written to p_out (device, FP64, one entry
 * per state entry).  The trajectory of that sweep starts from exactly these
 * momenta.  FP64: site t of a chain takes normal t%4 of Philox block t/4
 * (Box-Muller on the block's two pairs of 52-bit uniforms).  FP32-mixed:
 * site t takes normal t%8 of block t/8; word q of the block gives sites 2q
 * and 2q+1 by Box-Muller on u0 from its top 40 bits and u1 from its low 24,
 * formed in FP32 (as is the product with sqrt(m_t)), so the values are FP32
 * numbers. */
rsv_status rsv_hmc_momenta(rsv_ctx *c, uint64_t sweep, double *p_out);

/* One HMC trajectory for every chain (Sec. 3): momentum refresh, k leapfrog
 * steps of eqs. (6)-(8) (or of the scheme an integrator flag selects),
 * dH = H(p',h') - H(p,h) as a compensated FP64 sum
 * of per-site differences, and the Metropolis test accept iff
 * ln u < -dH (a non-finite dH rejects).  On acceptance the chain's state
 * becomes h', else it stays.  theta is not changed.
 *   lf       host, one rsv_leapfrog per series (k <= max_steps, dtau > 0).
 *   p0       device FP64 momenta overriding the refresh, or NULL.
 *   log_u    device FP64 per chain overriding ln u, or NULL.
 *   delta_h  device FP64 per chain, or NULL.   accepted: device int32 per
 *            chain, or NULL. */
rsv_status rsv_hmc_trajectory(rsv_ctx *c, uint64_t sweep, const rsv_leapfrog *lf,
                              const double *p0, const double *log_u,
                              double *delta_h, int32_t *accepted);

/* theta update of every chain from the current h (the paper's parameter
 * estimation by MCMC, Sec. 2; the sampler is a reading): Gibbs sweep
 * mu -> phi (independence Metropolis) -> sigma_eta^2 -> xi -> sigma_u^2,
 * each conditional formed from sufficient statistics of h reduced on the
 * GPU in FP64.
 *   suff_stats  device FP64, 7 per chain {B, B2, BB, D1, D2, b_first, b_last}
 *               with b_t = h_t - mu, e_t = ln RV_t - h_t - xi (theta before
 *               the update): B = sum b, B2 = sum b^2, BB = sum b_t b_{t+1},
 *               D1 = sum e, D2 = sum e^2; or NULL. */
rsv_status rsv_theta_update(rsv_ctx *c, uint64_t sweep, double *suff_stats);

/* n_sweeps sweeps, each one trajectory (as rsv_hmc_trajectory, streams of
 * sweep first_sweep + i) followed, if update_theta, by the theta update (as
 * rsv_theta_update).  trace (host struct of device pointers) may be NULL. */
rsv_status rsv_hmc_sweep(rsv_ctx *c, uint64_t first_sweep, int32_t n_sweeps,
                         const rsv_leapfrog *lf, int32_t update_theta,
                         const rsv_trace *trace);

/* Synchronise the stream and report device-side events since the last
 * check: *n_nonfinite (may be NULL) receives the number of trajectories
 * whose dH was not finite (diverged trajectories, which were rejected).
 * Recounts the current state: returns RSV_ENONFINITE if any chain holds a
 * non-finite value, else RSV_OK and clears the non-finite flag that the
 * other calls report. */
rsv_status rsv_hmc_check(rsv_ctx *c, int64_t *n_nonfinite);

/* Kernel timing (measurement support).  rsv_hmc_profile allocates
 * max_records pairs of HIP events (0 frees them); while records remain, each
 * later trajectory launch (in rsv_hmc_trajectory or one sweep of
 * rsv_hmc_sweep) is bracketed by a pair recorded on the context's stream
 * around the trajectory kernel only, and a resident launch (all sweeps of an
 * rsv_hmc_sweep call) by one pair around it.  rsv_hmc_kernel_time waits for
 * the last record, returns the summed milliseconds and the number of
 * trajectories the records cover (a resident launch of n sweeps counts n),
 * and starts a new series of records. */
rsv_status rsv_hmc_profile(rsv_ctx *c, int32_t max_records);
rsv_status rsv_hmc_kernel_time(rsv_ctx *c, double *total_ms, int64_t *n_records);

/* Free the host context (device memory stays the caller's). */
rsv_status rsv_hmc_destroy(rsv_ctx *c);

/* Message of the last non-OK status on this thread ("" if none). */
const char *rsv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
