// rsv_internal.h -- descriptors shared by the host library and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsv_hmc.h"

namespace rsv {

// A tile is the part of one chain that one group of NW wavefronts integrates
// through a whole trajectory.  It loads sites [la, la + 64*NW*S) (clipped to
// [0, T)),
// and after k steps the sites [a, b) are exact; the halo on either side is
// at least k+1 sites (absent at the ends of the series).  la is a multiple
// of 4 so that each lane's sites are whole Philox blocks.
struct TileDesc {
    int32_t chain;
    int32_t la;
    int32_t a;
    int32_t b;
    int32_t edge;  // 1 if the chain's last site lies strictly inside a lane
    int32_t pad[3];
};

struct ChainDesc {
    int64_t h_off;       // state index of site 0
    int64_t d_off;       // data index of site 0 (its series)
    int32_t T;
    int32_t series;
    int32_t tile_begin;  // tiles [tile_begin, tile_begin + tile_count) ...
    int32_t tile_count;
    int32_t edge_tile;   // ... plus this one (-1 if none)
    int32_t n_steps;     // leapfrog steps k
    double dtau;
};

// Per-tile partial results (doubles): dH, then {B,B2,BB,D1,D2} of the
// proposal h', then of the current h, then S = sum y_t^2 e^{-h_t} of h' and
// of h (the level move's statistic).  Padded to 16.
constexpr int kPart = 16;
constexpr int kPartDH = 0, kPartProp = 1, kPartCur = 6, kPartSyProp = 11, kPartSyCur = 12;
constexpr int kNQ = 13;  // partials in use
// Per-chain edge values: b_first', b_last', b_first, b_last.
constexpr int kEdge = 4;

// Counters (uint32 each) kept in the workspace.
enum { kCntNonfiniteDH = 0, kCntNonfiniteState = 1, kCntNonfiniteData = 2, kCntGammaExhausted = 3,
       kNumCounters = 8 };

// Integrators of the trajectory kernel.
enum : int32_t { kIntLeapfrog = 0, kIntOmelyan = 1, kIntForestRuth = 2 };

template <typename R>
struct TrajArgs {
    const TileDesc* tiles;
    int32_t tile_first;         // this launch handles tiles [tile_first, tile_first + n_list)
    int32_t n_list;
    const ChainDesc* chains;
    const rsv_theta* theta;
    const R* h_a;               // the caller's state buffer
    R* h_b;                     // the workspace's second state buffer
    const int32_t* state_sel;   // per chain: 1 if its current state is in h_b
    const R* y2;                // y_t^2 in R
    const R* lrv;               // ln RV_t in R
    const double* y2_d;         // FP64 copies for dH and the statistics
    const double* lrv_d;
    const R* mass_sqrt;         // per data site sqrt(m_t) in R, or nullptr (identity mass)
    const double* p0;           // momentum override (per state entry) or nullptr
    uint64_t seed;
    uint64_t sweep;
    double* partials;           // kPart per tile
    double* chain_edge;         // kEdge per chain
    double jitter;              // step-size jitter j (0: fixed dtau)
    const double* shift;        // per chain: pending level shift of the current
                                // state (value = stored + shift), or nullptr
    float* acc_sum;             // per state entry: add the state the trajectory
    float* acc_sq;              // starts from, and its square (or nullptr)
    R* h_prev_out;              // per state entry: the state the trajectory starts
                                // from (the previous sweep's trace row), or nullptr
    int32_t terms;
    int32_t integrator;         // kIntLeapfrog, kIntOmelyan or kIntForestRuth
    uint32_t* counters;         // kCntNonfiniteState is set on a non-finite state
};

struct FinalizeArgs {
    const ChainDesc* chains;
    int32_t chain_first;        // a launch finalizes chains [chain_first, + n_chains)
    int32_t n_chains;
    const double* partials;
    const double* chain_edge;
    rsv_theta* theta;
    rsv_prior prior;
    uint64_t seed;
    uint64_t sweep;
    int32_t terms;
    int32_t do_metropolis;      // use dH + Metropolis; else stats of the current h
    int32_t do_theta;
    const double* log_u;        // override or nullptr
    int32_t* state_sel;         // per chain: flipped when the proposal is accepted
    double* delta_h_out;        // per chain or nullptr
    int32_t* accepted_out;      // per chain or nullptr
    rsv_theta* theta_trace;     // per chain or nullptr
    double* stats_out;          // 7 per chain or nullptr
    uint32_t* counters;
    int32_t level_move;         // apply the level move before the Gibbs theta step
    double* shift;              // per chain pending level shift (with level_move)
    double* slices;             // split finalize: compensated slice sums (kNQ pairs each)
    uint32_t* arrive;           // split finalize: per chain, slices done (0 between launches)
};

// Split finalize: chains are reduced in slices of kSliceTiles tiles by one
// block each; slice s of chain c is stored at index c + tile_begin / kSliceTiles
// + s (disjoint across chains, at most tiles / kSliceTiles + n_chains).
constexpr int kSliceTiles = 128;

// Record the message returned by rsv_last_error() and return `code`.
rsv_status set_error(rsv_status code, const char* where, const char* what);

// Resident sweeps (rsv_bin.h): whole chains packed into bins, one per block.
struct BinDesc {
    int32_t chain_first;  // its chains are bin_chains[chain_first, + chain_count)
    int32_t chain_count;
    int32_t tile_first;   // their tiles are bin_tiles[tile_first, + tile_count)
    int32_t tile_count;
};

template <typename R>
struct BinArgs {
    TrajArgs<R> traj;          // sweep and acc_sum/acc_sq set per sweep
    FinalizeArgs fin;          // sweep and per-sweep outputs set per sweep
    const BinDesc* bins;
    const int32_t* bin_chains;  // chain indices
    const int32_t* bin_tiles;   // tile indices
    int32_t n_bins;
    int32_t n_sweeps;
    int32_t batch_len;         // sweeps per batch of the FP32 batch sums
    int32_t reserved;
    uint64_t first_sweep;
    int64_t n_state;
    double* dh_trace;          // n_sweeps * n_chains or nullptr
    int32_t* acc_trace;
    rsv_theta* theta_trace;
    R* h_trace;                // n_sweeps * n_state or nullptr
    float* acc_sum;            // FP32 sums of the current batch (or nullptr)
    float* acc_sq;
    double* batch_sum;         // the caller's accumulators (see rsv_trace) or nullptr
    double* sq_sum;
};

// Launchers (rsv_kernels.hip, rsv_traj_*.hip, rsv_resident.hip).  Each returns the hipError_t of its launch.
hipError_t launch_prepare(hipStream_t st, const double* y, const double* lrv, int64_t n,
                          double* y2_d, float* y2_f, float* lrv_f);
hipError_t launch_validate(hipStream_t st, const double* y, const double* lrv, int64_t n_data,
                           const void* h, int64_t n_state, int precision, uint32_t* counters);
hipError_t launch_traj(hipStream_t st, int precision, int S, int NW, bool mass,
                       const void* args);
// Per-precision, per-mass instantiations (rsv_traj_{f64,f32}[_mass].hip).
hipError_t launch_traj_f64(hipStream_t st, int S, int NW, const TrajArgs<double>& a);
hipError_t launch_traj_f64_mass(hipStream_t st, int S, int NW, const TrajArgs<double>& a);
hipError_t launch_traj_f32(hipStream_t st, int S, int NW, const TrajArgs<float>& a);
hipError_t launch_traj_f32_mass(hipStream_t st, int S, int NW, const TrajArgs<float>& a);
bool traj_shape_available(int precision, int S, int NW);
void traj_default_shape(int precision, int* S, int* NW);
hipError_t launch_finalize(hipStream_t st, const FinalizeArgs& a, int32_t max_tiles_per_chain);
// All n sweeps of chains that each fit one tile, packed into bins, in one launch.
hipError_t launch_bin(hipStream_t st, int precision, int S, int NW, bool mass, const void* args);
hipError_t launch_bin_f64(hipStream_t st, int S, int NW, bool mass, const BinArgs<double>& a);
hipError_t launch_bin_f32(hipStream_t st, int S, int NW, bool mass, const BinArgs<float>& a);
bool bin_shape_available(int precision, int S, int NW);
// Copy every chain's current state (selected by state_sel) into h_dst.
hipError_t launch_gather_state(hipStream_t st, const ChainDesc* chains, int32_t n_chains,
                               int32_t max_T, const int32_t* state_sel, const void* h_a,
                               const void* h_b, const double* shift, void* h_dst, int precision);
// Add every chain's current state to batch_sum (and its square to sq_sum):
// the FP32 per-batch accumulators of the per-kernel sweep path.
hipError_t launch_accumulate(hipStream_t st, const ChainDesc* chains, int32_t n_chains,
                             int32_t max_T, const int32_t* state_sel, const void* h_a,
                             const void* h_b, const double* shift, float* batch_sum,
                             float* sq_sum, int precision);
// batch_sum[i] += acc_sum[i], sq_sum[i] += acc_sq[i] (each may be nullptr),
// then acc_sum = acc_sq = 0, for i < n.
hipError_t launch_flush(hipStream_t st, int64_t n, float* acc_sum, float* acc_sq,
                        double* batch_sum, double* sq_sum);
// Leave every chain's current state (including a pending level shift) in h_a;
// clear state_sel and the shifts.
hipError_t launch_settle(hipStream_t st, const ChainDesc* chains, int32_t n_chains, int32_t max_T,
                         int32_t* state_sel, void* h_a, const void* h_b, double* shift,
                         int precision);
hipError_t launch_stats(hipStream_t st, const TileDesc* tiles, int32_t n_tiles,
                        const ChainDesc* chains, const rsv_theta* theta, const void* h_a,
                        const void* h_b, const int32_t* state_sel, const double* shift,
                        const double* y2_d, const double* lrv_d, double* partials,
                        double* chain_edge, int precision);
// sqrt(m_t) from ln m_t (once, at init), as an FP64 table (precision
// RSV_F64) or an FP32 table (RSV_F32_MIXED).
hipError_t launch_mass_table(hipStream_t st, const float* log_mass, int64_t n, void* sqrt_m,
                             int precision);
hipError_t launch_momenta(hipStream_t st, const ChainDesc* chains, int32_t n_chains,
                          int32_t max_T, const void* mass_sqrt, int precision, uint64_t seed,
                          uint64_t sweep, double* p_out);
hipError_t launch_count_nonfinite(hipStream_t st, const void* h, int64_t n, int precision,
                                  uint32_t* counter);

}  // namespace rsv
