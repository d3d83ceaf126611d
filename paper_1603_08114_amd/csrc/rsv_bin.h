// rsv_bin.h -- resident sweeps: every sweep of a call in one launch.
//
// Paper: T. Takaishi, arXiv:1603.08114.  Sec. 3: one HMC sweep is a momentum
// refresh, the leapfrog trajectory of eqs. (6)-(8) and the Metropolis test,
// here followed by the theta update; Sec. 5 maps each leapfrog equation to
// its own kernel over all sites (eqs. (9)-(11)).  The one-launch-per-kernel
// path of this library runs two kernels per sweep (the tiles of every chain,
// then one finalize block per chain).  Here a block owns a bin of whole
// chains for all sweeps of a call: per sweep it integrates the bin's tiles
// (the trajectory kernel's own tile code, in rounds of one tile per group of
// NW wavefronts), meets one barrier, lets one wavefront per chain run that
// chain's finalize (dH total, Metropolis test, theta update), meets a second
// barrier and goes on with the next sweep.  No kernel boundary and no
// finalize launch separate the sweeps, and while one block runs its
// finalize the other blocks on the compute unit keep integrating.
//
// The host packs chains into bins (whole chains, largest first, best fit);
// tiles, partial sums and the finalize are those of the per-kernel path, so
// the results equal it bit for bit.
#pragma once

#include "rsv_traj.h"

namespace rsv {

namespace {

// The finalize of one chain by one wavefront, as a call: its FP64 draws and
// Gibbs algebra then do not add to the registers of the tile loop.
__device__ __noinline__ void bin_finalize(const FinalizeArgs& F, int c, Comp (&part)[1][kNQ],
                                          ThetaDraws& draws, int lane) {
    finalize_chain<kWave>(F, c, part, draws, lane);
}

template <typename R, int S, int NW, bool MASS, bool RET>
__global__ __launch_bounds__(NW == 1 ? 256 : 64 * NW) void k_bin(BinArgs<R> B) {
    // tiles integrated at once by a block: four single-wavefront tiles, or
    // one tile of NW wavefronts (the per-kernel launch's grouping)
    constexpr int kTPB = NW == 1 ? 4 : 1;
    constexpr int kWaves = NW == 1 ? 4 : NW;
    using St = Stage<R, S, NW, kTPB>;
    __shared__ TileShared<R, NW> tsh[kTPB];
    __shared__ R stage_all[kTPB][St::n];
    __shared__ Comp part[kWaves][1][kNQ];
    __shared__ ThetaDraws draws[kWaves];

    const int lane = threadIdx.x & (kWave - 1);
    const int wb = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int grp = wb / NW;   // tile group of this wavefront
    const int wv = wb % NW;    // wavefront within its tile
    const BinDesc bd = B.bins[blockIdx.x];
    const int32_t* tiles = B.bin_tiles + bd.tile_first;
    const int32_t* chains = B.bin_chains + bd.chain_first;
    const int bl = B.batch_len;

    // batch-sum flush of a tile's exact sites (the per-kernel flush pass)
    auto flush_tile = [&](int tile_id, int64_t row) {
        const TileDesc td = B.traj.tiles[tile_id];
        const int64_t h_off = B.traj.chains[td.chain].h_off;
        for (int t = td.a + wv * kWave + lane; t < td.b; t += NW * kWave) {
            const int64_t idx = h_off + t;
            if (B.batch_sum) B.batch_sum[row * B.n_state + idx] += static_cast<double>(B.acc_sum[idx]);
            if (B.sq_sum) B.sq_sum[idx] += static_cast<double>(B.acc_sq[idx]);
            B.acc_sum[idx] = 0.0f;
            B.acc_sq[idx] = 0.0f;
        }
    };
    // value of the current state at the exact sites of a tile, for f(idx, v)
    auto for_state = [&](int tile_id, auto f) {
        const TileDesc td = B.traj.tiles[tile_id];
        const ChainDesc cd = B.traj.chains[td.chain];
        const R* src = (B.traj.state_sel[td.chain] ? B.traj.h_b : B.traj.h_a) + cd.h_off;
        const double sft = B.fin.shift ? B.fin.shift[td.chain] : 0.0;
        for (int t = td.a + wv * kWave + lane; t < td.b; t += NW * kWave)
            f(cd.h_off + t, state_at(src, t, sft));
    };

    for (int i = 0; i < B.n_sweeps; ++i) {
        TrajArgs<R> A = B.traj;
        A.sweep = B.first_sweep + static_cast<uint64_t>(i);
        // the trajectory of sweep i adds the state it starts from (the one
        // after sweep i - 1) to the FP32 batch sums
        const bool add = B.acc_sum && i > 0;
        A.acc_sum = add ? B.acc_sum : nullptr;
        A.acc_sq = add ? B.acc_sq : nullptr;
        for (int s = grp; s < bd.tile_count; s += kTPB) {
            const int tile_id = tiles[s];
            if (A.tiles[tile_id].edge)
                traj_tile<R, S, NW, MASS, true, RET, St::on>(A, tsh[grp], tile_id, wv, lane,
                                                             stage_all[grp]);
            else
                traj_tile<R, S, NW, MASS, false, RET, St::on>(A, tsh[grp], tile_id, wv, lane,
                                                              stage_all[grp]);
        }
        __syncthreads();
        // the batch that ended with the state after sweep i - 1 (after the
        // barrier: a lane flushes sites that other lanes accumulated)
        if (add && (i - 1) % bl == bl - 1)
            for (int s = grp; s < bd.tile_count; s += kTPB) flush_tile(tiles[s], (i - 1) / bl);

        FinalizeArgs F = B.fin;
        F.sweep = A.sweep;
        const int64_t ofs = static_cast<int64_t>(i) * F.n_chains;
        F.delta_h_out = B.dh_trace ? B.dh_trace + ofs : nullptr;
        F.accepted_out = B.acc_trace ? B.acc_trace + ofs : nullptr;
        F.theta_trace = B.theta_trace ? B.theta_trace + ofs : nullptr;
        for (int j = wb; j < bd.chain_count; j += kWaves)
            bin_finalize(F, chains[j], part[wb], draws[wb], lane);
        __syncthreads();

        if (B.h_trace) {
            R* ht = B.h_trace + static_cast<int64_t>(i) * B.n_state;
            for (int s = grp; s < bd.tile_count; s += kTPB)
                for_state(tiles[s], [&](int64_t idx, R v) { ht[idx] = v; });
        }
    }
    // the state after the last sweep, and its batch
    if (B.acc_sum && B.n_sweeps > 0) {
        for (int s = grp; s < bd.tile_count; s += kTPB) {
            for_state(tiles[s], [&](int64_t idx, R v) {
                const float vf = static_cast<float>(v);
                B.acc_sum[idx] += vf;
                B.acc_sq[idx] = __builtin_fmaf(vf, vf, B.acc_sq[idx]);
            });
            flush_tile(tiles[s], (B.n_sweeps - 1) / bl);
        }
    }
}

template <typename R, int S, int NW>
hipError_t launch_bin_shape(hipStream_t st, bool mass, const BinArgs<R>& a) {
    if (a.n_bins <= 0) return hipSuccess;
    const dim3 grid(a.n_bins), block(NW == 1 ? 256 : 64 * NW);
    const bool ret = (a.traj.terms & RSV_TERM_RETURN) != 0;
    if (mass) {
        if (ret) hipLaunchKernelGGL((k_bin<R, S, NW, true, true>), grid, block, 0, st, a);
        else     hipLaunchKernelGGL((k_bin<R, S, NW, true, false>), grid, block, 0, st, a);
    } else {
        if (ret) hipLaunchKernelGGL((k_bin<R, S, NW, false, true>), grid, block, 0, st, a);
        else     hipLaunchKernelGGL((k_bin<R, S, NW, false, false>), grid, block, 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace

}  // namespace rsv
