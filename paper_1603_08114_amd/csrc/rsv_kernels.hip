// rsv_kernels.hip -- HIP kernels (gfx950) of the RSV-model HMC update:
// finalize (dH reduction, Metropolis test, theta update), statistics, state
// movement, batch-means accumulation, data preparation and validation, and
// the dispatch of the trajectory kernels (instantiated in rsv_traj_*.hip).
//
// Paper: T. Takaishi, arXiv:1603.08114 (Sec. 3: HMC; Sec. 5: GPU mapping).
#include "rsv_traj.h"

namespace rsv {

namespace {


// ---------------------------------------------------------------------------
// State movement between the two buffers (one chain per grid row).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_gather_state(const ChainDesc* chains,
                                                      const int32_t* state_sel, const R* h_a,
                                                      const R* h_b, const double* shift,
                                                      R* h_dst) {
    const int c = blockIdx.y;
    const ChainDesc cd = chains[c];
    const R* src = (state_sel[c] ? h_b : h_a) + cd.h_off;
    const double sft = shift ? shift[c] : 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < cd.T;
         t += stride)
        h_dst[cd.h_off + t] = state_at(src, t, sft);
}

template <typename R>
__global__ __launch_bounds__(256) void k_accumulate(const ChainDesc* chains,
                                                    const int32_t* state_sel, const R* h_a,
                                                    const R* h_b, const double* shift,
                                                    float* batch_sum, float* sq_sum) {
    const int c = blockIdx.y;
    const ChainDesc cd = chains[c];
    const R* src = (state_sel[c] ? h_b : h_a) + cd.h_off;
    const double sft = shift ? shift[c] : 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < cd.T;
         t += stride) {
        const int64_t i = cd.h_off + t;
        const float v = static_cast<float>(state_at(src, t, sft));
        if (batch_sum) batch_sum[i] += v;
        if (sq_sum) sq_sum[i] = __builtin_fmaf(v, v, sq_sum[i]);
    }
}

__global__ __launch_bounds__(256) void k_flush(int64_t n, float* acc_sum, float* acc_sq,
                                               double* batch_sum, double* sq_sum) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += stride) {
        if (batch_sum) batch_sum[i] += static_cast<double>(acc_sum[i]);
        if (sq_sum) sq_sum[i] += static_cast<double>(acc_sq[i]);
        acc_sum[i] = 0.0f;
        acc_sq[i] = 0.0f;
    }
}

// Writes the current state (buffer h_b when selected, plus the pending shift)
// into h_a.  Chains already in h_a with no shift are left alone.
template <typename R>
__global__ __launch_bounds__(256) void k_settle(const ChainDesc* chains, const int32_t* state_sel,
                                                R* h_a, const R* h_b, const double* shift) {
    const int c = blockIdx.y;
    const double sft = shift ? shift[c] : 0.0;
    if (!state_sel[c] && sft == 0.0) return;
    const ChainDesc cd = chains[c];
    const R* src = (state_sel[c] ? h_b : h_a) + cd.h_off;
    R* dst = h_a + cd.h_off;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < cd.T;
         t += stride)
        dst[t] = state_at(src, t, sft);
}

__global__ void k_clear_sel(int32_t* state_sel, double* shift, int32_t n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        state_sel[i] = 0;
        if (shift) shift[i] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Diagonal mass table: sqrt(m_t) from the caller's ln m_t, in the precision
// of the state (FP64, or FP32 on the mixed path: 4 bytes per site).  The
// trajectory kernel forms 1/m_t from it; the stored value defines the mass.
// A site whose ln m_t is not finite, or whose sqrt(m_t) or 1/m_t would
// overflow or vanish in the state's precision, takes the identity mass
// m_t = 1 (any fixed positive mass keeps the chain exact).
// ---------------------------------------------------------------------------
template <typename M>
__global__ __launch_bounds__(256) void k_mass_table(const float* log_mass, int64_t n,
                                                    M* sqrt_m) {
    // |ln m| <= 80 keeps sqrt(m) and 1/m normal in FP32
    constexpr double kMaxLogMass = 80.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
         t += stride) {
        const double l = static_cast<double>(log_mass[t]);
        const bool ok = l >= -kMaxLogMass && l <= kMaxLogMass;  // false for NaN
        sqrt_m[t] = ok ? static_cast<M>(exp_fast(0.5 * l)) : M(1);
    }
}

// ---------------------------------------------------------------------------
// Standalone momentum refresh (same streams as the trajectory kernel).
// ---------------------------------------------------------------------------
template <typename M>
__global__ __launch_bounds__(256) void k_momenta(const ChainDesc* chains, const M* mass_sqrt,
                                                 uint64_t seed, uint64_t sweep, double* p_out) {
    constexpr int NB = kMomentumBlock<M>;
    const int c = blockIdx.y;
    const ChainDesc cd = chains[c];
    const int n_blocks = (cd.T + NB - 1) / NB;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n_blocks;
         g += gridDim.x * blockDim.x) {
        M z[NB];
        momentum_normals<M>(seed, static_cast<uint64_t>(g), sweep, static_cast<uint64_t>(c), z);
        for (int q = 0; q < NB; ++q) {
            const int t = NB * g + q;
            if (t >= cd.T) break;
            const M pm = mass_sqrt ? z[q] * mass_sqrt[cd.d_off + t] : z[q];
            p_out[cd.h_off + t] = static_cast<double>(pm);
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


}  // namespace

// Tile shapes compiled for each precision: (sites per lane, wavefronts per
// tile); the first is the default.
bool traj_shape_available(int precision, int S, int NW) {
    const bool nw = NW == 1 || NW == 2 || NW == 4 || NW == 8;
    if (precision == RSV_F64) return nw && (S == 4 || S == 8);
    return (S == 8 && nw) || (S == 16 && (NW == 1 || NW == 2 || NW == 4));
}
// Shapes of the resident kernel (rsv_bin.h): single-wavefront tiles and tiles
// of four wavefronts.
bool bin_shape_available(int precision, int S, int NW) {
    if (precision == RSV_F64) return (S == 4 || S == 8) && (NW == 1 || NW == 4);
    return (S == 8 || S == 16) && (NW == 1 || NW == 4);
}

hipError_t launch_bin(hipStream_t st, int precision, int S, int NW, bool mass, const void* args) {
    if (precision == RSV_F64)
        return launch_bin_f64(st, S, NW, mass, *static_cast<const BinArgs<double>*>(args));
    return launch_bin_f32(st, S, NW, mass, *static_cast<const BinArgs<float>*>(args));
}
void traj_default_shape(int precision, int* S, int* NW) {
    // fastest measured on a long series: FP64 (4, 4) (fewer registers, five
    // waves per SIMD), FP32 (8, 4)
    *S = precision == RSV_F64 ? 4 : 8;
    *NW = 4;
}

hipError_t launch_traj(hipStream_t st, int precision, int S, int NW, bool mass,
                       const void* args) {
    if (precision == RSV_F64) {
        const auto& a = *static_cast<const TrajArgs<double>*>(args);
        return mass ? launch_traj_f64_mass(st, S, NW, a) : launch_traj_f64(st, S, NW, a);
    }
    const auto& a = *static_cast<const TrajArgs<float>*>(args);
    return mass ? launch_traj_f32_mass(st, S, NW, a) : launch_traj_f32(st, S, NW, a);
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

hipError_t launch_finalize(hipStream_t st, const FinalizeArgs& a, int32_t max_tiles_per_chain) {
    // chains of at most 128 tiles: one wavefront each; longer chains: the
    // split finalize, one block per slice of kSliceTiles tiles
    if (max_tiles_per_chain <= 128 || !a.slices) {
        hipLaunchKernelGGL(k_finalize, dim3(a.n_chains), dim3(2 * kWave), 0, st, a);
    } else {
        const int n_sl = (max_tiles_per_chain + kSliceTiles - 1) / kSliceTiles;
        hipLaunchKernelGGL(k_finalize_split<256>, dim3(n_sl, a.n_chains), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_gather_state(hipStream_t st, const ChainDesc* chains, int32_t n_chains,
                               int32_t max_T, const int32_t* state_sel, const void* h_a,
                               const void* h_b, const double* shift, void* h_dst, int precision) {
    const dim3 g(grid_for(max_T, 256, 1024), n_chains), b(256);
    if (precision == RSV_F64)
        hipLaunchKernelGGL(k_gather_state<double>, g, b, 0, st, chains, state_sel,
                           static_cast<const double*>(h_a), static_cast<const double*>(h_b),
                           shift, static_cast<double*>(h_dst));
    else
        hipLaunchKernelGGL(k_gather_state<float>, g, b, 0, st, chains, state_sel,
                           static_cast<const float*>(h_a), static_cast<const float*>(h_b),
                           shift, static_cast<float*>(h_dst));
    return hipGetLastError();
}

hipError_t launch_flush(hipStream_t st, int64_t n, float* acc_sum, float* acc_sq,
                        double* batch_sum, double* sq_sum) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flush, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, n, acc_sum,
                       acc_sq, batch_sum, sq_sum);
    return hipGetLastError();
}

hipError_t launch_accumulate(hipStream_t st, const ChainDesc* chains, int32_t n_chains,
                             int32_t max_T, const int32_t* state_sel, const void* h_a,
                             const void* h_b, const double* shift, float* batch_sum,
                             float* sq_sum, int precision) {
    const dim3 g(grid_for(max_T, 256, 1024), n_chains), b(256);
    if (precision == RSV_F64)
        hipLaunchKernelGGL(k_accumulate<double>, g, b, 0, st, chains, state_sel,
                           static_cast<const double*>(h_a), static_cast<const double*>(h_b),
                           shift, batch_sum, sq_sum);
    else
        hipLaunchKernelGGL(k_accumulate<float>, g, b, 0, st, chains, state_sel,
                           static_cast<const float*>(h_a), static_cast<const float*>(h_b),
                           shift, batch_sum, sq_sum);
    return hipGetLastError();
}

hipError_t launch_settle(hipStream_t st, const ChainDesc* chains, int32_t n_chains, int32_t max_T,
                         int32_t* state_sel, void* h_a, const void* h_b, double* shift,
                         int precision) {
    const dim3 g(grid_for(max_T, 256, 1024), n_chains), b(256);
    if (precision == RSV_F64)
        hipLaunchKernelGGL(k_settle<double>, g, b, 0, st, chains, state_sel,
                           static_cast<double*>(h_a), static_cast<const double*>(h_b), shift);
    else
        hipLaunchKernelGGL(k_settle<float>, g, b, 0, st, chains, state_sel,
                           static_cast<float*>(h_a), static_cast<const float*>(h_b), shift);
    hipLaunchKernelGGL(k_clear_sel, dim3((n_chains + 255) / 256), dim3(256), 0, st, state_sel,
                       shift, n_chains);
    return hipGetLastError();
}

hipError_t launch_stats(hipStream_t st, const TileDesc* tiles, int32_t n_tiles,
                        const ChainDesc* chains, const rsv_theta* theta, const void* h_a,
                        const void* h_b, const int32_t* state_sel, const double* shift,
                        const double* y2_d, const double* lrv_d, double* partials,
                        double* chain_edge, int precision) {
    const dim3 g((n_tiles + 3) / 4), b(256);
    if (precision == RSV_F64)
        hipLaunchKernelGGL(k_stats<double>, g, b, 0, st, tiles, n_tiles, chains, theta,
                           static_cast<const double*>(h_a), static_cast<const double*>(h_b),
                           state_sel, shift, y2_d, lrv_d, partials, chain_edge);
    else
        hipLaunchKernelGGL(k_stats<float>, g, b, 0, st, tiles, n_tiles, chains, theta,
                           static_cast<const float*>(h_a), static_cast<const float*>(h_b),
                           state_sel, shift, y2_d, lrv_d, partials, chain_edge);
    return hipGetLastError();
}

hipError_t launch_mass_table(hipStream_t st, const float* log_mass, int64_t n, void* sqrt_m,
                             int precision) {
    if (n <= 0) return hipSuccess;
    const dim3 g(grid_for(n, 256, 4096)), b(256);
    if (precision == RSV_F64)
        hipLaunchKernelGGL(k_mass_table<double>, g, b, 0, st, log_mass, n,
                           static_cast<double*>(sqrt_m));
    else
        hipLaunchKernelGGL(k_mass_table<float>, g, b, 0, st, log_mass, n,
                           static_cast<float*>(sqrt_m));
    return hipGetLastError();
}

hipError_t launch_momenta(hipStream_t st, const ChainDesc* chains, int32_t n_chains,
                          int32_t max_T, const void* mass_sqrt, int precision, uint64_t seed,
                          uint64_t sweep, double* p_out) {
    const dim3 g(grid_for((max_T + 3) / 4, 256, 1024), n_chains), b(256);
    if (precision == RSV_F64)
        hipLaunchKernelGGL(k_momenta<double>, g, b, 0, st, chains,
                           static_cast<const double*>(mass_sqrt), seed, sweep, p_out);
    else
        hipLaunchKernelGGL(k_momenta<float>, g, b, 0, st, chains,
                           static_cast<const float*>(mass_sqrt), seed, sweep, p_out);
    return hipGetLastError();
}

}  // namespace rsv
