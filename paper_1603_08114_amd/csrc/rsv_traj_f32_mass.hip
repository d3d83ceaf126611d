// rsv_traj_f32_mass.hip -- instantiations of k_traj_mass for FP32-mixed
// with a diagonal mass, one per compiled tile shape.
#include "rsv_traj.h"

namespace rsv {

namespace {
template <int S, int NW>
hipError_t launch_shape(hipStream_t st, const TrajArgs<float>& a) {
    if (a.n_list <= 0) return hipSuccess;
    constexpr int per_block = NW == 1 ? 4 : 1;
    const dim3 grid((a.n_list + per_block - 1) / per_block), block(NW == 1 ? 256 : 64 * NW);
    if (a.terms & RSV_TERM_RETURN)
        hipLaunchKernelGGL((k_traj_mass<float, S, NW, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_traj_mass<float, S, NW, false>), grid, block, 0, st, a);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_traj_f32_mass(hipStream_t st, int S, int NW, const TrajArgs<float>& a) {
    if (S == 8 && NW == 1) return launch_shape<8, 1>(st, a);
    if (S == 8 && NW == 2) return launch_shape<8, 2>(st, a);
    if (S == 8 && NW == 4) return launch_shape<8, 4>(st, a);
    if (S == 8 && NW == 8) return launch_shape<8, 8>(st, a);
    if (S == 16 && NW == 1) return launch_shape<16, 1>(st, a);
    if (S == 16 && NW == 2) return launch_shape<16, 2>(st, a);
    if (S == 16 && NW == 4) return launch_shape<16, 4>(st, a);
    return hipErrorInvalidValue;
}

}  // namespace rsv
