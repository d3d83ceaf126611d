// rsv_resident.hip -- instantiations of the resident sweep kernels (every
// sweep of a call in one launch, one block per chain).
#include "rsv_traj.h"

namespace rsv {

namespace {

template <typename R, int S>
hipError_t launch_resident_t(hipStream_t st, bool mass, bool ret, const ResidentArgs<R>& a) {
    const dim3 grid(a.fin.n_chains), block(256);
    if (ret) {
        if (mass) hipLaunchKernelGGL((k_resident<R, S, true, true>), grid, block, 0, st, a);
        else      hipLaunchKernelGGL((k_resident<R, S, false, true>), grid, block, 0, st, a);
    } else {
        if (mass) hipLaunchKernelGGL((k_resident<R, S, true, false>), grid, block, 0, st, a);
        else      hipLaunchKernelGGL((k_resident<R, S, false, false>), grid, block, 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_resident(hipStream_t st, int precision, int S, bool mass, const void* args) {
    if (precision == RSV_F64) {
        const auto& a = *static_cast<const ResidentArgs<double>*>(args);
        const bool ret = (a.traj.terms & RSV_TERM_RETURN) != 0;
        if (S == 4) return launch_resident_t<double, 4>(st, mass, ret, a);
        if (S == 8) return launch_resident_t<double, 8>(st, mass, ret, a);
    } else {
        const auto& a = *static_cast<const ResidentArgs<float>*>(args);
        const bool ret = (a.traj.terms & RSV_TERM_RETURN) != 0;
        if (S == 8) return launch_resident_t<float, 8>(st, mass, ret, a);
        if (S == 16) return launch_resident_t<float, 16>(st, mass, ret, a);
    }
    return hipErrorInvalidValue;
}


}  // namespace rsv
