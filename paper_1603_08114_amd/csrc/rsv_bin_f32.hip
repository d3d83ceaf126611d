// rsv_bin_f32.hip -- instantiations of the resident sweep kernel (rsv_bin.h) for
// FP32-mixed: tiles of one and of four wavefronts.
#include "rsv_bin.h"

namespace rsv {

hipError_t launch_bin_f32(hipStream_t st, int S, int NW, bool mass, const BinArgs<float>& a) {
    if (S == 8 && NW == 1) return launch_bin_shape<float, 8, 1>(st, mass, a);
    if (S == 16 && NW == 1) return launch_bin_shape<float, 16, 1>(st, mass, a);
    if (S == 8 && NW == 4) return launch_bin_shape<float, 8, 4>(st, mass, a);
    if (S == 16 && NW == 4) return launch_bin_shape<float, 16, 4>(st, mass, a);
    return hipErrorInvalidValue;
}

}  // namespace rsv
