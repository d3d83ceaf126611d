// rsv_bin_f64.hip -- instantiations of the resident sweep kernel (rsv_bin.h) for
// FP64: tiles of one and of four wavefronts.
#include "rsv_bin.h"

namespace rsv {

hipError_t launch_bin_f64(hipStream_t st, int S, int NW, bool mass, const BinArgs<double>& a) {
    if (S == 4 && NW == 1) return launch_bin_shape<double, 4, 1>(st, mass, a);
    if (S == 8 && NW == 1) return launch_bin_shape<double, 8, 1>(st, mass, a);
    if (S == 4 && NW == 4) return launch_bin_shape<double, 4, 4>(st, mass, a);
    if (S == 8 && NW == 4) return launch_bin_shape<double, 8, 4>(st, mass, a);
    return hipErrorInvalidValue;
}

}  // namespace rsv
