// Step kernels with double particle state and double in-tile sums.
#include "m2m_step.h"

namespace m2m {

hipError_t launch_step_f64(int block, int kin, const FitDev* fits, const Tile* tiles,
                        const FitDev* one, int n_tiles, size_t lds, int32_t mode,
                        hipStream_t s) {
    if (block == 256) return launch_step_kin<double, double, 256>(kin, fits, tiles, one, n_tiles, lds, mode, s);
    return hipErrorInvalidValue;
}

}  // namespace m2m
