// tiles_r7.hip -- T-step LDS tile kernels of 56 rows (8 waves x 7 rows).
#include "tiles_impl.h"

namespace rdc {
template hipError_t launch_tiles<7>(const StepArgs<float>& a, int T, hipStream_t s);
template hipError_t launch_tiles<7>(const StepArgs<double>& a, int T, hipStream_t s);
}  // namespace rdc
