// tiles_r6.hip -- T-step LDS tile kernels of 48 rows (8 waves x 6 rows).
#include "tiles_impl.h"

namespace rdc {
template hipError_t launch_tiles<6>(const StepArgs<float>& a, int T, hipStream_t s);
template hipError_t launch_tiles<6>(const StepArgs<double>& a, int T, hipStream_t s);
}  // namespace rdc
