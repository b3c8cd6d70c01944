// tiles_r8.hip -- T-step LDS tile kernels of 64 rows (8 waves x 8 rows).
#include "tiles_impl.h"

namespace rdc {
template hipError_t launch_tiles<8>(const StepArgs<float>& a, int T, hipStream_t s);
template hipError_t launch_tiles<8>(const StepArgs<double>& a, int T, hipStream_t s);
}  // namespace rdc
