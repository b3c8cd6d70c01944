// tiles_r10.hip -- T-step LDS tile kernels of 80 rows (8 waves x 10 rows).
#include "tiles_impl.h"

namespace rdc {
template hipError_t launch_tiles<10>(const StepArgs<float>& a, int T, hipStream_t s);
template hipError_t launch_tiles<10>(const StepArgs<double>& a, int T, hipStream_t s);
}  // namespace rdc
