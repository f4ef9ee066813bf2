// Detection kernels for inputs padded to 2M = 128 (instantiation unit).
#include "detect_kernel.h"

namespace apsm {
namespace det {
hipError_t launch_detect_m128(const DetectArgs& a, hipStream_t stream) { return launch_m<128>(a, stream); }
}  // namespace det
}  // namespace apsm
