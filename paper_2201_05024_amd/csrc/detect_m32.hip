// Detection kernels for inputs padded to 2M = 32 (instantiation unit).
#include "detect_kernel.h"

namespace apsm {
namespace det {
hipError_t launch_detect_m32(const DetectArgs& a, hipStream_t stream) { return launch_m<32>(a, stream); }
}  // namespace det
}  // namespace apsm
