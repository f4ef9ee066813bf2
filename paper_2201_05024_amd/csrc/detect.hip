// Dispatch of apsm_detect to the kernel instance of the padded input dimension.
#include "detect_kernel.h"

namespace apsm {

hipError_t launch_detect(const DetectArgs& a, hipStream_t stream) {
  if (a.M2 <= 16) return det::launch_detect_m16(a, stream);
  if (a.M2 <= 32) return det::launch_detect_m32(a, stream);
  if (a.M2 <= 64) return det::launch_detect_m64(a, stream);
  if (a.M2 <= 128) return det::launch_detect_m128(a, stream);
  return hipErrorInvalidValue;
}

}  // namespace apsm
