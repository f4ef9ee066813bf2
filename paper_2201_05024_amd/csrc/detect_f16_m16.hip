// Split-FP16 detection kernels for inputs padded to 2M = 16 (instantiation unit).
#include "detect_f16.h"

namespace apsm {
namespace f16 {

template <int K>
static hipError_t launch_k(const DetectArgs& a, const unsigned char* packed, hipStream_t stream) {
  const int per_block = kWaves * 16;
  const int blocks = (a.S + per_block - 1) / per_block;
  hipLaunchKernelGGL((detect_f16_kernel<16, K>), dim3(blocks), dim3(kThreads), 0, stream, a, packed);
  return hipGetLastError();
}

hipError_t launch_detect_f16_m16(const DetectArgs& a, const unsigned char* packed, hipStream_t stream) {
  switch (a.K) {
    case 1: return launch_k<1>(a, packed, stream);
    case 2: return launch_k<2>(a, packed, stream);
    case 3: return launch_k<3>(a, packed, stream);
    case 4: return launch_k<4>(a, packed, stream);
    case 5: return launch_k<5>(a, packed, stream);
    case 6: return launch_k<6>(a, packed, stream);
    case 7: return launch_k<7>(a, packed, stream);
    case 8: return launch_k<8>(a, packed, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace f16
}  // namespace apsm
