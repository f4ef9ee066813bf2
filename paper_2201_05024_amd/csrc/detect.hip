// Dispatch of apsm_detect: split-FP16 MFMA kernels for 2M <= 64 and K <= 8
// (the common detector shapes), FP32 MFMA kernels for the others.
#include "detect_f16.h"
#include "detect_kernel.h"

namespace apsm {

size_t packed_model_bytes(int M2, int K, int cap) {
  return f16::supported(M2, K) ? f16::packed_bytes(M2, K, cap) : 0;
}

hipError_t launch_pack_model(const float* dict, const float* alpha, const int32_t* state, int cap, int M2,
                             int K, void* packed, hipStream_t stream) {
  return f16::launch_pack(dict, alpha, state, cap, M2, K, static_cast<unsigned char*>(packed), stream);
}

hipError_t launch_pack_model_batch(const PackJob* jobs, int n, int max_cap, hipStream_t stream) {
  return f16::launch_pack_batch(jobs, n, max_cap, stream);
}

hipError_t launch_detect(const DetectArgs& a, hipStream_t stream) {
  if (f16::supported(a.M2, a.K)) {
    const int M2P = f16::m2p_f16(a.M2);
    if (M2P == 16) return f16::launch_detect_f16_m16(a, a.packed, stream);
    if (M2P == 32) return f16::launch_detect_f16_m32(a, a.packed, stream);
    return f16::launch_detect_f16_m64(a, a.packed, stream);
  }
  if (a.M2 <= 16) return det::launch_detect_m16(a, stream);
  if (a.M2 <= 32) return det::launch_detect_m32(a, stream);
  if (a.M2 <= 64) return det::launch_detect_m64(a, stream);
  if (a.M2 <= 128) return det::launch_detect_m128(a, stream);
  return hipErrorInvalidValue;
}

}  // namespace apsm
