// Dispatch of apsm_detect and of model packing: split-FP16 kernels with the
// coefficients on VALU for 2M <= 64 and K <= 8 (the common detector shapes),
// the two-contraction kernel (coefficients on the matrix cores) for every
// wider shape.
#include "detect_f16.h"
#include "detect_wide.h"

namespace apsm {

bool detect_is_wide(int M2, int K) { return !f16::supported(M2, K); }

size_t packed_model_bytes(int M2, int K, int cap) {
  return f16::supported(M2, K) ? f16::packed_bytes(M2, K, cap) : wide::packed_bytes(M2, cap);
}

hipError_t launch_pack_model(const float* dict, const float* alpha, const float* w, const int32_t* state, int cap,
                             int M2, int K, void* packed, hipStream_t stream) {
  unsigned char* out = static_cast<unsigned char*>(packed);
  if (f16::supported(M2, K)) return f16::launch_pack(dict, alpha, state, cap, M2, K, out, stream);
  return wide::launch_pack(dict, alpha, w, state, cap, M2, K, out, stream);
}

hipError_t launch_pack_model_batch(const PackJob* jobs, int n, int max_cap, hipStream_t stream) {
  return f16::launch_pack_batch(jobs, n, max_cap, stream);
}

hipError_t launch_pack_wide_batch(const PackJob* jobs, int n, int max_threads, hipStream_t stream) {
  return wide::launch_pack_batch(jobs, n, max_threads, stream);
}

hipError_t launch_detect(const DetectArgs& a, hipStream_t stream) {
  if (f16::supported(a.M2, a.K)) {
    const int M2P = f16::m2p_f16(a.M2);
    if (M2P == 16) return f16::launch_detect_f16_m16(a, a.packed, stream);
    if (M2P == 32) return f16::launch_detect_f16_m32(a, a.packed, stream);
    return f16::launch_detect_f16_m64(a, a.packed, stream);
  }
  if (a.M2 > APSM_MAX_M2) return hipErrorInvalidValue;
  return wide::launch_detect(a, stream);
}

}  // namespace apsm
