// Dispatch of apsm_detect and of model packing.  Two detection kernels:
// split-FP16 with the coefficient sums on VALU (2M <= 64 and K <= 8) and
// the two-contraction kernel with them on the matrix cores (every shape).
// Shapes both hold ("dual") carry both packed images, so either kernel can
// run on any model; the one used is the tuned choice for the shape class,
// else the measured default (matrix-core coefficients from 2M > 16 on).
#include "detect_f16.h"
#include "detect_wide.h"

namespace apsm {

namespace {
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

bool detect_dual(int M2, int K) { return f16::supported(M2, K); }

int detect_default_kernel(int M2, int K) {
  if (!detect_dual(M2, K)) return kDetectWide;
  return f16::m2p_f16(M2) >= 32 ? kDetectWide : kDetectF16;
}

size_t wide_offset(int M2, int K, int cap) {
  return detect_dual(M2, K) ? align256(f16::packed_bytes(M2, K, cap)) : 0;
}

size_t packed_model_bytes(int M2, int K, int cap) { return wide_offset(M2, K, cap) + wide::packed_bytes(M2, cap); }

hipError_t launch_pack_model(const float* dict, const float* alpha, const float* w, const int32_t* state, int cap,
                             int M2, int K, void* packed, hipStream_t stream) {
  unsigned char* out = static_cast<unsigned char*>(packed);
  if (detect_dual(M2, K)) {
    hipError_t e = f16::launch_pack(dict, alpha, state, cap, M2, K, out, stream);
    if (e != hipSuccess) return e;
  }
  return wide::launch_pack(dict, alpha, w, state, cap, M2, K, out + wide_offset(M2, K, cap), stream);
}

hipError_t launch_pack_model_batch(const PackJob* jobs, int n, int max_cap, hipStream_t stream) {
  return f16::launch_pack_batch(jobs, n, max_cap, stream);
}

hipError_t launch_pack_wide_batch(const PackJob* jobs, int n, int max_threads, hipStream_t stream) {
  return wide::launch_pack_batch(jobs, n, max_threads, stream);
}

hipError_t launch_detect_with(const DetectArgs& a, int kernel, hipStream_t stream) {
  if (a.M2 > APSM_MAX_M2) return hipErrorInvalidValue;
  if (kernel == kDetectF16 && f16::supported(a.M2, a.K)) {
    const int M2P = f16::m2p_f16(a.M2);
    if (M2P == 16) return f16::launch_detect_f16_m16(a, a.packed, stream);
    if (M2P == 32) return f16::launch_detect_f16_m32(a, a.packed, stream);
    return f16::launch_detect_f16_m64(a, a.packed, stream);
  }
  DetectArgs b = a;
  b.packed = a.packed + wide_offset(a.M2, a.K, a.cap);
  return wide::launch_detect(b, stream);
}

hipError_t launch_detect(const DetectArgs& a, hipStream_t stream) {
  return launch_detect_with(a, detect_kernel_for(a.M2, a.K), stream);
}

}  // namespace apsm
