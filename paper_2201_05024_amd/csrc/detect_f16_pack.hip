// Packing of a model for the split-FP16 detection kernels: the dictionary,
// scaled by one power of two and split into FP16 hi/lo parts, the
// coefficients and the squared norms, laid out per chunk so that detection
// stages them with plain 16-byte copies.  Independent of sigma^2.
#include "detect_f16.h"

namespace apsm {
namespace f16 {
namespace {

// One workgroup: header[0] = exponent placing max |d| in [2^12, 2^13).
__global__ __launch_bounds__(1024) void dict_scale_kernel(const float* dict, const int32_t* state, int cap,
                                                          int M2, int* header) {
  int D = state[0];
  D = D < 0 ? 0 : (D > cap ? cap : D);
  float m = 0.0f;
  const size_t n = (size_t)D * M2;
  for (size_t i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, fabsf(dict[i]));
  __shared__ float red[1024];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    header[0] = scale_exp(red[0]);
    header[1] = D;
  }
}

template <int M2P, int K>
__global__ __launch_bounds__(256) void pack_kernel(const float* dict, const float* alpha, const int32_t* state,
                                                   int cap, int M2, unsigned char* out) {
  using G = Geo<M2P, K>;
  const int cap64 = cap64_of(cap);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap64) return;
  int D = state[0];
  D = D < 0 ? 0 : (D > cap ? cap : D);
  const bool valid = i < D;
  const float sc = ldexpf(1.0f, reinterpret_cast<const int*>(out)[0]);
  _Float16* row = reinterpret_cast<_Float16*>(out + kHeader) + (size_t)i * G::BSTR;
  float n = 0.0f;
#pragma unroll 4
  for (int m = 0; m < M2P; ++m) {
    const float d = (valid && m < M2) ? dict[(size_t)i * M2 + m] : 0.0f;
    n = fmaf(d, d, n);
    _Float16 hi, lo;
    split_f16(d * sc, hi, lo);
    row[m] = hi;
    row[M2P + m] = lo;
  }
  for (int v = 0; v < 8; ++v) row[2 * M2P + v] = (_Float16)0.0f;
  float* co = reinterpret_cast<float*>(out + kHeader + (size_t)cap64 * G::ROW_B) + (size_t)i * G::CSTR;
  for (int k = 0; k < G::K4; ++k) co[k] = (valid && k < K) ? alpha[(size_t)i * K + k] : 0.0f;
  co[G::K4] = n;
  co[G::K4 + 1] = co[G::K4 + 2] = co[G::K4 + 3] = 0.0f;
}

template <int M2P, int K>
hipError_t pack_mk(const float* dict, const float* alpha, const int32_t* state, int cap, int M2,
                   unsigned char* packed, hipStream_t stream) {
  hipLaunchKernelGGL(dict_scale_kernel, dim3(1), dim3(1024), 0, stream, dict, state, cap, M2,
                     reinterpret_cast<int*>(packed));
  const int cap64 = cap64_of(cap);
  hipLaunchKernelGGL((pack_kernel<M2P, K>), dim3((cap64 + 255) / 256), dim3(256), 0, stream, dict, alpha,
                     state, cap, M2, packed);
  return hipGetLastError();
}

template <int M2P>
hipError_t pack_m(const float* dict, const float* alpha, const int32_t* state, int cap, int M2, int K,
                  unsigned char* packed, hipStream_t stream) {
  switch (K) {
    case 1: return pack_mk<M2P, 1>(dict, alpha, state, cap, M2, packed, stream);
    case 2: return pack_mk<M2P, 2>(dict, alpha, state, cap, M2, packed, stream);
    case 3: return pack_mk<M2P, 3>(dict, alpha, state, cap, M2, packed, stream);
    case 4: return pack_mk<M2P, 4>(dict, alpha, state, cap, M2, packed, stream);
    case 5: return pack_mk<M2P, 5>(dict, alpha, state, cap, M2, packed, stream);
    case 6: return pack_mk<M2P, 6>(dict, alpha, state, cap, M2, packed, stream);
    case 7: return pack_mk<M2P, 7>(dict, alpha, state, cap, M2, packed, stream);
    case 8: return pack_mk<M2P, 8>(dict, alpha, state, cap, M2, packed, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_pack(const float* dict, const float* alpha, const int32_t* state, int cap, int M2, int K,
                       unsigned char* packed, hipStream_t stream) {
  if (!supported(M2, K)) return hipSuccess;      // shapes detected without a packed model
  const int M2P = pad16(M2);
  if (M2P == 16) return pack_m<16>(dict, alpha, state, cap, M2, K, packed, stream);
  if (M2P == 32) return pack_m<32>(dict, alpha, state, cap, M2, K, packed, stream);
  return pack_m<64>(dict, alpha, state, cap, M2, K, packed, stream);
}

}  // namespace f16
}  // namespace apsm
