// Packing of a model for the split-FP16 detection kernels: the dictionary,
// scaled by one power of two and split into FP16 hi/lo parts, the
// coefficients and the squared norms, laid out per chunk so that detection
// stages them with plain 16-byte copies.  Independent of sigma^2.
#include "detect_f16.h"

namespace apsm {
namespace f16 {
namespace {

// Global-memory view of a job pointer: accesses through it are global (not
// flat) instructions.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// One workgroup of 1024 threads: header[0] = exponent placing max |d| in
// [2^12, 2^13), header[1] = entries in use.
__device__ __forceinline__ void dict_scale_body(const float* dict, const int32_t* state, int cap, int M2,
                                                int* header, float* red) {
  int D = gmem(state)[0];
  D = D < 0 ? 0 : (D > cap ? cap : D);
  float m = 0.0f;
  for (int c = 0; c < M2; ++c)                      // component c of entries 0..D-1
    for (int i = threadIdx.x; i < D; i += blockDim.x) m = fmaxf(m, fabsf(gmem(dict)[(size_t)c * cap + i]));
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

__global__ __launch_bounds__(1024) void dict_scale_kernel(const float* dict, const int32_t* state, int cap,
                                                          int M2, int* header) {
  __shared__ float red[1024];
  dict_scale_body(dict, state, cap, M2, header, red);
}

// Row i of the packed model (one thread per row; rows up to cap_pad(cap)).
template <int M2P, int K>
__device__ __forceinline__ void pack_row(const float* dict, const float* alpha, const int32_t* state, int cap,
                                         int M2, unsigned char* out, int i) {
  using G = Geo<M2P, K>;
  const int capp = cap_pad(cap);
  if (i >= capp) return;
  int D = gmem(state)[0];
  D = D < 0 ? 0 : (D > cap ? cap : D);
  const bool valid = i < D;
  const float sc = ldexpf(1.0f, gmem(reinterpret_cast<const int*>(out))[0]);
  // The row (16-byte aligned: header and row stride are multiples of 16) is
  // assembled in registers, eight halves at a time, and written with
  // 16-byte stores.
  const auto row = gmem(reinterpret_cast<half8*>(out + kHeader + (size_t)i * G::ROW_B));
  float n = 0.0f;
#pragma unroll
  for (int m0 = 0; m0 < M2P; m0 += 8) {
    half8 hv, lv;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int m = m0 + v;
      const float d = (valid && m < M2) ? gmem(dict)[(size_t)m * cap + i] : 0.0f;
      n = fmaf(d, d, n);
      _Float16 hi, lo;
      split_f16(d * sc, hi, lo);
      hv[v] = hi;
      lv[v] = lo;
    }
    row[m0 / 8] = hv;
    row[(M2P + m0) / 8] = lv;
  }
  half8 zero8;
#pragma unroll
  for (int v = 0; v < 8; ++v) zero8[v] = (_Float16)0.0f;
  row[2 * M2P / 8] = zero8;
  const auto co = gmem(reinterpret_cast<floatx4*>(out + kHeader + (size_t)capp * G::ROW_B + (size_t)i * G::CSTR * 4));
#pragma unroll
  for (int q = 0; q < G::K4 / 4; ++q) {
    floatx4 c4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = 4 * q + v;
      c4[v] = (valid && k < K) ? gmem(alpha)[(size_t)i * K + k] : 0.0f;
    }
    co[q] = c4;
  }
  floatx4 tail = {n, 0.0f, 0.0f, 0.0f};
  co[G::K4 / 4] = tail;
}

template <int M2P, int K>
__global__ __launch_bounds__(256) void pack_kernel(const float* dict, const float* alpha, const int32_t* state,
                                                   int cap, int M2, unsigned char* out) {
  pack_row<M2P, K>(dict, alpha, state, cap, M2, out, blockIdx.x * blockDim.x + threadIdx.x);
}

// Batched packing: workgroup (x, y) packs rows 256 x .. 256 x + 255 of job y.
__global__ __launch_bounds__(1024) void dict_scale_batch_kernel(const PackJob* jobs) {
  __shared__ float red[1024];
  const PackJob j = jobs[blockIdx.x];
  dict_scale_body(j.dict, j.state, j.cap, j.M2, reinterpret_cast<int*>(j.packed), red);
}

__global__ __launch_bounds__(256) void pack_batch_kernel(const PackJob* jobs) {
  const PackJob j = jobs[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  switch (j.variant) {
#define APSM_PACK_CASE(M2P, K, id) \
  case id: pack_row<M2P, K>(j.dict, j.alpha, j.state, j.cap, j.M2, j.packed, i); break;
    APSM_PACK_CASE(16, 1, 0) APSM_PACK_CASE(16, 2, 1) APSM_PACK_CASE(16, 3, 2) APSM_PACK_CASE(16, 4, 3)
    APSM_PACK_CASE(16, 5, 4) APSM_PACK_CASE(16, 6, 5) APSM_PACK_CASE(16, 7, 6) APSM_PACK_CASE(16, 8, 7)
    APSM_PACK_CASE(32, 1, 8) APSM_PACK_CASE(32, 2, 9) APSM_PACK_CASE(32, 3, 10) APSM_PACK_CASE(32, 4, 11)
    APSM_PACK_CASE(32, 5, 12) APSM_PACK_CASE(32, 6, 13) APSM_PACK_CASE(32, 7, 14) APSM_PACK_CASE(32, 8, 15)
    APSM_PACK_CASE(64, 1, 16) APSM_PACK_CASE(64, 2, 17) APSM_PACK_CASE(64, 3, 18) APSM_PACK_CASE(64, 4, 19)
    APSM_PACK_CASE(64, 5, 20) APSM_PACK_CASE(64, 6, 21) APSM_PACK_CASE(64, 7, 22) APSM_PACK_CASE(64, 8, 23)
#undef APSM_PACK_CASE
    default: break;
  }
}

template <int M2P, int K>
hipError_t pack_mk(const float* dict, const float* alpha, const int32_t* state, int cap, int M2,
                   unsigned char* packed, hipStream_t stream) {
  hipLaunchKernelGGL(dict_scale_kernel, dim3(1), dim3(1024), 0, stream, dict, state, cap, M2,
                     reinterpret_cast<int*>(packed));
  const int capp = cap_pad(cap);
  hipLaunchKernelGGL((pack_kernel<M2P, K>), dim3((capp + 255) / 256), dim3(256), 0, stream, dict, alpha,
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

// The scale pass must finish before rows are packed (they read header[0]):
// two launches in stream order.
hipError_t launch_pack_batch(const PackJob* jobs, int n, int max_cap, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dict_scale_batch_kernel, dim3(n), dim3(1024), 0, stream, jobs);
  const int blocks = (cap_pad(max_cap) + 255) / 256;
  hipLaunchKernelGGL(pack_batch_kernel, dim3(blocks, n), dim3(256), 0, stream, jobs);
  return hipGetLastError();
}

hipError_t launch_pack(const float* dict, const float* alpha, const int32_t* state, int cap, int M2, int K,
                       unsigned char* packed, hipStream_t stream) {
  if (!supported(M2, K)) return hipSuccess;      // shapes detected without a packed model
  const int M2P = m2p_f16(M2);
  if (M2P == 16) return pack_m<16>(dict, alpha, state, cap, M2, K, packed, stream);
  if (M2P == 32) return pack_m<32>(dict, alpha, state, cap, M2, K, packed, stream);
  return pack_m<64>(dict, alpha, state, cap, M2, K, packed, stream);
}

}  // namespace f16
}  // namespace apsm
