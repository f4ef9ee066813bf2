// Generic projection engine beyond the detector's hyperslabs (Sec. I and
// Sec. VI: the GPU design serves other projection-based methods in RKHSs):
// the projection onto the ball {f : ||f_k||_H <= radius} of the sum space
// (norm of Fact 1, Sec. II-B) and cyclic projections (POCS) that alternate
// the windowed parallel projections of a training block with it.  The set
// kinds of the training samples (hyperplanes, halfspaces) live in the
// training kernel.
//
// Norm of user k's filter f_k(x) = w_k . x + sum_i alpha[i][k] kappa_G(d_i, x):
//   ||f_k||^2 = ||w_k||^2 / wL + sum_i alpha[i][k] fG_k(d_i) / wG,
// with fG_k(d_i) = f_k(d_i) - w_k . d_i the Gaussian part at the model's own
// dictionary vectors, which the detection kernels evaluate (the dictionary,
// transposed to received-vector rows, is detected with the model).
#include <cmath>

#include "apsm_internal.h"

namespace apsm {
namespace {

constexpr int kNormThreads = 256;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct BallLayout {
  size_t x, soft, scale, bytes;
};

BallLayout ball_layout(int M2, int K, int cap) {
  BallLayout l{};
  l.x = 0;
  l.soft = align256((size_t)cap * M2 * sizeof(float));
  l.scale = l.soft + align256((size_t)cap * K * 2 * sizeof(float));
  l.bytes = l.scale + align256((size_t)K * sizeof(float));
  return l;
}

// xt[i][m] = dict[m][i]: the dictionary entries as rows of received vectors.
__global__ __launch_bounds__(256) void transpose_kernel(const float* __restrict__ dict, int cap, int M2,
                                                        float* __restrict__ xt) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)cap * M2) return;
  const int i = (int)(e / M2), m = (int)(e - (size_t)i * M2);
  xt[e] = dict[(size_t)m * cap + i];
}

// One workgroup per user: the norm of f_k and its scale factor.
__global__ __launch_bounds__(kNormThreads) void ball_norm_kernel(const float* __restrict__ dict,
                                                                 const float* __restrict__ alpha,
                                                                 const float* __restrict__ w,
                                                                 const int32_t* __restrict__ state,
                                                                 const float* __restrict__ soft, int cap, int M2,
                                                                 int K, float wl, float wg, float radius,
                                                                 float* __restrict__ scale, float* norms) {
  __shared__ float wk[APSM_MAX_M2];
  __shared__ double red[kNormThreads];
  const int k = blockIdx.x, tid = threadIdx.x;
  for (int m = tid; m < M2; m += kNormThreads) wk[m] = w[(size_t)k * M2 + m];
  __syncthreads();
  const int size = min(max(state[0], 0), cap);
  double acc = 0.0;
  if (wg > 0.0f) {
    for (int i = tid; i < size; i += kNormThreads) {
      float wd = 0.0f;
      for (int m = 0; m < M2; ++m) wd = fmaf(wk[m], dict[(size_t)m * cap + i], wd);   // coalesced over i
      const float fg = soft[((size_t)i * K + k) * 2] - wd;
      acc += (double)alpha[(size_t)i * K + k] * (double)fg;
    }
  }
  red[tid] = acc;
  __syncthreads();
  for (int h = kNormThreads / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) {
    double lin = 0.0;
    for (int m = 0; m < M2; ++m) lin += (double)wk[m] * wk[m];
    double n2 = 0.0;
    if (wl > 0.0f) n2 += lin / wl;
    if (wg > 0.0f) n2 += red[0] / wg;
    const double nrm = sqrt(n2 > 0.0 ? n2 : 0.0);
    scale[k] = nrm > (double)radius ? (float)(radius / nrm) : 1.0f;
    if (norms) norms[k] = (float)nrm;
  }
}

__global__ __launch_bounds__(256) void ball_scale_kernel(float* __restrict__ w, float* __restrict__ alpha,
                                                         const float* __restrict__ scale, int cap, int M2, int K) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nw = (size_t)K * M2, na = (size_t)cap * K;
  if (e < nw) {
    w[e] *= scale[e / M2];
  } else if (e < nw + na) {
    const size_t a = e - nw;
    alpha[a] *= scale[a % K];
  }
}

int check_ball(const apsm_model_t* model, float sigma2, float w_lin, float w_gauss, float radius,
               const void* workspace, size_t ws_bytes) {
  if (int rc = check_model(model)) return rc;
  if (!finite_pos(sigma2) || !std::isfinite(w_lin) || !std::isfinite(w_gauss) || w_lin < 0.0f ||
      w_gauss < 0.0f || (w_lin == 0.0f && w_gauss == 0.0f))
    return APSM_ERR_INVALID_ARG;
  if (!std::isfinite(radius) || radius < 0.0f) return APSM_ERR_INVALID_ARG;
  const BallLayout l = ball_layout(model->M2, model->K, model->dict_cap);
  if (!workspace || ws_bytes < l.bytes || (reinterpret_cast<uintptr_t>(workspace) & 255)) return APSM_ERR_WORKSPACE;
  return APSM_OK;
}

// Launches only (arguments checked by the caller).
int ball_launch(const apsm_model_t* model, float sigma2, float w_lin, float w_gauss, float radius,
                void* workspace, float* norms, hipStream_t s) {
  const int M2 = model->M2, K = model->K, cap = model->dict_cap;
  const BallLayout l = ball_layout(M2, K, cap);
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  float* xt = reinterpret_cast<float*>(ws + l.x);
  float* soft = reinterpret_cast<float*>(ws + l.soft);
  float* scale = reinterpret_cast<float*>(ws + l.scale);
  if (w_gauss > 0.0f) {
    const size_t n = (size_t)cap * M2;
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, model->dict, cap, M2,
                       xt);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return hip_status(e);
    const DetectArgs a = detect_args(model, sigma2, cap, xt, soft, nullptr, APSM_MOD_NONE, nullptr, nullptr);
    if (hipError_t e = launch_detect(a, s); e != hipSuccess) return hip_status(e);
  }
  hipLaunchKernelGGL(ball_norm_kernel, dim3(K), dim3(kNormThreads), 0, s, model->dict, model->alpha, model->w,
                     model->state, soft, cap, M2, K, w_lin, w_gauss, radius, scale, norms);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return hip_status(e);
  const size_t n = (size_t)K * M2 + (size_t)cap * K;
  hipLaunchKernelGGL(ball_scale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, model->w, model->alpha,
                     scale, cap, M2, K);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return hip_status(e);
  return hip_status(launch_pack_model(model->dict, model->alpha, model->w, model->state, cap, M2, K, model->packed,
                                      s));
}

}  // namespace
}  // namespace apsm

extern "C" {

size_t apsm_ball_workspace_bytes(int M2, int K, int dict_cap) {
  if (M2 < 2 || (M2 & 1) || K < 1 || dict_cap < 1 || M2 > APSM_MAX_M2 || K > APSM_MAX_K ||
      dict_cap > APSM_MAX_DICT)
    return 0;
  return apsm::ball_layout(M2, K, dict_cap).bytes;
}

int apsm_project_ball(const apsm_model_t* model, float sigma2, float w_lin, float w_gauss, float radius,
                      void* workspace, size_t ws_bytes, float* norms, void* stream) {
  using namespace apsm;
  if (int rc = check_ball(model, sigma2, w_lin, w_gauss, radius, workspace, ws_bytes)) return rc;
  return ball_launch(model, sigma2, w_lin, w_gauss, radius, workspace, norms, (hipStream_t)stream);
}

int apsm_pocs(const apsm_params_t* params, int M2, int K, int P, const float* rx_pilot, const float* sym_pilot,
              const apsm_model_t* model, float radius, int cycles, void* workspace, size_t ws_bytes,
              void* stream) {
  using namespace apsm;
  if (int rc = check_params(params)) return rc;
  if (!model) return APSM_ERR_INVALID_ARG;
  if (cycles < 1) return APSM_ERR_INVALID_ARG;
  if (cycles > 1 && !(params->w_lin > 0.0f)) return APSM_ERR_INVALID_ARG;   // continued cycles: w = wL v
  if (!rx_pilot || !sym_pilot) return APSM_ERR_INVALID_ARG;
  if (P < 1 || M2 < 2 || (M2 & 1) || K < 1) return APSM_ERR_SHAPE;
  if (model->M2 != M2 || model->K != K || model->dict_cap != params->dict_cap) return APSM_ERR_SHAPE;
  if (int rc = check_ball(model, params->sigma2, params->w_lin, params->w_gauss, radius, workspace, ws_bytes))
    return rc;
  apsm_params_t pc = *params;
  for (int c = 0; c < cycles; ++c) {
    if (c > 0) pc.init = APSM_INIT_CONTINUE;
    if (int rc = train_impl(&pc, M2, K, P, 1, rx_pilot, sym_pilot, model, stream)) return rc;
    if (int rc = ball_launch(model, params->sigma2, params->w_lin, params->w_gauss, radius, workspace, nullptr,
                             (hipStream_t)stream))
      return rc;
  }
  return APSM_OK;
}

}  // extern "C"
