// Around the iteration: the linear MMSE receive filter used as the initial
// filter f_0 when a channel estimate exists (Sec. I: initialisation by a
// conventional linear filter; Sec. II-D: f_0 of eqn:apsm is arbitrary), and
// decision-directed tracking (Sec. II-E, remark on focusing on detection:
// gradual channel changes are tracked by running the iteration on the data
// symbols): detect a block with the frozen filter, take the slicer's
// decisions as the targets, continue the training over the block.
#include <cmath>

#include "apsm_internal.h"

namespace apsm {
namespace {

constexpr int kMmseThreads = 256;

// One workgroup per instance.  h: [K][2M] planar columns h_k = [Re; Im];
// w: [K][2M] the filters w_k = [Re u_k; Im u_k] with U = H (H^H H + n0 I)^-1,
// so that w_k . r1 + i w_k . r2 = u_k^H r.  The K x K Hermitian system is
// inverted by Gauss-Jordan elimination without pivoting (its matrix is
// positive definite for n0 > 0 or H of full column rank).
__global__ __launch_bounds__(kMmseThreads) void mmse_kernel(const float* h_all, float n0, int M2, int K, float* w_all) {
  __shared__ float hr[APSM_MAX_K][APSM_MAX_M2 / 2], hi[APSM_MAX_K][APSM_MAX_M2 / 2];
  __shared__ float gr[APSM_MAX_K][2 * APSM_MAX_K], gi[APSM_MAX_K][2 * APSM_MAX_K];   // [G | I] -> [I | G^-1]
  __shared__ float fr[APSM_MAX_K], fi[APSM_MAX_K];
  const int M = M2 / 2, tid = threadIdx.x;
  const float* h = h_all + (size_t)blockIdx.x * K * M2;
  float* w = w_all + (size_t)blockIdx.x * K * M2;
  for (int e = tid; e < K * M; e += kMmseThreads) {
    const int k = e / M, m = e - k * M;
    hr[k][m] = h[k * M2 + m];
    hi[k][m] = h[k * M2 + M + m];
  }
  __syncthreads();
  // G = H^H H + n0 I next to the identity
  for (int e = tid; e < K * 2 * K; e += kMmseThreads) {
    const int i = e / (2 * K), j = e - i * 2 * K;
    float re = 0.0f, im = 0.0f;
    if (j < K) {
      for (int m = 0; m < M; ++m) {       // conj(h_i[m]) h_j[m]
        re = fmaf(hr[i][m], hr[j][m], fmaf(hi[i][m], hi[j][m], re));
        im = fmaf(hr[i][m], hi[j][m], fmaf(-hi[i][m], hr[j][m], im));
      }
      if (i == j) re += n0;
    } else {
      re = (j - K == i) ? 1.0f : 0.0f;
    }
    gr[i][j] = re;
    gi[i][j] = im;
  }
  __syncthreads();
  for (int piv = 0; piv < K; ++piv) {
    // row factors f_i = g[i][piv] / g[piv][piv] (the pivot row is scaled to 1)
    if (tid < K) {
      const float pr = gr[piv][piv], pi = gi[piv][piv], d = pr * pr + pi * pi;
      const float ar = gr[tid][piv], ai = gi[tid][piv];
      fr[tid] = (ar * pr + ai * pi) / d;
      fi[tid] = (ai * pr - ar * pi) / d;
    }
    __syncthreads();
    float nr[2] = {0.0f, 0.0f}, ni[2] = {0.0f, 0.0f};
    for (int u = 0, e = tid; u < 2; ++u, e += kMmseThreads) {
      if (e >= K * 2 * K) continue;
      const int i = e / (2 * K), j = e - i * 2 * K;
      const float pr = gr[piv][j], pi = gi[piv][j];
      if (i == piv) {                     // pivot row / pivot
        const float dr = gr[piv][piv], di = gi[piv][piv], d = dr * dr + di * di;
        nr[u] = (pr * dr + pi * di) / d;
        ni[u] = (pi * dr - pr * di) / d;
      } else {                            // row i - f_i (pivot row / pivot) g[piv][piv] = row i - f_i row piv
        nr[u] = gr[i][j] - (fr[i] * pr - fi[i] * pi);
        ni[u] = gi[i][j] - (fr[i] * pi + fi[i] * pr);
      }
    }
    __syncthreads();
    for (int u = 0, e = tid; u < 2; ++u, e += kMmseThreads) {
      if (e >= K * 2 * K) continue;
      const int i = e / (2 * K), j = e - i * 2 * K;
      gr[i][j] = nr[u];
      gi[i][j] = ni[u];
    }
    __syncthreads();
  }
  // u_k[m] = sum_j h_j[m] (G^-1)[j][k]
  for (int e = tid; e < K * M; e += kMmseThreads) {
    const int k = e / M, m = e - k * M;
    float re = 0.0f, im = 0.0f;
    for (int j = 0; j < K; ++j) {
      const float ar = gr[j][K + k], ai = gi[j][K + k];
      re = fmaf(hr[j][m], ar, fmaf(-hi[j][m], ai, re));
      im = fmaf(hr[j][m], ai, fmaf(hi[j][m], ar, im));
    }
    w[k * M2 + m] = re;
    w[k * M2 + M + m] = im;
  }
}

// The decided constellation point of every soft value, in place (per axis
// the nearest level; a value exactly on a threshold takes the higher level).
__global__ __launch_bounds__(256) void slicer_kernel(float* v, size_t n, int bits) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = v[i];
  if (bits == 1) {
    v[i] = x >= 0.0f ? 0.70710678118654752440f : -0.70710678118654752440f;
  } else {
    const float th = 0.63245553203367586640f;   // 2 / sqrt(10)
    const int idx = (x >= -th) + (x >= 0.0f) + (x >= th);
    v[i] = (2 * idx - 3) * 0.31622776601683793320f;   // {-3, -1, 1, 3} / sqrt(10)
  }
}

}  // namespace
}  // namespace apsm

extern "C" {

int apsm_linear_mmse(const float* h, float n0, int M2, int K, int n_inst, float* w, void* stream) {
  using namespace apsm;
  if (!h || !w || !std::isfinite(n0) || n0 < 0.0f) return APSM_ERR_INVALID_ARG;
  if (M2 < 2 || (M2 & 1) || K < 1 || n_inst < 0) return APSM_ERR_SHAPE;
  if (M2 > APSM_MAX_M2 || K > APSM_MAX_K) return APSM_ERR_UNSUPPORTED;
  if (n_inst == 0) return APSM_OK;
  hipLaunchKernelGGL(mmse_kernel, dim3(n_inst), dim3(kMmseThreads), 0, (hipStream_t)stream, h, n0, M2, K, w);
  return hip_status(hipGetLastError());
}

int apsm_track(const apsm_params_t* p, const apsm_model_t* model, int S, const float* rx, int modulation,
               float* decided, uint8_t* hard, const uint8_t* truth, int64_t* err_count, void* stream) {
  using namespace apsm;
  if (int rc = check_params(p)) return rc;
  if (p->set_types) return APSM_ERR_UNSUPPORTED;     // the targets are decisions: hyperslabs
  if (int rc = check_model(model)) return rc;
  if (model->dict_cap != p->dict_cap) return APSM_ERR_SHAPE;
  if (!(p->w_lin > 0.0f)) return APSM_ERR_INVALID_ARG;
  if (modulation != APSM_MOD_QPSK && modulation != APSM_MOD_QAM16) return APSM_ERR_INVALID_ARG;
  if (S < 0) return APSM_ERR_SHAPE;
  if (S == 0) return APSM_OK;
  if (!decided) return APSM_ERR_INVALID_ARG;
  if (int rc = check_detect_args(model->M2, model->K, p->sigma2, S, rx, decided, hard, modulation, truth, err_count))
    return rc;
  if ((long long)S * 2 > (long long)INT32_MAX / 2) return APSM_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  // 1. the frozen filter's soft outputs (and optional decisions / error counts)
  const DetectArgs a = detect_args(model, p->sigma2, S, rx, decided, hard, modulation, truth, err_count);
  hipError_t e = launch_detect(a, s);
  // 2. the decided symbols as targets
  const size_t n = (size_t)S * model->K * 2;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(slicer_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, decided, n, modulation >> 1);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_status(e);
  // 3. the iteration continued over the block, then packing
  apsm_params_t pc = *p;
  pc.init = APSM_INIT_CONTINUE;
  return train_impl(&pc, model->M2, model->K, S, 1, rx, decided, model, stream);
}

}  // extern "C"
