// Host side of the C ABI: argument validation, parameter folding and dispatch
// to the kernel launchers.  Validation runs before any HIP call, so a
// rejected call touches neither the device nor the stream.
#include <cmath>
#include <cstring>
#include <string>

#include "apsm_internal.h"

namespace {

thread_local std::string g_last_hip_error;

int hip_status(hipError_t e) {
  if (e == hipSuccess) return APSM_OK;
  g_last_hip_error = hipGetErrorString(e);
  return APSM_ERR_HIP;
}

bool finite_pos(float x) { return std::isfinite(x) && x > 0.0f; }

int check_model(const apsm_model_t* m) {
  if (!m || !m->dict || !m->alpha || !m->w || !m->state) return APSM_ERR_INVALID_ARG;
  if (m->reserved != 0) return APSM_ERR_INVALID_ARG;
  if (m->M2 < 2 || (m->M2 & 1) || m->K < 1 || m->dict_cap < 1) return APSM_ERR_SHAPE;
  if (m->M2 > APSM_MAX_M2 || m->K > APSM_MAX_K || m->dict_cap > APSM_MAX_DICT)
    return APSM_ERR_UNSUPPORTED;
  return APSM_OK;
}

}  // namespace

extern "C" {

const char* apsm_version(void) { return "0.1.0"; }

const char* apsm_strerror(int code) {
  switch (code) {
    case APSM_OK: return "success";
    case APSM_ERR_INVALID_ARG: return "invalid argument (null pointer or parameter out of range)";
    case APSM_ERR_SHAPE: return "inconsistent sizes";
    case APSM_ERR_UNSUPPORTED: return "size beyond the limits of this build";
    case APSM_ERR_HIP: return "HIP runtime error (see apsm_last_hip_error)";
    default: return "unknown status code";
  }
}

const char* apsm_last_hip_error(void) { return g_last_hip_error.c_str(); }

int apsm_train(const apsm_params_t* p, int M2, int K, int P, const float* rx_pilot,
               const float* sym_pilot, const apsm_model_t* model, void* stream) {
  if (!p || !rx_pilot || !sym_pilot) return APSM_ERR_INVALID_ARG;
  if (int rc = check_model(model)) return rc;
  if (!finite_pos(p->sigma2) || !std::isfinite(p->eps) || p->eps < 0.0f) return APSM_ERR_INVALID_ARG;
  if (!(p->mu > 0.0f && p->mu < 2.0f)) return APSM_ERR_INVALID_ARG;
  if (!std::isfinite(p->w_lin) || !std::isfinite(p->w_gauss) || p->w_lin < 0.0f ||
      p->w_gauss < 0.0f || (p->w_lin == 0.0f && p->w_gauss == 0.0f))
    return APSM_ERR_INVALID_ARG;
  if (p->reserved != 0 || p->window < 1) return APSM_ERR_INVALID_ARG;
  if (p->window > APSM_MAX_WINDOW) return APSM_ERR_UNSUPPORTED;
  if (p->dict_cap < p->window) return APSM_ERR_INVALID_ARG;
  if (P < 1 || M2 < 2 || (M2 & 1) || K < 1) return APSM_ERR_SHAPE;
  if (M2 > APSM_MAX_M2 || K > APSM_MAX_K) return APSM_ERR_UNSUPPORTED;
  if (model->M2 != M2 || model->K != K || model->dict_cap != p->dict_cap) return APSM_ERR_SHAPE;
  if ((long long)P * 2 > (long long)INT32_MAX / 2) return APSM_ERR_UNSUPPORTED;

  apsm::TrainArgs a{};
  a.rx = rx_pilot;
  a.sym = sym_pilot;
  a.dict = model->dict;
  a.alpha = model->alpha;
  a.w = model->w;
  a.state = model->state;
  a.P = P;
  a.M2 = M2;
  a.M = M2 / 2;
  a.K = K;
  a.W = p->window;
  a.cap = p->dict_cap;
  a.c2 = apsm::kLog2e / (2.0f * p->sigma2);
  a.eps = p->eps;
  a.mu = p->mu;
  a.wl = p->w_lin;
  a.wg = p->w_gauss;
  for (int i = 0; i < APSM_MAX_WINDOW; ++i) a.omega[i] = 1.0f;
  if (p->pos_weights) {
    for (int i = 0; i < p->window; ++i) {
      if (!finite_pos(p->pos_weights[i])) return APSM_ERR_INVALID_ARG;
      a.omega[i] = p->pos_weights[i];
    }
  }
  return hip_status(apsm::launch_train(a, (hipStream_t)stream));
}

int apsm_detect(const apsm_model_t* model, float sigma2, int S, const float* rx, float* soft,
                uint8_t* hard, int modulation, const uint8_t* truth, int64_t* err_count,
                void* stream) {
  if (int rc = check_model(model)) return rc;
  if (!finite_pos(sigma2)) return APSM_ERR_INVALID_ARG;
  if (S < 0) return APSM_ERR_SHAPE;
  if (modulation != APSM_MOD_NONE && modulation != APSM_MOD_QPSK && modulation != APSM_MOD_QAM16)
    return APSM_ERR_INVALID_ARG;
  if (S == 0) return APSM_OK;                  // nothing to read or write; pointers may be NULL
  if ((hard || truth || err_count) && modulation == APSM_MOD_NONE) return APSM_ERR_INVALID_ARG;
  if ((truth == nullptr) != (err_count == nullptr)) return APSM_ERR_INVALID_ARG;
  if (!soft && !hard && !err_count) return APSM_ERR_INVALID_ARG;
  if (!rx) return APSM_ERR_INVALID_ARG;

  apsm::DetectArgs a{};
  a.dict = model->dict;
  a.alpha = model->alpha;
  a.w = model->w;
  a.state = model->state;
  a.rx = rx;
  a.soft = soft;
  a.hard = hard;
  a.truth = truth;
  a.err = reinterpret_cast<unsigned long long*>(err_count);
  a.cap = model->dict_cap;
  a.M2 = model->M2;
  a.M = model->M2 / 2;
  a.K = model->K;
  a.S = S;
  a.modulation = modulation;
  a.c2 = apsm::kLog2e / (2.0f * sigma2);
  return hip_status(apsm::launch_detect(a, (hipStream_t)stream));
}

int apsm_get_status(const apsm_model_t* model, int32_t* host_state) {
  if (int rc = check_model(model)) return rc;
  if (!host_state) return APSM_ERR_INVALID_ARG;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(host_state, model->state, 4 * sizeof(int32_t), hipMemcpyDeviceToHost);
  return hip_status(e);
}

}  // extern "C"
