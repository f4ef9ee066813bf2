// Host side of the C ABI: argument validation, parameter folding and dispatch
// to the kernel launchers.  Validation runs before any HIP call, so a
// rejected call touches neither the device nor the stream.
#include <cmath>
#include <cstring>
#include <string>

#include "apsm_internal.h"

namespace {
thread_local std::string g_last_hip_error;
}  // namespace

namespace apsm {

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
  if (!m->packed && apsm::packed_model_bytes(m->M2, m->K, m->dict_cap) > 0) return APSM_ERR_INVALID_ARG;
  return APSM_OK;
}

int check_params(const apsm_params_t* p) {
  if (!p) return APSM_ERR_INVALID_ARG;
  if (!finite_pos(p->sigma2) || !std::isfinite(p->eps) || p->eps < 0.0f) return APSM_ERR_INVALID_ARG;
  if (!(p->mu > 0.0f && p->mu < 2.0f)) return APSM_ERR_INVALID_ARG;
  if (!std::isfinite(p->w_lin) || !std::isfinite(p->w_gauss) || p->w_lin < 0.0f ||
      p->w_gauss < 0.0f || (p->w_lin == 0.0f && p->w_gauss == 0.0f))
    return APSM_ERR_INVALID_ARG;
  if ((p->extrapolate != 0 && p->extrapolate != 1) || p->window < 1) return APSM_ERR_INVALID_ARG;
  if (p->init != APSM_INIT_ZERO && p->init != APSM_INIT_LINEAR && p->init != APSM_INIT_CONTINUE)
    return APSM_ERR_INVALID_ARG;
  if (p->init != APSM_INIT_ZERO && !(p->w_lin > 0.0f)) return APSM_ERR_INVALID_ARG;   // w = wL v
  if (p->weights != APSM_WEIGHTS_POSITION && p->weights != APSM_WEIGHTS_VIOLATION &&
      p->weights != APSM_WEIGHTS_ACTIVE)
    return APSM_ERR_INVALID_ARG;
  if (p->weights != APSM_WEIGHTS_POSITION && p->pos_weights) return APSM_ERR_INVALID_ARG;
  if (p->window > APSM_MAX_WINDOW) return APSM_ERR_UNSUPPORTED;
  if (p->dict_cap < p->window) return APSM_ERR_INVALID_ARG;
  if (p->pos_weights) {
    for (int i = 0; i < p->window; ++i)
      if (!finite_pos(p->pos_weights[i])) return APSM_ERR_INVALID_ARG;
  }
  return APSM_OK;
}

void fill_common(const apsm_params_t* p, TrainCommon& cm) {
  cm.W = p->window;
  cm.eps = p->eps;
  cm.mu = p->mu;
  cm.wl = p->w_lin;
  cm.wg = p->w_gauss;
  cm.init = p->init;
  cm.weights = p->weights;
  cm.extrapolate = p->extrapolate;
  for (int i = 0; i < APSM_MAX_WINDOW; ++i) cm.omega[i] = 1.0f;
  if (p->pos_weights)
    for (int i = 0; i < p->window; ++i) cm.omega[i] = p->pos_weights[i];
}

int check_detect_args(int M2, int K, float sigma2, int S, const float* rx, float* soft, uint8_t* hard,
                      int modulation, const uint8_t* truth, int64_t* err_count) {
  (void)M2;
  (void)K;
  if (!finite_pos(sigma2)) return APSM_ERR_INVALID_ARG;
  if (S < 0) return APSM_ERR_SHAPE;
  if (modulation != APSM_MOD_NONE && modulation != APSM_MOD_QPSK && modulation != APSM_MOD_QAM16)
    return APSM_ERR_INVALID_ARG;
  if (S == 0) return APSM_OK;                  // nothing to read or write; pointers may be NULL
  if ((hard || truth || err_count) && modulation == APSM_MOD_NONE) return APSM_ERR_INVALID_ARG;
  if ((truth == nullptr) != (err_count == nullptr)) return APSM_ERR_INVALID_ARG;
  if (!soft && !hard && !err_count) return APSM_ERR_INVALID_ARG;
  if (!rx) return APSM_ERR_INVALID_ARG;
  return APSM_OK;
}

DetectArgs detect_args(const apsm_model_t* model, float sigma2, int S, const float* rx, float* soft,
                       uint8_t* hard, int modulation, const uint8_t* truth, int64_t* err_count) {
  DetectArgs a{};
  a.dict = model->dict;
  a.alpha = model->alpha;
  a.w = model->w;
  a.state = model->state;
  a.flags = model->state + 3;
  a.packed = static_cast<const unsigned char*>(model->packed);
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
  a.c2 = kLog2e / (2.0f * sigma2);
  return a;
}

}  // namespace apsm

extern "C" {

const char* apsm_version(void) { return "0.1.0"; }

const char* apsm_strerror(int code) {
  switch (code) {
    case APSM_OK: return "success";
    case APSM_ERR_INVALID_ARG: return "invalid argument (null pointer or parameter out of range)";
    case APSM_ERR_SHAPE: return "inconsistent sizes";
    case APSM_ERR_UNSUPPORTED: return "size beyond the limits of this build";
    case APSM_ERR_HIP: return "HIP runtime error (see apsm_last_hip_error)";
    case APSM_ERR_WORKSPACE: return "workspace missing, too small or not 256-byte aligned";
    case APSM_ERR_NONFINITE: return "non-finite values flagged in the model status";
    default: return "unknown status code";
  }
}

const char* apsm_last_hip_error(void) { return g_last_hip_error.c_str(); }

}  // extern "C"

namespace apsm {

// Shared by apsm_train, apsm_train_batched and apsm_track: every check
// happens before the first launch.
int train_impl(const apsm_params_t* p, int M2, int K, int P, int n_inst, const float* rx_pilot,
               const float* sym_pilot, const apsm_model_t* models, void* stream) {
  if (int rc = check_params(p)) return rc;
  if (!rx_pilot || !sym_pilot || !models) return APSM_ERR_INVALID_ARG;
  if (P < 1 || M2 < 2 || (M2 & 1) || K < 1 || n_inst < 0) return APSM_ERR_SHAPE;
  if (M2 > APSM_MAX_M2 || K > APSM_MAX_K) return APSM_ERR_UNSUPPORTED;
  if ((long long)P * 2 > (long long)INT32_MAX / 2) return APSM_ERR_UNSUPPORTED;
  for (int i = 0; i < n_inst; ++i) {
    if (int rc = check_model(&models[i])) return rc;
    if (models[i].M2 != M2 || models[i].K != K || models[i].dict_cap != p->dict_cap) return APSM_ERR_SHAPE;
  }

  apsm::TrainArgs a{};
  fill_common(p, a.cm);
  a.rx = rx_pilot;
  a.sym = sym_pilot;
  a.P = P;
  a.M2 = M2;
  a.K = K;
  a.cap = p->dict_cap;
  a.c2 = apsm::kLog2e / (2.0f * p->sigma2);

  for (int b0 = 0; b0 < n_inst; b0 += apsm::kMaxTrainBatch) {
    const int nb = n_inst - b0 < apsm::kMaxTrainBatch ? n_inst - b0 : apsm::kMaxTrainBatch;
    a.rx = rx_pilot + (size_t)b0 * P * M2;
    a.sym = sym_pilot + (size_t)b0 * P * K * 2;
    a.st = p->set_types ? p->set_types + (size_t)b0 * P * K * 2 : nullptr;
    a.n_inst = nb;
    for (int i = 0; i < nb; ++i) {
      a.dict[i] = models[b0 + i].dict;
      a.alpha[i] = models[b0 + i].alpha;
      a.w[i] = models[b0 + i].w;
      a.state[i] = models[b0 + i].state;
    }
    hipError_t e = apsm::launch_train(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_status(e);
  }
  for (int i = 0; i < n_inst; ++i) {
    const apsm_model_t& m = models[i];
    hipError_t e = apsm::launch_pack_model(m.dict, m.alpha, m.w, m.state, m.dict_cap, M2, K, m.packed,
                                           (hipStream_t)stream);
    if (e != hipSuccess) return hip_status(e);
  }
  return APSM_OK;
}

}  // namespace apsm

using namespace apsm;

extern "C" {

int apsm_train(const apsm_params_t* p, int M2, int K, int P, const float* rx_pilot,
               const float* sym_pilot, const apsm_model_t* model, void* stream) {
  if (!model) return APSM_ERR_INVALID_ARG;
  return train_impl(p, M2, K, P, 1, rx_pilot, sym_pilot, model, stream);
}

int apsm_train_batched(const apsm_params_t* p, int M2, int K, int P, int n_inst, const float* rx_pilot,
                       const float* sym_pilot, const apsm_model_t* models, void* stream) {
  if (n_inst == 0) return APSM_OK;
  return train_impl(p, M2, K, P, n_inst, rx_pilot, sym_pilot, models, stream);
}

size_t apsm_model_packed_bytes(int M2, int K, int dict_cap) {
  if (M2 < 2 || (M2 & 1) || K < 1 || dict_cap < 1 || M2 > APSM_MAX_M2 || K > APSM_MAX_K ||
      dict_cap > APSM_MAX_DICT)
    return 0;
  return apsm::packed_model_bytes(M2, K, dict_cap);
}

int apsm_model_pack(const apsm_model_t* model, void* stream) {
  if (int rc = check_model(model)) return rc;
  return hip_status(apsm::launch_pack_model(model->dict, model->alpha, model->w, model->state, model->dict_cap,
                                            model->M2, model->K, model->packed, (hipStream_t)stream));
}

int apsm_detect(const apsm_model_t* model, float sigma2, int S, const float* rx, float* soft,
                uint8_t* hard, int modulation, const uint8_t* truth, int64_t* err_count,
                void* stream) {
  if (int rc = check_model(model)) return rc;
  if (int rc = check_detect_args(model->M2, model->K, sigma2, S, rx, soft, hard, modulation, truth, err_count))
    return rc;
  if (S == 0) return APSM_OK;
  const DetectArgs a = detect_args(model, sigma2, S, rx, soft, hard, modulation, truth, err_count);
  return hip_status(launch_detect(a, (hipStream_t)stream));
}

int apsm_get_status(const apsm_model_t* model, int32_t* host_state) {
  if (int rc = check_model(model)) return rc;
  if (!host_state) return APSM_ERR_INVALID_ARG;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(host_state, model->state, 4 * sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_status(e);
  return host_state[3] != 0 ? APSM_ERR_NONFINITE : APSM_OK;
}

}  // extern "C"
