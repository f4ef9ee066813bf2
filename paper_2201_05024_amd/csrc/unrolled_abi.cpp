// Host side of the unrolled-training entry points: validation, workspace
// layout and launch.
#include "apsm_internal.h"

namespace {

using namespace apsm;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool check(const apsm_unrolled_t* u) {
  if (!u) return false;
  if (u->n_inst < 1 || u->P < 1 || u->P > 2048 || u->M2 < 2 || (u->M2 & 1) || u->M2 > APSM_MAX_M2) return false;
  if (u->K < 1 || u->K > APSM_MAX_K || u->S < 1 || u->passes < 1 || u->ckpt_every < 1) return false;
  if (u->window < 1 || u->window > APSM_MAX_WINDOW) return false;
  if (!(u->w_lin >= 0.0f) || !(u->w_gauss >= 0.0f) || (u->w_lin == 0.0f && u->w_gauss == 0.0f)) return false;
  return true;
}

// Layout of one instance's part of the workspace (byte offsets).
UnrolledArgs layout(const apsm_unrolled_t* u) {
  UnrolledArgs a{};
  a.n = u->n_inst;
  a.P = u->P;
  a.T = 2 * u->P;
  a.M2 = u->M2;
  a.M2P = (u->M2 + 3) / 4 * 4;
  a.K = u->K;
  a.KP = u->K <= 4 ? 4 : u->K <= 8 ? 8 : 16;
  a.S = u->S;
  a.W = u->window;
  a.WP = 1;
  while (a.WP < a.W) a.WP <<= 1;
  a.passes = u->passes;
  a.E = u->ckpt_every < u->passes ? u->ckpt_every : u->passes;
  a.wl = u->w_lin;
  a.wg = u->w_gauss;
  a.inv_count = (float)(1.0 / ((double)u->n_inst * u->S * u->K));
  const size_t T = a.T, KP = a.KP, SW = (size_t)a.K * a.M2P + T * KP;
  const size_t NC = (a.passes + a.E - 1) / a.E;
  const size_t Sr = 2 * (size_t)a.S;
  size_t o = 0;
  a.off_G = o;     o = align256(o + T * T * 4);
  a.off_D = o;     o = align256(o + T * T * 4);
  a.off_ck = o;    o = align256(o + NC * SW * 4);
  a.off_st = o;    o = align256(o + SW * 4);
  a.off_sc = o;    o = align256(o + SW * 4);
  a.off_tx = o;    o = align256(o + (size_t)a.E * T * a.W * KP * 4);
  a.off_th = o;    o = align256(o + (size_t)a.E * T * a.W * KP * 4);
  a.off_adj = o;   o = align256(o + SW * 4);
  a.off_X = o;     o = align256(o + T * KP * 4);
  a.off_fbar = o;  o = align256(o + Sr * KP * 4);
  a.off_lpart = o; o = align256(o + (Sr + 255) / 256 * 4);
  a.off_spart = o; o = align256(o + (T + 63) / 64 * 4);
  a.off_gpart = o; o = align256(o + (4 + APSM_MAX_WINDOW) * 8);
  a.inst_bytes = o;
  return a;
}

int prepare(const apsm_unrolled_t* u, const float* theta, const float* rx_pilot, const float* sym_pilot,
            const float* rx_val, const float* sym_val, void* ws, size_t ws_bytes, UnrolledArgs* out) {
  if (!check(u)) return APSM_ERR_INVALID_ARG;
  if (!theta || !rx_pilot || !sym_pilot || !rx_val || !sym_val) return APSM_ERR_INVALID_ARG;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return APSM_ERR_WORKSPACE;
  UnrolledArgs a = layout(u);
  if (ws_bytes < a.inst_bytes * (size_t)a.n) return APSM_ERR_WORKSPACE;
  a.theta = theta;
  a.rx_pilot = rx_pilot;
  a.sym_pilot = sym_pilot;
  a.rx_val = rx_val;
  a.sym_val = sym_val;
  a.ws = ws;
  *out = a;
  return APSM_OK;
}

}  // namespace

extern "C" {

size_t apsm_unrolled_workspace_bytes(const apsm_unrolled_t* u) {
  if (!check(u)) return 0;
  const UnrolledArgs a = layout(u);
  return a.inst_bytes * (size_t)a.n;
}

int apsm_unrolled_forward(const apsm_unrolled_t* u, const float* theta, const float* rx_pilot,
                          const float* sym_pilot, const float* rx_val, const float* sym_val, void* workspace,
                          size_t ws_bytes, float* loss, void* stream) {
  UnrolledArgs a;
  if (int rc = prepare(u, theta, rx_pilot, sym_pilot, rx_val, sym_val, workspace, ws_bytes, &a)) return rc;
  if (!loss) return APSM_ERR_INVALID_ARG;
  return hip_status(launch_unrolled_forward(a, loss, (hipStream_t)stream));
}

int apsm_unrolled_backward(const apsm_unrolled_t* u, const float* theta, const float* rx_pilot,
                           const float* sym_pilot, const float* rx_val, const float* sym_val, void* workspace,
                           size_t ws_bytes, const float* upstream, float* grad, void* stream) {
  UnrolledArgs a;
  if (int rc = prepare(u, theta, rx_pilot, sym_pilot, rx_val, sym_val, workspace, ws_bytes, &a)) return rc;
  if (!grad) return APSM_ERR_INVALID_ARG;
  return hip_status(launch_unrolled_backward(a, grad, upstream, (hipStream_t)stream));
}

}  // extern "C"
