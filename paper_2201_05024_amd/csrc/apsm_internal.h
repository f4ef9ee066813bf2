// Internal declarations shared by the host ABI layer and the kernel launchers
// of libapsm.  Not part of the public interface (include/apsm.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/apsm.h"

namespace apsm {

// log2(e): the kernels evaluate exp(-x) as exp2(-x * log2 e) on v_exp_f32.
constexpr float kLog2e = 1.4426950408889634f;

// Instances per training launch (one workgroup each); bounded so that the
// per-instance pointers fit the kernel-argument block.
constexpr int kMaxTrainBatch = 32;

// Everything the training kernel needs, by value (kernel arguments; no device
// allocation, and a captured graph keeps a copy).  Workgroup b trains
// instance b: pilots at rx + b * P * M2 and sym + b * P * K * 2, model
// arrays dict[b], alpha[b], w[b], state[b].
struct TrainArgs {
  const float* rx;        // [n][P][M2] pilot vectors, r1 layout
  const float* sym;       // [n][P][K][2]
  float* dict[kMaxTrainBatch];   // [cap][M2] each
  float* alpha[kMaxTrainBatch];  // [cap][K]
  float* w[kMaxTrainBatch];      // [K][M2]
  int32_t* state[kMaxTrainBatch];// [4]
  int n_inst;
  int P, M2, M, K, W, cap;
  float c2;               // log2e / (2 sigma^2)
  float eps, mu, wl, wg;
  float omega[APSM_MAX_WINDOW];   // position weights, omega[0] for j = n
};

struct DetectArgs {
  const float* dict;      // [cap][M2]
  const float* alpha;     // [cap][K]
  const float* w;         // [K][M2]
  const int32_t* state;   // [4], state[0] = entries in use
  const unsigned char* packed;  // packed model (split-FP16 path) or null
  const float* rx;        // [S][M2]
  float* soft;            // [S][K][2] or null
  uint8_t* hard;          // [S][K] or null
  const uint8_t* truth;   // [S][K] or null
  unsigned long long* err;// [K] or null
  int cap, M2, M, K, S;
  int modulation;         // bits per symbol (0, 2, 4)
  float c2;               // log2e / (2 sigma^2)
};

// Launchers: return a hipError_t from the launch.
hipError_t launch_train(const TrainArgs& a, hipStream_t stream);
hipError_t launch_detect(const DetectArgs& a, hipStream_t stream);
// Packed model for the split-FP16 detection path: bytes (0 when the shape
// uses the FP32 path) and the packing launch (no-op for such shapes).
size_t packed_model_bytes(int M2, int K, int cap);
hipError_t launch_pack_model(const float* dict, const float* alpha, const int32_t* state, int cap,
                             int M2, int K, void* packed, hipStream_t stream);

}  // namespace apsm
