// Internal declarations shared by the host ABI layer and the kernel launchers
// of libapsm.  Not part of the public interface (include/apsm.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/apsm.h"

namespace apsm {

// log2(e): the kernels evaluate exp(-x) as exp2(-x * log2 e) on v_exp_f32.
constexpr float kLog2e = 1.4426950408889634f;

// Everything the training kernel needs, by value (kernel arguments; no device
// allocation, and a captured graph keeps a copy).
struct TrainArgs {
  const float* rx;        // [P][M2] pilot vectors, r1 layout
  const float* sym;       // [P][K][2]
  float* dict;            // [cap][M2]
  float* alpha;           // [cap][K]
  float* w;               // [K][M2]
  int32_t* state;         // [4]
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

}  // namespace apsm
