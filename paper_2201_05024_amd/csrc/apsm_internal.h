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

// Initial filter and set weights of a training (apsm_params_t.init, .weights).
enum { kInitZero = APSM_INIT_ZERO, kInitLinear = APSM_INIT_LINEAR, kInitContinue = APSM_INIT_CONTINUE };
enum { kWeightsPosition = APSM_WEIGHTS_POSITION, kWeightsViolation = APSM_WEIGHTS_VIOLATION,
       kWeightsActive = APSM_WEIGHTS_ACTIVE };
enum { kSetSlab = APSM_SET_SLAB, kSetPlane = APSM_SET_PLANE, kSetUpper = APSM_SET_UPPER, kSetLower = APSM_SET_LOWER };

// Parameters shared by every detector of a training launch.
struct TrainCommon {
  int W;                  // window size
  float eps, mu, wl, wg;
  int init;               // kInit*: f_0 = 0, the model's linear part, or the whole model continued
  int weights;            // kWeights*: position weights (uniform by default), violation or active-set weights
  int extrapolate;        // 1: extrapolated relaxation mu M_n
  float omega[APSM_MAX_WINDOW];   // position weights, omega[0] for j = n
};

// One detector's training job as the kernel body sees it.
struct TrainJob {
  const float* rx;        // [P][M2] pilot vectors, r1 layout
  const float* sym;       // [P][K][2]
  float* dict;            // [M2][cap] component-major
  float* alpha;           // [cap][K]
  float* w;               // [K][M2]
  int32_t* state;         // [4]
  int P, M2, K, cap;      // K: users this job trains (k0 .. k0 + K - 1)
  int Kt, k0;             // the detector's users (row stride of sym and alpha), first user of the job
  float c2;               // log2e / (2 sigma^2)
  int variant;            // kernel specialisation (train_variant), table launches only
  // Precomputed kernel rows (rows launches only, else null): for step n,
  // glag[n * cap + l] = kappa_G(r_n, r_{n-l}) (0 for l > n) and
  // kw[n * W + q] = K(r_n, r_{n-q}) = wL r_n.r_{n-q} + wG kappa_G(r_n, r_{n-q}).
  float* glag;
  float* kw;
  const uint8_t* st;      // [P][Kt][2] set kinds (APSM_SET_*) or null for hyperslabs
};

// Training launch of n_inst detectors of one shape, all by value (kernel
// arguments; no device allocation, and a captured graph keeps a copy).
// Workgroup b trains detector b: pilots at rx + b * P * M2 and
// sym + b * P * K * 2, model arrays dict[b], alpha[b], w[b], state[b].
struct TrainArgs {
  TrainCommon cm;
  const float* rx;        // [n][P][M2]
  const float* sym;       // [n][P][K][2]
  const uint8_t* st;      // [n][P][K][2] set kinds or null
  float* dict[kMaxTrainBatch];
  float* alpha[kMaxTrainBatch];
  float* w[kMaxTrainBatch];
  int32_t* state[kMaxTrainBatch];
  int n_inst;
  int P, M2, K, cap;
  float c2;
};

struct DetectArgs {
  const float* dict;      // [M2][cap] component-major
  const float* alpha;     // [cap][K]
  const float* w;         // [K][M2]
  const int32_t* state;   // [4], state[0] = entries in use
  int32_t* flags;         // state + 3: APSM_FLAG_DETECT_NONFINITE is ORed in
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

// One detection job of a batched launch (same field names as DetectArgs).
struct DetJob {
  const unsigned char* packed;  // packed model (split-FP16 path)
  const float* w;         // [K][M2]
  const int32_t* state;   // [4]
  int32_t* flags;         // state + 3
  const float* rx;        // [S][M2]
  float* soft;            // [S][K][2] or null
  uint8_t* hard;          // [S][K] or null
  const uint8_t* truth;   // [S][K] or null
  unsigned long long* err;// [K] or null
  int cap, M2, K, S;
  int modulation;
  float c2;
  int variant;            // detect_batch_variant
  int pad;
};

// Launchers: return a hipError_t from the launch.
hipError_t launch_train(const TrainArgs& a, hipStream_t stream);
// Heterogeneous training: workgroup b runs jobs[b] (device table of n jobs,
// each with its variant set by train_variant) with lds_bytes of dynamic LDS
// (the largest train_lds_bytes of the jobs).
bool train_in_table(int M2);              // shapes the table launch holds
int train_variant(int M2, int K, int W, int cap);
size_t train_lds_bytes(int W, int M2, int K, int cap);
hipError_t launch_train_table(const TrainJob* jobs, int n, const TrainCommon& cm, size_t lds_bytes,
                              hipStream_t stream);
// Training from precomputed kernel rows (every shape up to 2M = 128 whose
// dictionary fits 8 register slots per thread, cap <= 4096): the rows are
// written by launch_kernel_rows from the same job table, one workgroup per
// item (job, n0, l0, 0) covering steps n0 .. n0 + kernel_rows_tile_steps() - 1
// and lags l0 .. l0 + kernel_rows_tile_lags() - 1 (max_M2: the largest 2M of
// the jobs), then launch_train_rows trains, workgroup b running jobs[b] with
// the variant train_rows_variant set.
int train_rows_variant(int M2, int K, int cap);   // -1 if the shape is not covered
// Users one rows job may train for this capacity (16, or 4 when the
// coefficients of dict_cap > 4096 slots need 16 register slots per thread):
// detectors with more users train as several jobs of consecutive users.
int train_rows_max_users(int cap);
size_t train_rows_lds_bytes(int W, int M2, int K);
int kernel_rows_tile_steps();
int kernel_rows_tile_lags();
hipError_t launch_kernel_rows(const TrainJob* jobs, const int4* items, int n_items, int max_M2,
                              const TrainCommon& cm, hipStream_t stream);
hipError_t launch_train_rows(const TrainJob* jobs, int n, const TrainCommon& cm, size_t lds_bytes,
                             hipStream_t stream);
hipError_t launch_detect(const DetectArgs& a, hipStream_t stream);
// Packed model of the detection kernels (split-FP16 layout for 2M <= 64 and
// K <= 8, two-contraction layout otherwise): bytes and the packing launch.
size_t packed_model_bytes(int M2, int K, int cap);
hipError_t launch_pack_model(const float* dict, const float* alpha, const float* w, const int32_t* state, int cap,
                             int M2, int K, void* packed, hipStream_t stream);

// One model to pack in a batched packing launch; variant =
// detect_batch_variant(M2, K) for the split-FP16 (VALU-coefficient) layout,
// unused for the two-contraction layout.
struct PackJob {
  const float* dict;
  const float* alpha;
  const float* w;
  const int32_t* state;
  unsigned char* packed;
  int cap, M2, K, variant;
};
// Packs jobs[0..n) (device table) in the split-FP16 layout, max_cap the
// largest capacity among them.
hipError_t launch_pack_model_batch(const PackJob* jobs, int n, int max_cap, hipStream_t stream);

// Two-contraction detection (detect_wide.h).  Packing many models in one
// launch pair (max_threads: the largest wide_pack_threads of the jobs) and
// detection of many jobs of one padded width (variant = wide_detect_variant)
// in one launch over (job, item) pairs, item i of a job covering received
// vectors 128 i .. 128 i + 127 (persistent form with ctr as for
// launch_detect_batch).
// Detection kernels: kDetectF16 (split-FP16 distance block, coefficients on
// VALU; 2M <= 64 and K <= 8) and kDetectWide (both contractions on the
// matrix cores; every shape).  Shapes both kernels hold ("dual") carry both
// packed images, the two-contraction one at wide_offset.
enum { kDetectF16 = 0, kDetectWide = 1 };
bool detect_dual(int M2, int K);
int detect_default_kernel(int M2, int K);
size_t wide_offset(int M2, int K, int cap);
hipError_t launch_detect_with(const DetectArgs& a, int kernel, hipStream_t stream);
int wide_pack_threads(int M2, int cap);
int wide_detect_variant(int M2);
int wide_detect_items(int S);
hipError_t launch_pack_wide_batch(const PackJob* jobs, int n, int max_threads, hipStream_t stream);
hipError_t launch_detect_wide_batch(const DetJob* jobs, const int2* items, int n_items, unsigned int* ctr, int grid,
                                    int variant, hipStream_t stream);

// Batched detection.  Jobs whose shape has detect_batch_variant >= 0 run in
// one launch over a global sequence of work items, item i being tile
// items[i].y (64 received vectors) of job items[i].x, ordered by the host
// (most expensive tiles first).  With ctr == null, workgroup b runs item b
// (grid = n_items); otherwise `grid` persistent workgroups claim items in
// order through ctr[0], ctr[1] counts finished workgroups and the last one
// resets both to zero (they must be zero before the first launch and stay
// zero between launches).
int detect_batch_variant(int M2, int K);
int detect_tiles(int S);
int device_cus();
hipError_t launch_detect_batch(const DetJob* jobs, const int2* items, int n_items, unsigned int* ctr,
                               int grid, hipStream_t stream);

// Tuning cache (tune.cpp): host-side, mutex-guarded, keyed by the GPU's
// architecture name and HIP runtime version.  detect_kernel_for gives the
// kernel recorded for a dual shape class (2M padded as the split-FP16
// kernel pads it, K), else detect_default_kernel.
int detect_kernel_for(int M2, int K);
void tune_set_kernel(int M2, int K, int kernel);
bool tune_get_form(uint64_t signature, bool* persistent);
void tune_set_form(uint64_t signature, bool persistent);
void tune_clear();

// Unrolled training and its adjoint.  Instance b's part of the workspace
// starts at ws + b * inst_bytes; the off_* are byte offsets inside it.
struct UnrolledArgs {
  const float* theta;       // [3 + W] sigma, eps, mu, omega[0..W-1]
  const float* rx_pilot;    // [n][P][M2]
  const float* sym_pilot;   // [n][P][K][2]
  const float* rx_val;      // [n][S][M2]
  const float* sym_val;     // [n][S][K][2]
  void* ws;
  size_t inst_bytes;
  size_t off_G, off_D, off_ck, off_st, off_sc, off_tx, off_th, off_adj, off_X, off_fbar, off_lpart, off_spart,
      off_gpart;
  int n, P, T, M2, M2P, K, KP, S, W, WP, passes, E;
  float wl, wg;
  float inv_count;          // 1 / (n * S * K)
};
size_t unrolled_pass_lds(const UnrolledArgs& a);
size_t unrolled_reverse_lds(const UnrolledArgs& a);
hipError_t launch_unrolled_forward(const UnrolledArgs& a, float* loss, hipStream_t stream);
hipError_t launch_unrolled_backward(const UnrolledArgs& a, float* grad, const float* upstream, hipStream_t stream);

// Host helpers of the ABI layer (apsm_abi.cpp), shared with the batch layer.
int hip_status(hipError_t e);              // APSM_OK or APSM_ERR_HIP (text kept)
bool finite_pos(float x);
int check_model(const apsm_model_t* m);
int check_params(const apsm_params_t* p);
void fill_common(const apsm_params_t* p, TrainCommon& cm);
int check_detect_args(int M2, int K, float sigma2, int S, const float* rx, float* soft, uint8_t* hard,
                      int modulation, const uint8_t* truth, int64_t* err_count);
DetectArgs detect_args(const apsm_model_t* model, float sigma2, int S, const float* rx, float* soft,
                       uint8_t* hard, int modulation, const uint8_t* truth, int64_t* err_count);
// apsm_train / apsm_train_batched after the argument checks of the public
// entry points: n_inst detectors of one shape, pilots contiguous per detector.
int train_impl(const apsm_params_t* p, int M2, int K, int P, int n_inst, const float* rx_pilot,
               const float* sym_pilot, const apsm_model_t* models, void* stream);

}  // namespace apsm
