// Allocation-free training of one detector from precomputed kernel rows.
//
// The same two launches as the batch path (kernel rows of every pilot step
// against the dictionary entries it sees, then the training kernel reading
// one row per step) and the packing launch, with the job table, the tile
// list and the rows in a static device array of this library instead of a
// caller-provided workspace.  Each GPU the library runs on holds its own copy
// of the array (kScratchBytes) until the process ends; every call on a GPU
// uses that GPU's copy, so calls that overlap in time on one GPU race.
#include <map>
#include <mutex>

#include "apsm_internal.h"

namespace apsm {
namespace {

constexpr size_t kScratchBytes = APSM_NOALLOC_SCRATCH_BYTES;
constexpr size_t kJobBytes = 256;          // the one TrainJob, padded

// The device array.  In host code its name is only a stand-in for the
// symbol: its device address (different on every GPU) comes from
// hipGetSymbolAddress, and only that address is passed to kernels.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
std::map<int, unsigned char*> g_scratch;   // device ordinal -> address of its scratch

// Address of the current device's scratch array, looked up once per device
// (with that device current).
hipError_t scratch_ptr(unsigned char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  auto f = g_scratch.find(dev);
  if (f != g_scratch.end()) {
    *out = f->second;
    return hipSuccess;
  }
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch[dev] = static_cast<unsigned char*>(p);
  *out = static_cast<unsigned char*>(p);
  return hipSuccess;
}

// Job table (one entry) and the rows tiles (job 0, first step, first lag)
// written on the device, so the call copies nothing from host memory.
__global__ void write_job_kernel(TrainJob j, TrainJob* job, int4* items, int n_items, int lag_tiles, int tile_steps,
                                 int tile_lags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *job = j;
  if (i < n_items) items[i] = make_int4(0, (i / lag_tiles) * tile_steps, (i % lag_tiles) * tile_lags, 0);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace
}  // namespace apsm

extern "C" {

int apsm_train_noalloc(const apsm_params_t* p, int M2, int K, int P, const float* rx_pilot, const float* sym_pilot,
                       const apsm_model_t* model, void* stream) {
  using namespace apsm;
  if (int rc = check_params(p)) return rc;
  if (p->set_types) return APSM_ERR_UNSUPPORTED;
  if (p->init == APSM_INIT_CONTINUE) return APSM_ERR_UNSUPPORTED;   // kernel rows cover the pilots only
  if (!rx_pilot || !sym_pilot || !model) return APSM_ERR_INVALID_ARG;
  if (P < 1 || M2 < 2 || (M2 & 1) || K < 1) return APSM_ERR_SHAPE;
  if (M2 > APSM_MAX_M2 || K > APSM_MAX_K) return APSM_ERR_UNSUPPORTED;
  if ((long long)P * 2 > (long long)INT32_MAX / 2) return APSM_ERR_UNSUPPORTED;
  if (int rc = check_model(model)) return rc;
  if (model->M2 != M2 || model->K != K || model->dict_cap != p->dict_cap) return APSM_ERR_SHAPE;
  const int cap = p->dict_cap, W = p->window, T = 2 * P;
  const int variant = train_rows_variant(M2, K, cap);
  if (variant < 0 || cap > 4096) return APSM_ERR_UNSUPPORTED;
  const int ts = kernel_rows_tile_steps(), tl = kernel_rows_tile_lags();
  const long long lag_tiles = (cap + tl - 1) / tl, step_tiles = (T + ts - 1) / ts;
  const long long n_items = lag_tiles * step_tiles;
  const size_t off_items = kJobBytes;
  const size_t off_rows = align256(off_items + (size_t)n_items * sizeof(int4));
  const size_t need = off_rows + (size_t)T * (size_t)(cap + W) * sizeof(float);
  if (n_items > INT32_MAX || need > kScratchBytes) return APSM_ERR_WORKSPACE;

  hipStream_t s = (hipStream_t)stream;
  unsigned char* base = nullptr;
  if (hipError_t e = scratch_ptr(&base); e != hipSuccess) return hip_status(e);

  TrainCommon cm{};
  fill_common(p, cm);
  TrainJob j{};
  j.rx = rx_pilot;
  j.sym = sym_pilot;
  j.dict = model->dict;
  j.alpha = model->alpha;
  j.w = model->w;
  j.state = model->state;
  j.P = P;
  j.M2 = M2;
  j.K = K;
  j.Kt = K;
  j.k0 = 0;
  j.cap = cap;
  j.c2 = kLog2e / (2.0f * p->sigma2);
  j.variant = variant;
  j.glag = reinterpret_cast<float*>(base + off_rows);
  j.kw = j.glag + (size_t)T * cap;
  TrainJob* job = reinterpret_cast<TrainJob*>(base);
  int4* items = reinterpret_cast<int4*>(base + off_items);

  const int threads = 256, blocks = (int)((n_items + threads - 1) / threads);
  hipLaunchKernelGGL(write_job_kernel, dim3(blocks), dim3(threads), 0, s, j, job, items, (int)n_items,
                     (int)lag_tiles, ts, tl);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_kernel_rows(job, items, (int)n_items, M2, cm, s);
  if (e == hipSuccess) e = launch_train_rows(job, 1, cm, train_rows_lds_bytes(W, M2, K), s);
  if (e == hipSuccess)
    e = launch_pack_model(model->dict, model->alpha, model->w, model->state, cap, M2, K, model->packed, s);
  return hip_status(e);
}

}  // extern "C"
