// Batched detection (Sec. III-B evaluation of many frozen filters at once):
// one launch over the tiles of many detectors of different shapes (user
// count K, input dimension 2M, dictionary size).  Each tile runs the
// split-FP16 tile body specialised for its detector's (2M, K), chosen by a
// switch on the job's variant, so a single function holds every
// specialisation and the LDS of the largest.
//
// Work items are (job, tile) pairs in an order the host fixes (most
// expensive tiles first).  In the persistent form a grid sized to the chip
// claims them one at a time from an atomic counter, so expensive tiles start
// first and the short ones fill the tail; in the plain form workgroup b runs
// item b and the hardware dispatcher hands out workgroups in that same order.
#include "detect_f16.h"

namespace apsm {
namespace f16 {
namespace {

// variant = 8 * (M2P / 16 == 1 ? 0 : M2P == 32 ? 1 : 2) + K - 1
#define APSM_F16_VARIANTS_M(X, base, M2P)                                           \
  X(base + 0, M2P, 1) X(base + 1, M2P, 2) X(base + 2, M2P, 3) X(base + 3, M2P, 4)   \
  X(base + 4, M2P, 5) X(base + 5, M2P, 6) X(base + 6, M2P, 7) X(base + 7, M2P, 8)
#define APSM_F16_VARIANTS(X) \
  APSM_F16_VARIANTS_M(X, 0, 16) APSM_F16_VARIANTS_M(X, 8, 32) APSM_F16_VARIANTS_M(X, 16, 64)

// LDS of the largest specialisation (the 2M <= 32 ones stage 128 entries;
// both parts grow with K)
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kBatchStage =
    cmax(cmax(Geo<16, 8>::STAGE_BYTES, Geo<32, 8>::STAGE_BYTES), Geo<64, 8>::STAGE_BYTES);
constexpr int kBatchSide = cmax(cmax(side_lds_bytes<16, 8>(), side_lds_bytes<32, 8>()), side_lds_bytes<64, 8>());
static_assert(Geo<64, 7>::STAGE_BYTES <= kBatchStage && Geo<32, 7>::STAGE_BYTES <= kBatchStage &&
                  side_lds_bytes<64, 7>() <= kBatchSide && side_lds_bytes<32, 7>() <= kBatchSide,
              "LDS bound");

// Values every lane holds alike, moved to scalar registers so that the
// compiler treats the control flow that depends on them (the item loop, the
// switch, the dictionary-chunk loop around the tile's barriers) as uniform,
// as it is: barriers must sit in uniform control flow.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) { return __int_as_float(uni(__float_as_int(v))); }
template <class P>
__device__ __forceinline__ P* uni(P* p) {
  const unsigned long long u = reinterpret_cast<unsigned long long>(p);
  const unsigned long long lo = (unsigned)uni((int)(unsigned)u), hi = (unsigned)uni((int)(unsigned)(u >> 32));
  return reinterpret_cast<P*>(lo | (hi << 32));
}

__device__ __forceinline__ DetJob load_job(const DetJob* p) {
  DetJob d;
  d.packed = uni(p->packed);
  d.w = uni(p->w);
  d.state = uni(p->state);
  d.flags = uni(p->flags);
  d.rx = uni(p->rx);
  d.soft = uni(p->soft);
  d.hard = uni(p->hard);
  d.truth = uni(p->truth);
  d.err = uni(p->err);
  d.cap = uni(p->cap);
  d.M2 = uni(p->M2);
  d.K = uni(p->K);
  d.S = uni(p->S);
  d.modulation = uni(p->modulation);
  d.c2 = uni(p->c2);
  d.variant = uni(p->variant);
  d.pad = 0;
  return d;
}

__device__ __forceinline__ void run_item(const DetJob* jobs, const int2* items, int item, unsigned char* buf0,
                                         unsigned char* buf1, unsigned char* side, unsigned int* werr) {
  const int jx = uni(items[item].x), tile = uni(items[item].y);
  const DetJob d = load_job(jobs + jx);
  switch (d.variant) {
#define APSM_F16_CASE(id, M2P, K) \
  case id: detect_f16_tile<M2P, K, false>(d, d.packed, tile, buf0, buf1, side, werr); break;
    APSM_F16_VARIANTS(APSM_F16_CASE)
#undef APSM_F16_CASE
    default: break;
  }
}

// Next item of the persistent form: thread 0 claims it, every thread reads it
// between two barriers (so the next claim cannot overwrite it early).
__device__ __forceinline__ int claim(unsigned int* ctr, int* s_item) {
  if (threadIdx.x == 0) *s_item = (int)atomicAdd(ctr, 1u);
  __syncthreads();
  const int item = uni(*s_item);
  __syncthreads();
  return item;
}

__global__ __launch_bounds__(kThreads, 2) void detect_batch_kernel(const DetJob* jobs, const int2* items,
                                                                   int n_items, unsigned int* ctr) {
  __shared__ __attribute__((aligned(16))) unsigned char buf0[kBatchStage];
  __shared__ __attribute__((aligned(16))) unsigned char buf1[kBatchStage];
  __shared__ __attribute__((aligned(16))) unsigned char side[kBatchSide];
  __shared__ unsigned int werr[8];
  __shared__ int s_item;
  if (ctr == nullptr) {
    run_item(jobs, items, blockIdx.x, buf0, buf1, side, werr);
    return;
  }
  for (int item = claim(ctr, &s_item); item < n_items; item = claim(ctr, &s_item))
    run_item(jobs, items, item, buf0, buf1, side, werr);
  if (threadIdx.x == 0) {
    __threadfence();
    // This workgroup's last claim precedes its count; the workgroup that
    // counts last therefore sees every claim done and restores the zeros.
    const unsigned int done = atomicAdd(ctr + 1, 1u);
    if (done == gridDim.x - 1) {
      atomicExch(ctr, 0u);
      atomicExch(ctr + 1, 0u);
    }
  }
}

}  // namespace
}  // namespace f16

int detect_batch_variant(int M2, int K) {
  if (!f16::supported(M2, K)) return -1;
  const int M2P = f16::m2p_f16(M2);
  return 8 * (M2P == 16 ? 0 : M2P == 32 ? 1 : 2) + K - 1;
}

int detect_tiles(int S) { return (S + f16::kWaves * 16 - 1) / (f16::kWaves * 16); }

// Compute units of the current device (256 if it cannot be queried).  The
// persistent form of this kernel runs two workgroups per CU: the
// specialisations use up to 256 VGPRs (two waves per SIMD) and two copies of
// the largest LDS footprint fit a CU.
int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return 256;
  return cus;
}

hipError_t launch_detect_batch(const DetJob* jobs, const int2* items, int n_items, unsigned int* ctr, int grid,
                               hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  const int blocks = ctr ? grid : n_items;
  hipLaunchKernelGGL(f16::detect_batch_kernel, dim3(blocks), dim3(f16::kThreads), 0, stream, jobs, items,
                     n_items, ctr);
  return hipGetLastError();
}

}  // namespace apsm
