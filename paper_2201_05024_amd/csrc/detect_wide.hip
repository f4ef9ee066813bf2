// Packing of a model for the two-contraction detection kernel (detect_wide.h)
// and its launches: one detector per launch, and many detectors of any
// widths in one persistent launch.
//
// Packed image (independent of sigma^2):
//   header   int[4] = {e_d, e_a, e_w, entries in use}, padded to 256 bytes;
//   weights  w_k scaled by 2^e_w as the A operand of the linear contraction:
//            hi halves [jb][g][u][8], then lo halves (u the user, padded to
//            16; component 32 jb + 8 g + i);
//   stages   per 64 entries: the entries (2^e_d d) as the A fragments of
//            the distance contraction, per (32-entry block, 16-entry row
//            tile, 32-component block) a KiB of hi halves then a KiB of lo
//            halves, lane 16 g + r holding components 8 g .. 8 g + 7 of the
//            tile's row r (the LDS image: one conflict-free ds_read_b128
//            per wave and fragment),
//            per 32-entry block the coefficients^T (2^e_a alpha) hi then lo
//            as [g][u][8] in the block's contraction order, then the squared
//            norms ||d||^2 (unscaled FP32) per block as [g][8], padded to 1 KiB.
// Entries at or past the ones in use are zero rows with zero coefficients.
#include "detect_wide.h"

namespace apsm {
namespace wide {
namespace {

template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ int entries_in_use(const int32_t* state, int cap) {
  int D = gmem(state)[0];
  return D < 0 ? 0 : (D > cap ? cap : D);
}

// One workgroup of 1024 threads: header = {e_d, e_a, e_w, D}, each exponent
// placing the largest magnitude of its array in [2^12, 2^13).
__device__ __forceinline__ void scale_body(const float* dict, const float* alpha, const float* w, const int32_t* state,
                                           int cap, int M2, int K, int* header, float* red) {
  const int D = entries_in_use(state, cap);
  float md = 0.0f, ma = 0.0f, mw = 0.0f;
  for (int c = 0; c < M2; ++c)
    for (int i = threadIdx.x; i < D; i += blockDim.x) md = fmaxf(md, fabsf(gmem(dict)[(size_t)c * cap + i]));
  for (int i = threadIdx.x; i < D * K; i += blockDim.x) ma = fmaxf(ma, fabsf(gmem(alpha)[i]));
  for (int i = threadIdx.x; i < K * M2; i += blockDim.x) mw = fmaxf(mw, fabsf(gmem(w)[i]));
  float* r0 = red;
  float* r1 = red + 1024;
  float* r2 = red + 2048;
  r0[threadIdx.x] = md;
  r1[threadIdx.x] = ma;
  r2[threadIdx.x] = mw;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      r0[threadIdx.x] = fmaxf(r0[threadIdx.x], r0[threadIdx.x + s]);
      r1[threadIdx.x] = fmaxf(r1[threadIdx.x], r1[threadIdx.x + s]);
      r2[threadIdx.x] = fmaxf(r2[threadIdx.x], r2[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    header[0] = scale_exp(r0[0]);
    header[1] = scale_exp(r1[0]);
    header[2] = scale_exp(r2[0]);
    header[3] = D;
  }
}

__global__ __launch_bounds__(1024) void scale_kernel(const float* dict, const float* alpha, const float* w,
                                                     const int32_t* state, int cap, int M2, int K, int* header) {
  __shared__ float red[3 * 1024];
  scale_body(dict, alpha, w, state, cap, M2, K, header, red);
}

// Entry e of the packed model (e < stages * 64), and for e < NB * 64 the
// weight operand slot e.  Reads the exponents the scale pass wrote.
template <int M2P>
__device__ __forceinline__ void pack_entry(const float* dict, const float* alpha, const float* w, const int32_t* state,
                                           int cap, int M2, int K, unsigned char* out, int e) {
  using G = Geo<M2P>;
  constexpr int NB = G::NB;
  const int nst = stages_of(cap);
  const auto hdr = gmem(reinterpret_cast<const int*>(out));
  if (e < NB * 64) {
    // weight slot (jb, g, u): halves i = 0..7 of component 32 jb + 8 g + i of user u
    const int jb = e >> 6, g = (e >> 4) & 3, u = e & 15;
    const float sc = ldexpf(1.0f, hdr[2]);
    half8 hv, lv;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int m = 32 * jb + 8 * g + i;
      const float v = (u < K && m < M2) ? gmem(w)[(size_t)u * M2 + m] : 0.0f;
      _Float16 hi, lo;
      split_f16(v * sc, hi, lo);
      hv[i] = hi;
      lv[i] = lo;
    }
    auto wp = gmem(reinterpret_cast<half8*>(out + kHeader));
    wp[e] = hv;
    wp[NB * 64 + e] = lv;
  }
  if (e >= nst * kStage) return;
  const int D = entries_in_use(state, cap);
  const bool valid = e < D && e < cap;
  const int s = e / kStage, r = e % kStage, blk = r / 32, q = r % 32;
  unsigned char* st = out + kHeader + G::W_BYTES + (size_t)s * G::STAGE_BYTES;
  // the entry's A fragments, eight halves at a time (16-byte stores): entry
  // q of block blk is row q % 16 of row tile q / 16; components 32 jb + 8 g
  // + 0..7 go to lane 16 g + q % 16 of fragment (blk, tile, jb)
  const float scd = ldexpf(1.0f, hdr[0]);
  const int rt = q >> 4, rc = q & 15;
  float n = 0.0f;
#pragma unroll
  for (int m0 = 0; m0 < M2P; m0 += 8) {
    half8 hv, lv;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int m = m0 + v;
      const float d = (valid && m < M2) ? gmem(dict)[(size_t)m * cap + e] : 0.0f;
      n = fmaf(d, d, n);
      _Float16 hi, lo;
      split_f16(d * scd, hi, lo);
      hv[v] = hi;
      lv[v] = lo;
    }
    const int jb = m0 >> 5, gq = (m0 >> 3) & 3;
    auto fr = gmem(reinterpret_cast<half8*>(st + (((blk * 2 + rt) * NB + jb) * 2) * 1024));
    fr[gq * 16 + rc] = hv;
    fr[64 + gq * 16 + rc] = lv;
  }
  // contraction position of this entry in its block: entry 4 g + i (i < 4)
  // or 16 + 4 g + (i - 4)
  const int g = (q & 15) >> 2, i = (q & 3) + (q >= 16 ? 4 : 0);
  const float sca = ldexpf(1.0f, hdr[1]);
  auto ahi = gmem(reinterpret_cast<_Float16*>(st + G::D_BYTES + blk * 2048));
  auto alo = gmem(reinterpret_cast<_Float16*>(st + G::D_BYTES + blk * 2048 + 1024));
  for (int u = 0; u < 16; ++u) {
    const float a = (valid && u < K) ? gmem(alpha)[(size_t)e * K + u] : 0.0f;
    _Float16 hi, lo;
    split_f16(a * sca, hi, lo);
    ahi[(g * 16 + u) * 8 + i] = hi;
    alo[(g * 16 + u) * 8 + i] = lo;
  }
  gmem(reinterpret_cast<float*>(st + G::D_BYTES + G::A_BYTES))[blk * 32 + g * 8 + i] = n;
}

template <int M2P>
__global__ __launch_bounds__(256) void pack_kernel(const float* dict, const float* alpha, const float* w,
                                                   const int32_t* state, int cap, int M2, int K, unsigned char* out) {
  pack_entry<M2P>(dict, alpha, w, state, cap, M2, K, out, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(1024) void scale_batch_kernel(const PackJob* jobs) {
  __shared__ float red[3 * 1024];
  const PackJob j = jobs[blockIdx.x];
  scale_body(j.dict, j.alpha, j.w, j.state, j.cap, j.M2, j.K, reinterpret_cast<int*>(j.packed), red);
}

__global__ __launch_bounds__(256) void pack_batch_kernel(const PackJob* jobs) {
  const PackJob j = jobs[blockIdx.y];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  switch (m2p_wide(j.M2)) {
    case 32: pack_entry<32>(j.dict, j.alpha, j.w, j.state, j.cap, j.M2, j.K, j.packed, e); break;
    case 64: pack_entry<64>(j.dict, j.alpha, j.w, j.state, j.cap, j.M2, j.K, j.packed, e); break;
    default: pack_entry<128>(j.dict, j.alpha, j.w, j.state, j.cap, j.M2, j.K, j.packed, e); break;
  }
}

// Threads the entry pass needs: every entry of the padded capacity and every
// weight slot.
int pack_threads(int M2, int cap) {
  const int NB = m2p_wide(M2) / 32;
  const int n = stages_of(cap) * kStage;
  return n > NB * 64 ? n : NB * 64;
}

// ---- detection launches

template <int M2P>
__global__ __launch_bounds__(kThreads) void detect_wide_kernel(DetectArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned char buf0[Geo<M2P>::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) unsigned char buf1[Geo<M2P>::STAGE_BYTES];
  __shared__ unsigned int werr[16];
  detect_wide_tile<M2P>(a, a.packed, blockIdx.x, buf0, buf1, werr);
}

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

__device__ __forceinline__ int claim(unsigned int* ctr, int* s_item) {
  if (threadIdx.x == 0) *s_item = (int)atomicAdd(ctr, 1u);
  __syncthreads();
  const int item = uni(*s_item);
  __syncthreads();
  return item;
}

// Many detectors of one padded width in one launch.  Persistent form (ctr
// != null): workgroups claim items in list order; the last one to finish
// restores the counters to zero.  Plain form: workgroup b runs item b.
// Waves per SIMD the register budget is sized for: four for the 32-wide
// specialisation (two workgroups per CU, at most 128 VGPRs), two for the
// wider ones.
template <int M2P>
constexpr int batch_waves_per_simd() { return M2P == 32 ? 4 : 2; }

template <int M2P>
__global__ __launch_bounds__(kThreads, batch_waves_per_simd<M2P>()) void detect_wide_batch_kernel(
    const DetJob* jobs, const int2* items, int n_items, unsigned int* ctr) {
  __shared__ __attribute__((aligned(16))) unsigned char buf0[Geo<M2P>::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) unsigned char buf1[Geo<M2P>::STAGE_BYTES];
  __shared__ unsigned int werr[16];
  __shared__ int s_item;
  const bool persistent = ctr != nullptr;
  // one call site of the tile body (the loop runs once in the plain form)
  int item = persistent ? claim(ctr, &s_item) : (int)blockIdx.x;
  while (item < n_items) {
    const int jx = uni(items[item].x), tile = uni(items[item].y);
    const DetJob d = load_job(jobs + jx);
    detect_wide_tile<M2P>(d, d.packed, tile, buf0, buf1, werr);
    if (!persistent) break;
    item = claim(ctr, &s_item);
  }
  if (!persistent) return;
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned int done = atomicAdd(ctr + 1, 1u);
    if (done == gridDim.x - 1) {
      atomicExch(ctr, 0u);
      atomicExch(ctr + 1, 0u);
    }
  }
}

}  // namespace

// Two launches in stream order: the entry pass reads the exponents the scale
// pass writes.
hipError_t launch_pack(const float* dict, const float* alpha, const float* w, const int32_t* state, int cap, int M2,
                       int K, unsigned char* packed, hipStream_t stream) {
  hipLaunchKernelGGL(scale_kernel, dim3(1), dim3(1024), 0, stream, dict, alpha, w, state, cap, M2, K,
                     reinterpret_cast<int*>(packed));
  const int blocks = (pack_threads(M2, cap) + 255) / 256;
  switch (m2p_wide(M2)) {
    case 32: hipLaunchKernelGGL(pack_kernel<32>, dim3(blocks), dim3(256), 0, stream, dict, alpha, w, state, cap, M2, K, packed); break;
    case 64: hipLaunchKernelGGL(pack_kernel<64>, dim3(blocks), dim3(256), 0, stream, dict, alpha, w, state, cap, M2, K, packed); break;
    default: hipLaunchKernelGGL(pack_kernel<128>, dim3(blocks), dim3(256), 0, stream, dict, alpha, w, state, cap, M2, K, packed); break;
  }
  return hipGetLastError();
}

// max_cap: the largest capacity of the jobs, max over their pack_threads.
hipError_t launch_pack_batch(const PackJob* jobs, int n, int max_threads, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_batch_kernel, dim3(n), dim3(1024), 0, stream, jobs);
  hipLaunchKernelGGL(pack_batch_kernel, dim3((max_threads + 255) / 256, n), dim3(256), 0, stream, jobs);
  return hipGetLastError();
}

hipError_t launch_detect(const DetectArgs& a, hipStream_t stream) {
  const int blocks = (int)(((long long)2 * a.S + kVecPerItem - 1) / kVecPerItem);
  switch (m2p_wide(a.M2)) {
    case 32: hipLaunchKernelGGL(detect_wide_kernel<32>, dim3(blocks), dim3(kThreads), 0, stream, a); break;
    case 64: hipLaunchKernelGGL(detect_wide_kernel<64>, dim3(blocks), dim3(kThreads), 0, stream, a); break;
    default: hipLaunchKernelGGL(detect_wide_kernel<128>, dim3(blocks), dim3(kThreads), 0, stream, a); break;
  }
  return hipGetLastError();
}

}  // namespace wide

int wide_pack_threads(int M2, int cap) { return wide::pack_threads(M2, cap); }
int wide_detect_variant(int M2) { const int p = wide::m2p_wide(M2); return p == 32 ? 0 : p == 64 ? 1 : 2; }
int wide_detect_items(int S) { return (int)(((long long)2 * S + wide::kVecPerItem - 1) / wide::kVecPerItem); }

hipError_t launch_detect_wide_batch(const DetJob* jobs, const int2* items, int n_items, unsigned int* ctr, int grid,
                                    int variant, hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  const int blocks = ctr ? grid : n_items;
  switch (variant) {
    case 0: hipLaunchKernelGGL(wide::detect_wide_batch_kernel<32>, dim3(blocks), dim3(wide::kThreads), 0, stream, jobs, items, n_items, ctr); break;
    case 1: hipLaunchKernelGGL(wide::detect_wide_batch_kernel<64>, dim3(blocks), dim3(wide::kThreads), 0, stream, jobs, items, n_items, ctr); break;
    default: hipLaunchKernelGGL(wide::detect_wide_batch_kernel<128>, dim3(blocks), dim3(wide::kThreads), 0, stream, jobs, items, n_items, ctr); break;
  }
  return hipGetLastError();
}

}  // namespace apsm
