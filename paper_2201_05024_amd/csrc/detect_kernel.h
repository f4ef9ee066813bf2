// APSM detection kernel for gfx950 (Sec. III-B): evaluates the frozen filter
//   f_k(x) = w_k^T x + sum_i alpha[i][k] exp(-||x - d_i||^2 / (2 sigma^2))
// on both real vectors r1, r2 of every received sample (Sec. II-D), forms
// g_k = f_k(r1) + i f_k(r2), and optionally decides and counts symbol errors.
//
// Design (one wave = 32 complex samples = 64 real vectors = two 32-column
// MFMA tiles; 4 waves per workgroup):
//  * The sample x d_i inner-product block runs on FP32 MFMA
//    (v_mfma_f32_32x32x2_f32) with the dictionary as the A operand (rows) and
//    the samples as the B operand (columns).  The contraction is augmented by
//    two extra depth terms so that the accumulator directly holds
//        c2 * (2 d.x - ||d||^2 - ||x||^2) = -log2(e) ||x - d||^2 / (2 sigma^2):
//    A row = [2 c2 d, -c2 ||d||^2, 1],  B column = [x, 1, -c2 ||x||^2].
//  * The exp2 and the K coefficient FMAs run on VALU in the accumulator
//    layout: accumulator register r of lane l holds dictionary row
//    8 (r/4) + 4 (l/32) + r%4 and sample column l%32, so a lane accumulates
//    K partial outputs for its one sample column; the two wave halves are
//    summed once at the end.
//  * Dictionary chunks of 64 rows are staged in LDS (pre-scaled, with their
//    norms) once per workgroup and double buffered; each A fragment read from
//    LDS feeds both column tiles.
//  * The sample tile (B fragments) is loaded once into registers and stays
//    there for the whole dictionary sweep; r2 = [Im; -Re] is formed at load
//    time from the stored r1 row.
#pragma once

#include "apsm_internal.h"

namespace apsm {
namespace det {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
template <int M2P>
struct Geo {
  static constexpr int KH = M2P / 2 + 1;             // MFMA depth steps (2 each)
  static constexpr int KHP = (KH + 3) / 4 * 4;       // padded for 16-byte LDS reads
  static constexpr int ASTR = 2 * KHP + 4;           // row stride (floats), = 4 mod 8: conflict-free b128 reads
  static constexpr int CH = M2P >= 128 ? 32 : 64;    // dictionary rows per LDS stage
  static constexpr int TPR = kThreads / CH;          // staging threads per row (4 or 8)
};

// Per-stage LDS: A rows [CH][ASTR] then alpha [CH][K].
template <int M2P, int K>
struct StageLds {
  static constexpr int A = Geo<M2P>::CH * Geo<M2P>::ASTR;
  static constexpr int K4 = (K + 3) / 4 * 4;          // alpha row stride: 16-byte aligned rows
  static constexpr int AL = Geo<M2P>::CH * K4;
  static constexpr int FLOATS = A + AL;
};

// Sum over aligned groups of TPR (4 or 8) lanes.
template <int TPR>
__device__ __forceinline__ float group_sum(float v) {
  v += __builtin_amdgcn_update_dpp(0.0f, v, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
  v += __builtin_amdgcn_update_dpp(0.0f, v, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
  if constexpr (TPR == 8)
    v += __builtin_amdgcn_update_dpp(0.0f, v, 0x141, 0xF, 0xF, false); // row_half_mirror
  return v;
}

// Stage dictionary rows [row0, row0 + CH) into one LDS stage: TPR threads
// per row, pre-scaled by 2 c2, with the two augmentation columns.
template <int M2P, int K>
__device__ __forceinline__ void stage_chunk(float* st, const DetectArgs& a, int row0, int D) {
  using G = Geo<M2P>;
  constexpr int TPR = G::TPR;
  const int t = threadIdx.x;
  const int rr = t / TPR, qq = t % TPR;
  const int row = row0 + rr;
  const bool valid = row < D;
  const float* src = a.dict + (valid ? row : 0);     // component m at src[m * cap]
  float* dst = st + rr * G::ASTR;
  float nrm = 0.0f;
#pragma unroll
  for (int m0 = 0; m0 < M2P; m0 += TPR) {
    const int m = m0 + qq;
    const float v = ((valid && m < a.M2) ? 1.0f : 0.0f) * src[(size_t)(m < a.M2 ? m : 0) * a.cap];
    nrm = fmaf(v, v, nrm);
    dst[(m & 1) * G::KHP + (m >> 1)] = 2.0f * a.c2 * v;
  }
  nrm = group_sum<TPR>(nrm);
  if (qq == 0) dst[M2P / 2] = -a.c2 * nrm;            // depth M2P   (h = 0)
  if (qq == 1) dst[G::KHP + M2P / 2] = 1.0f;          // depth M2P+1 (h = 1)
  float* al = st + StageLds<M2P, K>::A;
  constexpr int K4 = StageLds<M2P, K>::K4;
  for (int e = t; e < G::CH * K4; e += kThreads) {
    const int r = e / K4, k = e - r * K4;
    al[e] = (k < K && row0 + r < D) ? a.alpha[(size_t)(row0 + r) * K + k] : 0.0f;
  }
}

// Waves per SIMD the register budget is sized for: two (256 VGPRs) lets one
// wave's MFMA overlap the other's exp/FMA epilogue; the widest inputs need the
// full 512-register file.
template <int M2P>
constexpr int min_waves() { return M2P >= 128 ? 1 : 2; }

template <int M2P, int K, int NT>
__global__ __launch_bounds__(kThreads, min_waves<M2P>()) void detect_kernel(DetectArgs a) {
  using G = Geo<M2P>;
  constexpr int KH = G::KH;
  constexpr int STAGE = StageLds<M2P, K>::FLOATS;
  __shared__ __attribute__((aligned(16))) float lds[2 * STAGE + K * M2P];
  float* wl = lds + 2 * STAGE;                        // [K][M2P] linear coefficients

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int j = lane & 31, h = lane >> 5;
  const int M2 = a.M2, M = a.M;
  int D = a.state[0];
  D = D < 0 ? 0 : (D > a.cap ? a.cap : D);

  for (int e = tid; e < K * M2P; e += kThreads) {
    const int k = e / M2P, m = e - k * M2P;
    wl[e] = m < M2 ? a.w[k * M2 + m] : 0.0f;
  }

  // ---- B fragments: this lane's column of each column tile
  const int samples_per_wave = 16 * NT;
  const int smp_base = (blockIdx.x * kWaves + wave) * samples_per_wave;
  const int part = j & 1;
  float b[NT][KH];
  int smp[NT];
  bool bad = false;                                   // a non-finite input component or output
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    smp[nt] = smp_base + nt * 16 + (j >> 1);
    const bool valid = smp[nt] < a.S;
    const float* x = a.rx + (size_t)(valid ? smp[nt] : 0) * M2;
    float nrm = 0.0f;
#pragma unroll
    for (int s = 0; s < KH - 1; ++s) {
      const int k = 2 * s + h;
      // r1 = x; r2 = [x_M .. x_{2M-1}, -x_0 .. -x_{M-1}]: one unconditional
      // (clamped) load per component keeps this loop straight-line code.
      int src = part == 0 ? k : (k < M ? k + M : k - M);
      src = src < M2 ? src : M2 - 1;
      const float sgn = (valid && k < M2) ? ((part == 1 && k >= M) ? -1.0f : 1.0f) : 0.0f;
      const float v = sgn * x[src];
      bad |= valid && k < M2 && !__builtin_isfinite(v);
      b[nt][s] = v;
      nrm = fmaf(v, v, nrm);
    }
    nrm += __shfl_xor(nrm, 32);
    b[nt][KH - 1] = h == 0 ? 1.0f : -a.c2 * nrm;
  }

  float acc_k[NT][K];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int k = 0; k < K; ++k) acc_k[nt][k] = 0.0f;

  constexpr int CH = G::CH;
  const int nchunks = (D + CH - 1) / CH;
  if (nchunks > 0) stage_chunk<M2P, K>(lds, a, 0, D);
  __syncthreads();

  for (int c = 0; c < nchunks; ++c) {
    const float* st = lds + (c & 1) * STAGE;
    const float* al = st + StageLds<M2P, K>::A;
#pragma unroll 1
    for (int rt = 0; rt < CH / 32; ++rt) {
      // A fragment: row rt*32 + j, depth 2 s + h  ->  contiguous in LDS.
      const float* arow = st + (rt * 32 + j) * G::ASTR + h * G::KHP;
      floatx16 acc[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[nt] = floatx16{};
#pragma unroll
      for (int s0 = 0; s0 < KH; s0 += 4) {
        const floatx4 v4 = *reinterpret_cast<const floatx4*>(arow + s0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (s0 + u < KH) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
              acc[nt] = __builtin_amdgcn_mfma_f32_32x32x2f32(v4[u], b[nt][s0 + u], acc[nt], 0, 0, 0);
          }
        }
      }

      // Epilogue on VALU: rows 8g + 4h + i, i = 0..3, of this row tile.
      constexpr int K4 = StageLds<M2P, K>::K4;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float* ap = al + (rt * 32 + 8 * g + 4 * h + i) * K4;
          float alr[K4];
#pragma unroll
          for (int q = 0; q < K4; q += 4) {
            floatx4 v4 = *reinterpret_cast<const floatx4*>(ap + q);
            alr[q] = v4[0]; alr[q + 1] = v4[1]; alr[q + 2] = v4[2]; alr[q + 3] = v4[3];
          }
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const float kap = __builtin_amdgcn_exp2f(acc[nt][4 * g + i]);
#pragma unroll
            for (int k = 0; k < K; ++k) acc_k[nt][k] = fmaf(alr[k], kap, acc_k[nt][k]);
          }
        }
      }
    }
    if (c + 1 < nchunks) stage_chunk<M2P, K>(lds + ((c + 1) & 1) * STAGE, a, (c + 1) * CH, D);
    __syncthreads();
  }

  // ---- linear part, sum of the two wave halves, outputs
  const bool has_err = a.err != nullptr;
  const int bits = a.modulation >> 1;                 // per axis: 1 (QPSK) or 2 (16-QAM)
  __shared__ unsigned int werr[K];                    // workgroup error counts
  if (tid < K) werr[tid] = 0;
  __syncthreads();
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const bool valid = smp[nt] < a.S;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      float lin = 0.0f;
#pragma unroll
      for (int s = 0; s < KH - 1; ++s) lin = fmaf(wl[k * M2P + 2 * s + h], b[nt][s], lin);
      float v = acc_k[nt][k] + lin;
      v += __shfl_xor(v, 32);
      bad |= valid && !__builtin_isfinite(v);
      if (a.soft && valid && (k & 1) == h)
        a.soft[((size_t)smp[nt] * a.K + k) * 2 + part] = v;
      if (a.modulation) {
        int idx;
        if (bits == 1) {
          idx = v >= 0.0f ? 1 : 0;
        } else {
          const float t = 0.63245553203367586640f;       // 2 / sqrt(10)
          idx = (v >= -t) + (v >= 0.0f) + (v >= t);
        }
        const int gr = idx ^ (idx >> 1);
        const int other = __shfl_xor(gr, 1);
        const int label = part == 0 ? ((gr << bits) | other) : ((other << bits) | gr);
        if (part == 0 && valid && (k & 1) == h) {
          if (a.hard) a.hard[(size_t)smp[nt] * a.K + k] = (uint8_t)label;
          if (has_err && label != a.truth[(size_t)smp[nt] * a.K + k]) atomicAdd(&werr[k], 1u);
        }
      }
    }
  }
  if (__ballot(bad) != 0 && lane == 0) atomicOr(a.flags, APSM_FLAG_DETECT_NONFINITE);
  if (has_err) {
    __syncthreads();
    if (tid < K && werr[tid]) atomicAdd(a.err + tid, (unsigned long long)werr[tid]);
  }
}

template <int M2P, int K>
hipError_t launch_mk(const DetectArgs& a, hipStream_t stream) {
  constexpr int NT = (M2P >= 128 || K > 8) ? 1 : 2;
  const int per_block = kWaves * 16 * NT;
  const int blocks = (a.S + per_block - 1) / per_block;
  hipLaunchKernelGGL((detect_kernel<M2P, K, NT>), dim3(blocks), dim3(kThreads), 0, stream, a);
  return hipGetLastError();
}

// The FP32 path serves 2M > 64 (every K) and K > 8 (every 2M); smaller
// shapes take the split-FP16 kernels.
template <int M2P>
hipError_t launch_m(const DetectArgs& a, hipStream_t stream) {
  if constexpr (M2P > 64) {
    switch (a.K) {
      case 1: return launch_mk<M2P, 1>(a, stream);
      case 2: return launch_mk<M2P, 2>(a, stream);
      case 3: return launch_mk<M2P, 3>(a, stream);
      case 4: return launch_mk<M2P, 4>(a, stream);
      case 5: return launch_mk<M2P, 5>(a, stream);
      case 6: return launch_mk<M2P, 6>(a, stream);
      case 7: return launch_mk<M2P, 7>(a, stream);
      case 8: return launch_mk<M2P, 8>(a, stream);
      default: break;
    }
  }
  switch (a.K) {
    case 9: return launch_mk<M2P, 9>(a, stream);
    case 10: return launch_mk<M2P, 10>(a, stream);
    case 11: return launch_mk<M2P, 11>(a, stream);
    case 12: return launch_mk<M2P, 12>(a, stream);
    case 13: return launch_mk<M2P, 13>(a, stream);
    case 14: return launch_mk<M2P, 14>(a, stream);
    case 15: return launch_mk<M2P, 15>(a, stream);
    case 16: return launch_mk<M2P, 16>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

// One translation unit per padded input dimension keeps compile units small.
hipError_t launch_detect_m16(const DetectArgs& a, hipStream_t stream);
hipError_t launch_detect_m32(const DetectArgs& a, hipStream_t stream);
hipError_t launch_detect_m64(const DetectArgs& a, hipStream_t stream);
hipError_t launch_detect_m128(const DetectArgs& a, hipStream_t stream);

}  // namespace det
}  // namespace apsm
