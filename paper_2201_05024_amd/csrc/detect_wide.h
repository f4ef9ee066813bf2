// Detection (Sec. III-B evaluation of the frozen filter) with both
// contractions of the kernel expansion on the matrix cores, for any input
// width 2M <= 128 and up to 16 users.
//
//   f_k(x) = w_k . x + sum_i alpha[i][k] exp(-||x - d_i||^2 / (2 sigma^2))
//
// Stage 1, the distance block: for a block of 32 dictionary entries and a
// tile of 16 real vectors, G = D X^T on v_mfma_f32_16x16x32_f16 (entries as
// rows, vectors as columns, the 2M components as the contraction), each FP32
// operand split into FP16 hi + lo parts and the products hi*hi + lo*hi +
// hi*lo accumulated in FP32 (the dropped lo*lo term is ~2^-22 relative).  The
// row term -||x||^2 / 2 enters as the C operand, so with a per-entry
// -c ||d||^2 the exponent argument is one FMA per kernel value:
//   log2 kappa = fma(acc, 2c 2^-(e_x+e_d), -c ||d||^2),   c = log2(e) / (2 sigma^2).
// Stage 2, the coefficients: F = A^T K on the same instruction, users as
// rows (padded to 16), the 32 entries of the block as the contraction and
// the 16 vectors as columns.  The kernel values leave stage 1 in the
// accumulator layout (lane l: vector l%16, entries 4(l/16)+i of each 16-row
// half of the block), which is the B-operand layout of stage 2 once the 32
// entries are numbered in that order: contraction index 8g + i is entry
// 4g + i for i < 4 and 16 + 4g + (i - 4) otherwise (g = l/16).  The
// coefficients are packed in the same order, so nothing moves between
// lanes.  The kernel values are split into FP16 hi + lo as well (three
// products again).  The linear part w_k . x is a third contraction of the
// same kind on the vectors' operands, once per tile.
//
// Per kernel value the VALU does one FMA, one exp2 and the hi/lo split
// (about 3 instructions); the K coefficient FMAs of a VALU formulation move
// to the matrix cores, which run 6 (2M + 16) FP16 flops per value.
//
// Operands are scaled by powers of two only (exact re-scalings): the
// dictionary by 2^e_d, the coefficients by 2^e_a and the linear weights by
// 2^e_w (fixed when the model is packed) and each wave's tile of vectors by
// 2^e_x, so that the largest magnitude of each lands in [2^12, 2^13) and the
// lo parts stay clear of FP16 subnormals.
//
// Dictionary stages of 64 entries (two blocks) are copied from the packed
// model straight into LDS (global_load_lds_dwordx4), double-buffered: the
// packed layout is the LDS image of each stage.
#pragma once

#include "apsm_internal.h"

namespace apsm {
namespace wide {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kNS = 2;                     // 16-vector tiles per wave
constexpr int kVecPerItem = kWaves * kNS * 16;   // real vectors per work item (128 received vectors)
constexpr int kStage = 64;                 // dictionary entries per LDS stage (two 32-entry blocks)
constexpr int kHeader = 256;               // packed-model header bytes

// Padded input width of the specialisation for 2M = m2.
__host__ __device__ constexpr int m2p_wide(int m2) { return m2 <= 32 ? 32 : m2 <= 64 ? 64 : 128; }

template <int M2P>
struct Geo {
  static constexpr int NB = M2P / 32;          // 32-deep component blocks
  // The stage's entries as MFMA A fragments: per (block, row tile, component
  // block, hi/lo) one KiB, lane l's eight halves at 16 l (one conflict-free
  // ds_read_b128 per wave).
  static constexpr int D_BYTES = 2 * 2 * NB * 2 * 1024;
  static constexpr int A_BYTES = 2 * 2048;     // per block: coefficients^T hi (1 KiB), then lo (1 KiB)
  static constexpr int N_BYTES = 1024;         // squared norms: per block [g][8] floats, padded
  static constexpr int STAGE_BYTES = D_BYTES + A_BYTES + N_BYTES;
  static constexpr int W_BYTES = NB * 2048;    // linear weights: hi (NB KiB), then lo
  static_assert(D_BYTES % 1024 == 0 && STAGE_BYTES % 1024 == 0, "stages in whole KiB");
};

__host__ __device__ inline int stages_of(int cap) { return (cap + kStage - 1) / kStage; }

// Packed model: header (e_d, e_a, e_w, entries in use at packing), the
// linear weights, then the stages.
inline size_t packed_bytes(int M2, int cap) {
  switch (m2p_wide(M2)) {
    case 32: return kHeader + Geo<32>::W_BYTES + (size_t)stages_of(cap) * Geo<32>::STAGE_BYTES;
    case 64: return kHeader + Geo<64>::W_BYTES + (size_t)stages_of(cap) * Geo<64>::STAGE_BYTES;
    default: return kHeader + Geo<128>::W_BYTES + (size_t)stages_of(cap) * Geo<128>::STAGE_BYTES;
  }
}

// Contraction index 8g + i of a 32-entry block <-> entry of the block.
__host__ __device__ constexpr int block_entry(int g, int i) { return i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4); }

__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Power-of-two exponent e with 2^e * maxabs in [2^12, 2^13); 0 for zero or
// non-finite input.
__device__ __forceinline__ int scale_exp(float maxabs) {
  if (!(maxabs > 0.0f) || !__builtin_isfinite(maxabs)) return 0;
  int ex;
  frexpf(maxabs, &ex);
  return 13 - ex;
}

__device__ __forceinline__ void split_f16(float v, _Float16& hi, _Float16& lo) {
#pragma clang fp contract(off)
  hi = (_Float16)v;
  lo = (_Float16)(v - (float)hi);
}

typedef __attribute__((address_space(1))) void global_void;
typedef __attribute__((address_space(3))) void lds_void;

// Copy of stage s of the packed model into LDS (1 KiB per wave instruction).
// Asynchronous: stage_wait() before the barrier that publishes it.
template <int M2P>
__device__ __forceinline__ void stage_async(const unsigned char* packed, int s, unsigned char* st, int wave,
                                            int lane) {
  using G = Geo<M2P>;
  constexpr int NK = G::STAGE_BYTES / 1024;
  const unsigned char* src = packed + kHeader + G::W_BYTES + (size_t)s * G::STAGE_BYTES;
#pragma unroll
  for (int u = 0; u < (NK + kWaves - 1) / kWaves; ++u) {
    const int blk = u * kWaves + wave;         // wave-uniform
    if (blk < NK)
      __builtin_amdgcn_global_load_lds((global_void*)(src + blk * 1024 + lane * 16), (lds_void*)(st + blk * 1024),
                                       16, 0, 0);
  }
}

// s_waitcnt vmcnt(0), other counters left open.
__device__ __forceinline__ void stage_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ floatx4 mfma(const half8& a, const half8& b, const floatx4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Detection of work item `item` (received vectors item * kVecPerItem / 2 ..)
// by the whole workgroup.  A is DetectArgs or DetJob (same field names);
// buf0 and buf1 are two distinct LDS arrays of Geo<M2P>::STAGE_BYTES bytes
// each (16-byte aligned), the double buffer of dictionary stages, werr 16
// counters.  A workgroup may run items back to back on the same LDS when a
// barrier separates them.
template <int M2P, class A>
__device__ __forceinline__ void detect_wide_tile(const A& a, const unsigned char* packed, int item,
                                                 unsigned char* buf0, unsigned char* buf1, unsigned int* werr) {
  using G = Geo<M2P>;
  constexpr int NB = G::NB, NS = kNS;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = lane & 15, g = lane >> 4;
  const int M2 = a.M2, M = a.M2 / 2, K = a.K;
  int D = __builtin_amdgcn_readfirstlane(a.state[0]);
  D = D < 0 ? 0 : (D > a.cap ? a.cap : D);
  const int* hdr = reinterpret_cast<const int*>(packed);
  const int e_d = __builtin_amdgcn_readfirstlane(hdr[0]);
  const int e_a = __builtin_amdgcn_readfirstlane(hdr[1]);
  const int e_w = __builtin_amdgcn_readfirstlane(hdr[2]);
  if (tid < 16) werr[tid] = 0;

  // ---- the wave's tiles: B operands of its 16 vectors (vector col holds
  // components 32 j + 8 g + i), r2 = [Im; -Re] formed at load time
  half8 xh[NS][NB], xl[NS][NB];
  floatx4 cinit[NS];
  float desc[NS];
  int ex[NS];
  bool bad = false;                        // a non-finite input component or output
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int v = ((item * kWaves + wave) * NS + t) * 16 + col;
    const int smp = v >> 1, part = v & 1;
    const bool valid = smp < a.S;
    const float* x = a.rx + (size_t)(valid ? smp : 0) * M2;
    float xv[NB][8];
    float nrm = 0.0f, mx = 0.0f;
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int m = 32 * jb + 8 * g + i;
        int src = part == 0 ? m : (m < M ? m + M : m - M);
        src = src < M2 ? src : M2 - 1;
        const float sg = (valid && m < M2) ? ((part == 1 && m >= M) ? -1.0f : 1.0f) : 0.0f;
        const float xc = sg * x[src];
        bad |= valid && m < M2 && !__builtin_isfinite(xc);
        xv[jb][i] = xc;
        nrm = fmaf(xc, xc, nrm);
        mx = fmaxf(mx, fabsf(xc));
      }
    nrm += __shfl_xor(nrm, 16);
    nrm += __shfl_xor(nrm, 32);
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) mx = fmaxf(mx, __shfl_xor(mx, s));
    ex[t] = __builtin_amdgcn_readfirstlane(scale_exp(mx));
    const float xsc = ldexpf(1.0f, ex[t]);
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        _Float16 hi, lo;
        split_f16(xv[jb][i] * xsc, hi, lo);
        xh[t][jb][i] = hi;
        xl[t][jb][i] = lo;
      }
    const float ci = ldexpf(-0.5f * nrm, ex[t] + e_d);
    cinit[t] = floatx4{ci, ci, ci, ci};
    desc[t] = uniform_f(ldexpf(2.0f * a.c2, -(ex[t] + e_d)));
  }

  floatx4 acc2[NS], acc2x[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    acc2[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    acc2x[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  const float mc2 = uniform_f(-a.c2);
  const int nst = (D + kStage - 1) / kStage;
  if (nst > 0) stage_async<M2P>(packed, 0, buf0, wave, lane);
  stage_wait();
  __syncthreads();

  // Stage c is read from st while stage c + 1 is copied into nx, the other
  // buffer (last read in stage c - 1, which every wave has left).  The two
  // buffers are distinct LDS arrays and each stage body names them
  // statically (the loop below is unrolled by two), so the compiler can tell
  // that the reads of st do not alias the copy into nx and issues them
  // without first waiting for the copy; with one array split in halves it
  // waits for the whole copy before the stage's first read.
  //
  // At the widest specialisation the copy is waited for at once (before
  // the stage's first read): a full dictionary (8192 entries, 4.85 MB
  // packed) exceeds the 4 MB L2 of an XCD, and the workgroups of an XCD
  // share its stages through L2 only while they walk the dictionary in
  // step.  A workgroup that runs ahead of the others, whose copy misses to
  // HBM, then waits for it, which keeps them in step: measured on 16
  // detectors in one launch, 62 GB fetched from HBM against 296 GB with the
  // copy overlapped (216 GB with the copy started halfway through the
  // stage), for 2 % more time.  Narrower dictionaries fit L2; their copy
  // overlaps the stage.
  constexpr bool kCopySync = M2P == 128;
  auto stage = [&](const unsigned char* st, unsigned char* nx, int c) {
    if (c + 1 < nst) stage_async<M2P>(packed, c + 1, nx, wave, lane);
    if (kCopySync) stage_wait();
    // The A fragments of each (row tile, component block) group are read
    // one group ahead (two register buffers), so that the LDS latency of a
    // group is covered by the previous group's matrix instructions.
    constexpr int NG = 2 * NB;               // (row tile, component block) groups per 32-entry block
    half8 pdh[2], pdl[2];
    auto load_group = [&](int blk, int gi, int buf) {
      const int rt = gi / NB, jb = gi % NB;
      const unsigned char* fr = st + (((blk * 2 + rt) * NB + jb) * 2) * 1024 + lane * 16;
      pdh[buf] = *reinterpret_cast<const half8*>(fr);
      pdl[buf] = *reinterpret_cast<const half8*>(fr + 1024);
    };
    load_group(0, 0, 0);
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const float* nb = reinterpret_cast<const float*>(st + G::D_BYTES + G::A_BYTES + blk * 128) + 8 * g;
      const floatx4 n0 = *reinterpret_cast<const floatx4*>(nb);
      const floatx4 n1 = *reinterpret_cast<const floatx4*>(nb + 4);
      const half8 ah = *reinterpret_cast<const half8*>(st + G::D_BYTES + blk * 2048 + lane * 16);
      const half8 al = *reinterpret_cast<const half8*>(st + G::D_BYTES + blk * 2048 + 1024 + lane * 16);
      floatx4 acc1[NS][2];
#pragma unroll
      for (int gi = 0; gi < NG; ++gi) {
        const int cur = (blk * NG + gi) & 1;
        if (gi + 1 < NG) load_group(blk, gi + 1, cur ^ 1);
        else if (blk == 0) load_group(1, 0, cur ^ 1);
        const int rt = gi / NB, jb = gi % NB;
        const half8 dh = pdh[cur], dl = pdl[cur];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          floatx4 c0 = jb == 0 ? cinit[t] : acc1[t][rt];
          c0 = mfma(dh, xh[t][jb], c0);
          c0 = mfma(dl, xh[t][jb], c0);
          acc1[t][rt] = mfma(dh, xl[t][jb], c0);
        }
      }
      const float cn[8] = {mc2 * n0[0], mc2 * n0[1], mc2 * n0[2], mc2 * n0[3],
                           mc2 * n1[0], mc2 * n1[1], mc2 * n1[2], mc2 * n1[3]};
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        float kap[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
          kap[i] = __builtin_amdgcn_exp2f(fmaf(acc1[t][i >> 2][i & 3], desc[t], cn[i]));
        half8 kh, kl;
#pragma unroll
        for (int i = 0; i < 8; i += 2) {
          const float2v kv = {kap[i], kap[i + 1]};
          const half2v hv = __builtin_convertvector(kv, half2v);
          const float2v rv = {kap[i] - (float)hv[0], kap[i + 1] - (float)hv[1]};
          const half2v lv = __builtin_convertvector(rv, half2v);
          kh[i] = hv[0];
          kh[i + 1] = hv[1];
          kl[i] = lv[0];
          kl[i + 1] = lv[1];
        }
        acc2[t] = mfma(ah, kh, acc2[t]);
        acc2x[t] = mfma(ah, kl, acc2x[t]);
        acc2x[t] = mfma(al, kh, acc2x[t]);
      }
    }
    stage_wait();
    __syncthreads();
  };
  for (int c = 0; c < nst; c += 2) {
    stage(buf0, buf1, c);
    if (c + 1 < nst) stage(buf1, buf0, c + 1);
  }

  // ---- linear part (third contraction), outputs, decisions
  const half8* wp = reinterpret_cast<const half8*>(packed + kHeader);
  half8 wh[NB], wl[NB];
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) {
    wh[jb] = wp[jb * 64 + lane];
    wl[jb] = wp[NB * 64 + jb * 64 + lane];
  }
  const float sa = ldexpf(1.0f, -e_a);
  const int bits = a.modulation >> 1;              // per axis: 1 (QPSK) or 2 (16-QAM)
  const bool has_err = __builtin_amdgcn_readfirstlane((int)(a.err != nullptr)) != 0;
  // vector stores of the outputs: rows of 2K floats (K even) from a 16-byte
  // aligned base start 16-byte aligned; rows of K labels (K a multiple of 4)
  // from a 4-byte aligned base start 4-byte aligned
  const bool vec_soft = (K % 2 == 0) && (reinterpret_cast<uintptr_t>(a.soft) & 15) == 0;
  const bool vec_hard = (K % 4 == 0) && (reinterpret_cast<uintptr_t>(a.hard) & 3) == 0;
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    floatx4 accl = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) {
      accl = mfma(wh[jb], xh[t][jb], accl);
      accl = mfma(wl[jb], xh[t][jb], accl);
      accl = mfma(wh[jb], xl[t][jb], accl);
    }
    const float sl = ldexpf(1.0f, -(e_w + ex[t]));
    const int v = ((item * kWaves + wave) * NS + t) * 16 + col;
    const int smp = v >> 1, part = v & 1;
    const bool valid = smp < a.S;
    float vals[4];
    unsigned int labels = 0;                     // users 4g .. 4g + 3, one byte each
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * g + i;
      const bool kval = k < K;
      const float val = fmaf(accl[i], sl, (acc2[t][i] + acc2x[t][i]) * sa);
      vals[i] = val;
      bad |= valid && kval && !__builtin_isfinite(val);
      if (a.modulation) {
        int idx;
        if (bits == 1) {
          idx = val >= 0.0f ? 1 : 0;
        } else {
          const float th = 0.63245553203367586640f;  // 2 / sqrt(10)
          idx = (val >= -th) + (val >= 0.0f) + (val >= th);
        }
        const int gr = idx ^ (idx >> 1);
        const int other = __shfl_xor(gr, 1);       // the lane holding the other part of this sample
        const int label = part == 0 ? ((gr << bits) | other) : ((other << bits) | gr);
        labels |= (unsigned int)(label & 0xff) << (8 * i);
        if (part == 0 && valid && kval && has_err && label != a.truth[(size_t)smp * K + k])
          atomicAdd(&werr[k], 1u);
      }
    }
    // Soft outputs: lanes col and col ^ 1 hold the two parts of a sample, so
    // each writes two users x two parts, 16 contiguous bytes (one store
    // where the row offsets allow it); together the eight lanes of a sample
    // cover its row.
    if (a.soft) {
      float oth[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) oth[i] = __shfl_xor(vals[i], 1);
      const int kb = 4 * g + 2 * part;
      const float q0 = part ? oth[2] : vals[0], q1 = part ? vals[2] : oth[0];
      const float q2 = part ? oth[3] : vals[1], q3 = part ? vals[3] : oth[1];
      if (valid) {
        float* dst = a.soft + ((size_t)smp * K + kb) * 2;
        if (vec_soft && kb + 1 < K) {
          *reinterpret_cast<floatx4*>(dst) = floatx4{q0, q1, q2, q3};
        } else {
          if (kb < K) { dst[0] = q0; dst[1] = q1; }
          if (kb + 1 < K) { dst[2] = q2; dst[3] = q3; }
        }
      }
    }
    if (a.modulation && a.hard && part == 0 && valid) {
      uint8_t* hd = a.hard + (size_t)smp * K + 4 * g;
      if (vec_hard && 4 * g + 3 < K) {
        *reinterpret_cast<unsigned int*>(hd) = labels;
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (4 * g + i < K) hd[i] = (uint8_t)(labels >> (8 * i));
      }
    }
  }
  if (__ballot(bad) != 0 && lane == 0) atomicOr(a.flags, APSM_FLAG_DETECT_NONFINITE);
  if (has_err) {
    __syncthreads();
    if (tid < K && werr[tid]) atomicAdd(a.err + tid, (unsigned long long)werr[tid]);
  }
}

hipError_t launch_pack(const float* dict, const float* alpha, const float* w, const int32_t* state, int cap, int M2,
                       int K, unsigned char* packed, hipStream_t stream);
hipError_t launch_pack_batch(const PackJob* jobs, int n, int max_cap, hipStream_t stream);
hipError_t launch_detect(const DetectArgs& a, hipStream_t stream);

}  // namespace wide
}  // namespace apsm
