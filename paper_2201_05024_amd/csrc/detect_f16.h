// Detection with split-FP16 MFMA (Sec. III-B evaluation of the frozen filter)
// for inputs 2M <= 64 and K <= 8 users.
//
// The sample x dictionary inner products run on v_mfma_f32_32x32x16_f16 with
// each FP32 operand split into two FP16 parts, v = hi + lo, and the three
// products hi*hi + lo*hi + hi*lo accumulated in FP32.  This keeps about 22
// significant bits per product (the dropped lo*lo term is ~2^-22 relative),
// and, unlike FP32 MFMA, these matrix instructions execute concurrently with
// the VALU work of other waves (exp2 and the coefficient FMAs), which is the
// binding pipe of this kernel.
//
// Both operands are scaled by powers of two only (so the splits are exact
// re-scalings): the dictionary by 2^e_d, fixed when the model is packed, and
// the 16 samples of a wave by a common 2^e_x, so that their largest
// component lands in [2^12, 2^13) and the lo parts stay clear of FP16
// subnormals (for any sample within 2^15 of the largest in its wave; below
// that the lo parts lose bits only far under the products' rounding).  With
// acc = 2^(e_x+e_d) (x.d - ||x||^2 / 2) from the MFMA (the row term enters as
// its C operand), the exponent argument is
//   log2(kappa_G) = fma(acc, 2c 2^-(e_x+e_d), -c ||d||^2),  c = log2(e) / (2 sigma^2),
// with the multiplier the same for the whole wave (a scalar register).
//
// Layout: samples are the MFMA rows (A operand), held in registers for the
// whole dictionary sweep; dictionary entries are the columns (B operand),
// streamed through LDS in chunks of 128 (2M <= 32) or 64 entries from the
// packed model with a plain 16-byte copy that is prefetched one chunk ahead.
// For 2M <= 32, within a chunk the products of the next 32-entry tile are
// issued before the exp2 and coefficient work of the current one, so that
// the matrix cores run them while the VALU works.  Accumulator element r of
// lane l is sample row 8(r/4) + 4(l/32) + r%4 against dictionary column l%32,
// so each lane needs the K coefficients of one dictionary entry per tile and
// keeps 16 x K partial outputs; a reduce-scatter across the 32 columns at the
// end leaves each lane with K/2 finished outputs of one real vector.
#pragma once

#include "apsm_internal.h"

namespace apsm {
namespace f16 {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kPad = 128;                  // packed-model rows are padded to a multiple of this
constexpr int kHeader = 64;                // packed-model header bytes

template <int M2P, int K>
struct Geo {
  static constexpr int CH = M2P <= 32 ? 128 : 64;  // dictionary entries per LDS stage
  static constexpr int CT = CH / 32;               // 32-entry tiles per stage
  // products of the next tile issued ahead of the current tile's VALU work
  // (a second accumulator set: 2M = 64 has no registers to spare for it)
  static constexpr bool PIPE = M2P <= 32;
  static constexpr int NB = M2P / 16;              // 16-deep blocks per segment
  static constexpr int NSTEP = 3 * NB;             // [hi|lo|hi] x [hi|hi|lo]
  static constexpr int BSTR = 2 * M2P + 8;         // packed row: d_hi | d_lo | pad (halves)
  static constexpr int ROW_B = BSTR * 2;           // bytes; dwords = 4 (mod 8): conflict-free b128 reads
  static constexpr int K4 = (K + 3) / 4 * 4;
  static constexpr int CSTR = K4 + 4;              // per-entry floats: K4 coefficients, ||d||^2, pad
  static constexpr int KE = K + (K & 1);           // even user count for the reduce-scatter
  static constexpr int A_BYTES = CH * ROW_B;
  static constexpr int C_BYTES = CH * CSTR * 4;
  static constexpr int STAGE_BYTES = A_BYTES + C_BYTES;
};

// Padded input width of the specialisation that handles 2M = m2: 16, 32 or
// 64.  The packed layout, its size and the kernel dispatch all use this one
// value (a 2M of 40 runs, and is packed, with the 64-wide layout).
__host__ __device__ inline int m2p_f16(int m2) { return m2 <= 16 ? 16 : m2 <= 32 ? 32 : 64; }
__host__ __device__ inline int cap_pad(int cap) { return (cap + kPad - 1) / kPad * kPad; }

inline bool supported(int M2, int K) { return M2 <= 64 && K <= 8; }

// Bytes of the packed model for a supported shape.
inline size_t packed_bytes(int M2, int K, int cap) {
  const int M2P = m2p_f16(M2), K4 = (K + 3) / 4 * 4;
  return kHeader + (size_t)cap_pad(cap) * ((2 * M2P + 8) * 2 + (K4 + 4) * 4);
}

// A float every lane holds alike, in a scalar register (the readfirstlane
// builtin takes and returns int: the bits are moved, not the value converted).
__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ void split_f16(float v, _Float16& hi, _Float16& lo) {
#pragma clang fp contract(off)
  hi = (_Float16)v;
  lo = (_Float16)(v - (float)hi);
}

// Power-of-two exponent e with 2^e * maxabs in [2^12, 2^13); 0 for zero input.
__device__ __forceinline__ int scale_exp(float maxabs) {
  if (!(maxabs > 0.0f)) return 0;
  int ex;
  frexpf(maxabs, &ex);
  return 13 - ex;
}

hipError_t launch_pack_batch(const PackJob* jobs, int n, int max_cap, hipStream_t stream);
hipError_t launch_pack(const float* dict, const float* alpha, const int32_t* state, int cap, int M2,
                       int K, unsigned char* packed, hipStream_t stream);
hipError_t launch_detect_f16_m16(const DetectArgs& a, const unsigned char* packed, hipStream_t stream);
hipError_t launch_detect_f16_m32(const DetectArgs& a, const unsigned char* packed, hipStream_t stream);
hipError_t launch_detect_f16_m64(const DetectArgs& a, const unsigned char* packed, hipStream_t stream);

typedef __attribute__((address_space(1))) void global_void;
typedef __attribute__((address_space(3))) void lds_void;

// Copy of one stage of the packed model (rows row0 .. row0 + CH - 1: their
// halves, then their coefficients) straight from global memory into LDS with
// gfx950's global_load_lds_dwordx4: each lane moves 16 bytes, so one
// instruction of a wave fills a contiguous KiB of the stage.  Asynchronous:
// stage_wait() before the barrier that publishes the stage.
template <int M2P, int K>
__device__ __forceinline__ void stage_async(const unsigned char* packed, int capp, int row0,
                                            unsigned char* st, int wave, int lane) {
  using G = Geo<M2P, K>;
  static_assert(G::A_BYTES % 1024 == 0 && G::C_BYTES % 1024 == 0, "stage sections in whole KiB");
  constexpr int NA = G::A_BYTES / 1024, NC = G::C_BYTES / 1024;
  const unsigned char* srcA = packed + kHeader + (size_t)row0 * G::ROW_B;
  const unsigned char* srcC = packed + kHeader + (size_t)capp * G::ROW_B + (size_t)row0 * G::CSTR * 4;
#pragma unroll
  for (int u = 0; u < (NA + NC + kWaves - 1) / kWaves; ++u) {
    const int blk = u * kWaves + wave;       // wave-uniform
    if (blk < NA) {
      __builtin_amdgcn_global_load_lds((global_void*)(srcA + blk * 1024 + lane * 16),
                                       (lds_void*)(st + blk * 1024), 16, 0, 0);
    } else if (blk < NA + NC) {
      __builtin_amdgcn_global_load_lds((global_void*)(srcC + (blk - NA) * 1024 + lane * 16),
                                       (lds_void*)(st + G::A_BYTES + (blk - NA) * 1024), 16, 0, 0);
    }
  }
}

// Wait for this wave's outstanding global loads (stage copies included):
// s_waitcnt vmcnt(0) with the other counters left open.
__device__ __forceinline__ void stage_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// LDS of one tile: two dictionary stages of STAGE_BYTES each (two distinct
// arrays), and beside them the linear coefficients and each wave's linear
// terms (32 rows x KE users).
template <int M2P, int K>
constexpr int side_lds_bytes() {
  return K * M2P * 4 + kWaves * 32 * Geo<M2P, K>::KE * 4;
}

// Detection of one tile of kWaves * 16 received vectors (vectors tile * 64 ..
// tile * 64 + 63) by the whole workgroup.  ALLOW_PIPE: the caller has the
// registers for the one-tile-ahead products (a function holding every
// specialisation does not).  A is DetectArgs or DetJob (the same
// field names); buf0 and buf1 are two distinct LDS arrays of at least
// Geo<M2P, K>::STAGE_BYTES bytes, side one of side_lds_bytes<M2P, K>()
// bytes (all 16-byte aligned), werr 8 counters.  A workgroup may run tiles
// back to back on the same LDS when a barrier separates them.
template <int M2P, int K, bool ALLOW_PIPE, class A>
__device__ __forceinline__ void detect_f16_tile(const A& a, const unsigned char* packed, int tile,
                                                unsigned char* buf0, unsigned char* buf1, unsigned char* side,
                                                unsigned int* werr) {
  using G = Geo<M2P, K>;
  constexpr int NSTEP = G::NSTEP, NB = G::NB, KE = G::KE, K4 = G::K4, CSTR = G::CSTR;
  float* wl = reinterpret_cast<float*>(side);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  float* lin_w = wl + K * M2P + wave * 32 * KE;     // this wave's linear terms: [32][KE]
  const int j = lane & 31, h = lane >> 5;
  const int M2 = a.M2, M = a.M2 / 2;
  const int capp = cap_pad(a.cap);
  // Entries in use and the dictionary exponent are the same for every lane;
  // in scalar registers they keep the chunk loop (which holds barriers)
  // uniform control flow.
  int D = __builtin_amdgcn_readfirstlane(a.state[0]);
  D = D < 0 ? 0 : (D > a.cap ? a.cap : D);
  const int e_d = __builtin_amdgcn_readfirstlane(reinterpret_cast<const int*>(packed)[0]);

  for (int e = tid; e < K * M2P; e += kThreads) {
    const int k = e / M2P, m = e - k * M2P;
    wl[e] = m < M2 ? a.w[k * M2 + m] : 0.0f;
  }
  if (tid < 8) werr[tid] = 0;

  // ---- A fragments: row j of this wave's tile is sample s0 + j/2, part j%2
  // (r1 for part 0, r2 = [Im; -Re] for part 1); this lane holds components
  // 16 b + 8 h + v of it.
  const int s0 = (tile * kWaves + wave) * 16;
  const int my_smp = s0 + (j >> 1), my_part = j & 1;
  const bool my_valid = my_smp < a.S;
  const float* x = a.rx + (size_t)(my_valid ? my_smp : 0) * M2;
  float xv[M2P / 2];
  float nrm = 0.0f, mx = 0.0f;
  bool bad = false;                        // a non-finite input component or output
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int m = 16 * b + 8 * h + v;
      int src = my_part == 0 ? m : (m < M ? m + M : m - M);
      src = src < M2 ? src : M2 - 1;
      const float sg = (my_valid && m < M2) ? ((my_part == 1 && m >= M) ? -1.0f : 1.0f) : 0.0f;
      const float t = sg * x[src];
      bad |= my_valid && m < M2 && !__builtin_isfinite(t);
      xv[8 * b + v] = t;
      nrm = fmaf(t, t, nrm);
      mx = fmaxf(mx, fabsf(t));
    }
  nrm += __shfl_xor(nrm, 32);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
  const int e_x = __builtin_amdgcn_readfirstlane(scale_exp(mx));
  const float xsc = ldexpf(1.0f, e_x);
  half8 afr[NSTEP];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      _Float16 hi, lo;
      split_f16(xv[8 * b + v] * xsc, hi, lo);
      afr[b][v] = hi;
      afr[NB + b][v] = lo;
      afr[2 * NB + b][v] = hi;
    }
  const float my_cinit = ldexpf(-0.5f * nrm, e_x + e_d);
  const float desc = uniform_f(ldexpf(2.0f * a.c2, -(e_x + e_d)));
  floatx16 cinit;
#pragma unroll
  for (int r = 0; r < 16; ++r) cinit[r] = __shfl(my_cinit, 8 * (r / 4) + 4 * h + (r % 4));

  float acc_k[16][KE];
#pragma unroll
  for (int r = 0; r < 16; ++r)
#pragma unroll
    for (int k = 0; k < KE; ++k) acc_k[r][k] = 0.0f;

  // ---- dictionary sweep
  constexpr int CH = G::CH, CT = G::CT;
  const float mc2 = uniform_f(-a.c2);
  // products of tile ct of a stage: acc = cinit + x.d (split FP16)
  auto products = [&](const _Float16* dh, int ct) {
    const _Float16* brow = dh + (ct * 32 + j) * G::BSTR + 8 * h;
    floatx16 acc = cinit;
#pragma unroll
    for (int s = 0; s < NSTEP; ++s) {
      // B steps: d_hi blocks (paired with x_hi, then x_lo), then d_lo blocks
      const int off = s < NB ? 16 * s : (s < 2 * NB ? 16 * (s - NB) : M2P + 16 * (s - 2 * NB));
      const half8 bv = *reinterpret_cast<const half8*>(brow + off);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(afr[s], bv, acc, 0, 0, 0);
    }
    return acc;
  };
  // exp2 and the coefficient FMAs of tile ct
  auto expand = [&](const float* co, int ct, const floatx16& acc) {
    float cr[CSTR];
    const float* cp = co + (ct * 32 + j) * CSTR;
#pragma unroll
    for (int q = 0; q < CSTR; q += 4) {
      const floatx4 v4 = *reinterpret_cast<const floatx4*>(cp + q);
      cr[q] = v4[0]; cr[q + 1] = v4[1]; cr[q + 2] = v4[2]; cr[q + 3] = v4[3];
    }
    const float coln = mc2 * cr[K4];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float kap = __builtin_amdgcn_exp2f(fmaf(acc[r], desc, coln));
#pragma unroll
      for (int k = 0; k < K; ++k) acc_k[r][k] = fmaf(cr[k], kap, acc_k[r][k]);
    }
  };
  const int nchunks = (D + CH - 1) / CH;
  if (nchunks > 0) stage_async<M2P, K>(packed, capp, 0, buf0, wave, lane);
  stage_wait();
  __syncthreads();

  // ---- linear part w_k . r of this lane's A row (half of its components
  // here, the other half in lane ^ 32: summed by the row-half swap), kept
  // in this wave's LDS rows for the lanes that finish the row.  Only this
  // wave reads them, after its own writes (LDS operations of a wave are
  // processed in order).
  {
    float plin[KE];
#pragma unroll
    for (int k = 0; k < KE; ++k) plin[k] = 0.0f;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 8; ++v)
#pragma unroll
        for (int k = 0; k < K; ++k) plin[k] = fmaf(wl[k * M2P + 16 * b + 8 * h + v], xv[8 * b + v], plin[k]);
#pragma unroll
    for (int k = 0; k < KE; ++k) {
      const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(plin[k]), __float_as_uint(plin[k]),
                                                        false, false);
      plin[k] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
    }
    if (h == 0) {
#pragma unroll
      for (int k = 0; k < KE; ++k) lin_w[j * KE + k] = plin[k];
    }
    __builtin_amdgcn_wave_barrier();
  }
  // Chunk c is read from st while chunk c + 1 is copied into nx, the other
  // buffer (last read in chunk c - 1, which every wave has left).  The two
  // buffers are distinct LDS arrays named statically by each chunk body
  // (the loop below is unrolled by two), so the compiler can tell that the
  // reads of st do not alias the copy and issues them without first waiting
  // for it.
  auto chunk = [&](const unsigned char* st, unsigned char* nx, int c) {
    if (c + 1 < nchunks) stage_async<M2P, K>(packed, capp, (c + 1) * CH, nx, wave, lane);
    const _Float16* dh = reinterpret_cast<const _Float16*>(st);
    const float* co = reinterpret_cast<const float*>(st + G::A_BYTES);
    if constexpr (G::PIPE && ALLOW_PIPE) {
      floatx16 acc = products(dh, 0);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        floatx16 next;
        if (ct + 1 < CT) next = products(dh, ct + 1);
        expand(co, ct, acc);
        if (ct + 1 < CT) acc = next;
      }
    } else {
#pragma unroll 1
      for (int ct = 0; ct < CT; ++ct) expand(co, ct, products(dh, ct));
    }
    stage_wait();
    __syncthreads();
  };
  for (int c = 0; c < nchunks; c += 2) {
    chunk(buf0, buf1, c);
    if (c + 1 < nchunks) chunk(buf1, buf0, c + 1);
  }

  // ---- reduce-scatter over the 32 dictionary columns of each wave half
  float v[16 * KE];
#pragma unroll
  for (int r = 0; r < 16; ++r)
#pragma unroll
    for (int k = 0; k < KE; ++k) v[r * KE + k] = acc_k[r][k];
  // (The DPP lambdas state their float return type: deduced, the builtin's
  // result would be taken as an int.)
  // Five exchange levels between lanes of the same half whose column
  // indices differ by 16 (gfx950 row swap: both halves of a pair move at
  // once), 8 (row_ror:8), 7 (row_half_mirror), 1 and 2 (quad_perm).  Each
  // level keeps half of the values, chosen by one bit of the column index
  // (4, 3, 2, 0, 1 in that order), and adds the partner's copy of them.
  constexpr int N = 16 * KE;
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[N / 2 + i]),
                                                      false, false);
    v[i] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
  }
  auto level = [&](int half, bool upper, auto dpp) {
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const float send = upper ? v[i] : v[half + i];
      const float keep = upper ? v[half + i] : v[i];
      v[i] = keep + dpp(send);
    }
  };
  level(N / 4, (lane & 8) != 0, [](float x) -> float { return __builtin_amdgcn_update_dpp(0.0f, x, 0x128, 0xF, 0xF, false); });
  level(N / 8, (lane & 4) != 0, [](float x) -> float { return __builtin_amdgcn_update_dpp(0.0f, x, 0x141, 0xF, 0xF, false); });
  level(N / 16, (lane & 1) != 0, [](float x) -> float { return __builtin_amdgcn_update_dpp(0.0f, x, 0xB1, 0xF, 0xF, false); });
  level(N / 32, (lane & 2) != 0, [](float x) -> float { return __builtin_amdgcn_update_dpp(0.0f, x, 0x4E, 0xF, 0xF, false); });
  // Lane (j, h) now holds accumulator row r = jj/2 (sample row
  // 8(r/4) + 4h + r%4) for users k0 .. k0 + KE/2 - 1, k0 = (jj%2) KE/2,
  // where jj is j with its bits 0 and 1 exchanged (the order of the levels).
  const int jj = (j & ~3) | ((j & 1) << 1) | ((j >> 1) & 1);
  const int r = jj >> 1;
  const int rho = 8 * (r >> 2) + 4 * h + (r & 3);
  const int smp = s0 + (rho >> 1), part = rho & 1;
  const bool valid = smp < a.S;
  const int k0 = (jj & 1) * (KE / 2);
  float lin[KE / 2];
#pragma unroll
  for (int u = 0; u < KE / 2; ++u) lin[u] = lin_w[rho * KE + k0 + u];
  const int bits = a.modulation >> 1;              // per axis: 1 (QPSK) or 2 (16-QAM)
  // uniform by construction (it guards a barrier)
  const bool has_err = __builtin_amdgcn_readfirstlane((int)(a.err != nullptr)) != 0;
#pragma unroll
  for (int u = 0; u < KE / 2; ++u) {
    const int k = k0 + u;
    const bool kval = k < K;
    const float val = v[u] + lin[u];
    bad |= valid && kval && !__builtin_isfinite(val);
    if (a.soft && valid && kval) a.soft[((size_t)smp * a.K + k) * 2 + part] = val;
    if (a.modulation) {
      int idx;
      if (bits == 1) {
        idx = val >= 0.0f ? 1 : 0;
      } else {
        const float th = 0.63245553203367586640f;  // 2 / sqrt(10)
        idx = (val >= -th) + (val >= 0.0f) + (val >= th);
      }
      const int gr = idx ^ (idx >> 1);
      const int other = __shfl_xor(gr, 1);         // the lane holding the other part of this sample
      const int label = part == 0 ? ((gr << bits) | other) : ((other << bits) | gr);
      if (part == 0 && valid && kval) {
        if (a.hard) a.hard[(size_t)smp * a.K + k] = (uint8_t)label;
        if (has_err && label != a.truth[(size_t)smp * a.K + k]) atomicAdd(&werr[k], 1u);
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
__global__ __launch_bounds__(kThreads, 2) void detect_f16_kernel(DetectArgs a, const unsigned char* packed) {
  __shared__ __attribute__((aligned(16))) unsigned char buf0[Geo<M2P, K>::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) unsigned char buf1[Geo<M2P, K>::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) unsigned char side[side_lds_bytes<M2P, K>()];
  __shared__ unsigned int werr[8];
  detect_f16_tile<M2P, K, true>(a, packed, blockIdx.x, buf0, buf1, side, werr);
}

}  // namespace f16
}  // namespace apsm
