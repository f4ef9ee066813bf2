// APSM training kernel for gfx950: windowed parallel hyperslab projections
// (Sec. II-D, eqn:apsm, eqn:beta) over the real training sequence
// r_{2t} = r1(t), r_{2t+1} = r2(t) of the pilot block.
//
// One workgroup trains one detector; the n-loop runs on the device.  Training
// is serial in n, so the design goal is a short critical path per step with
// two workgroup barriers:
//
//   A  every thread: append r_n to the dictionary ring (FIFO eviction), the
//      kernel row kappa_G(r_n, d_i) over its own dictionary slots, the
//      alpha-weighted partial sums of f_n(r_n), the new row/column of the
//      window Gram matrix K(r_j, r_i) = wL r_j.r_i + wG kappa_G(r_j, r_i),
//      and the kernel values of r_n against the dictionary entries that will
//      be evicted while r_n is still in the window.
//   -- barrier --
//   C  one thread per (window member j, user k): f_n(r_j) (new member: the
//      reduced partial sums plus w_k.r_n; old members: their running value
//      minus the evicted Gaussian term), beta from eqn:beta, c = mu q_j beta.
//   -- barrier --
//   D  running predictions e_i += sum_j c_j K(r_j, r_i) for the members that
//      stay, alpha[slot(j)] += c_j wG (slot owners), w_k += wL sum_j c_j r_j.
//      The two sums over members are small dense contractions (Gram block
//      times coefficients, coefficients times member vectors) and run as
//      16 x 16 tiles of v_mfma_f32_16x16x4_f32; the linear weights stay in
//      the accumulator registers of their tiles for the whole training.
//
// The window predictions are thus updated incrementally (D Gaussian
// evaluations per step instead of |J_n| * D); this is exact up to rounding
// because every change of f is a finite sum of kernel sections whose values
// at the window members are known.  All W projections use the same f_n, as
// eqn:apsm requires.
//
// Dictionary slots are owned round-robin by the threads (slot s by thread
// s % 512).  When cap * M2 fits, each thread keeps its slots' vectors and
// coefficients in registers; otherwise the coefficients live in LDS or, with
// the vectors, in the model buffers.  Training from precomputed kernel rows
// (the batch path) replaces the row evaluation of phase A by one row read.
#include "apsm_internal.h"

namespace apsm {
namespace {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;

// Wave sums of KP values per lane, scattered over the lanes: afterwards
// every lane holds the sum over the wave of v[user_of_lane(lane)].  Each
// exchange level pairs lanes whose indices differ by a fixed xor pattern
// (7 by row_half_mirror, 1 and 2 by quad_perm, 8 by row_ror:8); the lane
// keeps half of its values, adds the partner's matching half and sends the
// other half, so level by level the values per lane halve.  Levels past
// one value per lane add the partner's value whole; the four 16-lane rows
// are then summed by the gfx950 row-swap permutes.
template <int N>
__device__ __forceinline__ void scatter_level(float* v, bool upper, int ctrl) {
#pragma unroll
  for (int j = 0; j < N / 2; ++j) {
    const float keep = upper ? v[j + N / 2] : v[j];
    const float send = upper ? v[j] : v[j + N / 2];
    float got;
    switch (ctrl) {
      case 0x141: got = __builtin_amdgcn_update_dpp(0.0f, send, 0x141, 0xF, 0xF, false); break;
      case 0xB1: got = __builtin_amdgcn_update_dpp(0.0f, send, 0xB1, 0xF, 0xF, false); break;
      case 0x4E: got = __builtin_amdgcn_update_dpp(0.0f, send, 0x4E, 0xF, 0xF, false); break;
      default: got = __builtin_amdgcn_update_dpp(0.0f, send, 0x128, 0xF, 0xF, false); break;
    }
    v[j] = keep + got;
  }
}

__device__ __forceinline__ float cross_rows(float x) {
  const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  x = __uint_as_float(a[0]) + __uint_as_float(a[1]);          // rows r and r ^ 1
  const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(b[0]) + __uint_as_float(b[1]);       // halves
}

// User whose sum lane `lane` holds after wave_sum_scatter<KP>, and whether
// the lane is the one that stores it (one lane per user, all below 16).
template <int KP>
__device__ __forceinline__ int scatter_user(int lane) {
  const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
  if constexpr (KP == 16) return 8 * b2 + 4 * b0 + 2 * b1 + b3;
  else if constexpr (KP == 8) return 4 * b2 + 2 * b0 + b1;
  else return 2 * b2 + b0;
}
template <int KP>
__device__ __forceinline__ bool scatter_writer(int lane) {
  if constexpr (KP == 16) return lane < 16;
  else if constexpr (KP == 8) return lane < 8;
  else return lane < 8 && (lane & 2) == 0;
}

template <int KP>
__device__ __forceinline__ float wave_sum_scatter(float* v, int lane) {
  const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4, b3 = lane & 8;
  scatter_level<KP>(v, b2, 0x141);
  scatter_level<KP / 2>(v, b0, 0xB1);
  float x;
  if constexpr (KP == 4) {
    x = v[0];
    x += __builtin_amdgcn_update_dpp(0.0f, x, 0x4E, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0.0f, x, 0x128, 0xF, 0xF, false);
  } else if constexpr (KP == 8) {
    scatter_level<2>(v, b1, 0x4E);
    x = v[0];
    x += __builtin_amdgcn_update_dpp(0.0f, x, 0x128, 0xF, 0xF, false);
  } else {
    scatter_level<4>(v, b1, 0x4E);
    scatter_level<2>(v, b3, 0x128);
    x = v[0];
  }
  return cross_rows(x);
}

__device__ __forceinline__ float soft_threshold(float x, float eps) {
  float m = fabsf(x) - eps;
  return m > 0.0f ? copysignf(m, x) : 0.0f;
}

// Shared-memory layout, sized at launch from W, K and M2P.  Rings indexed by
// the training index modulo W (or R = W + 1) hold the window members.  The
// rings that phase D reads member by member are stored twice (positions r
// and r + size), so that the L newest members sit at the contiguous
// positions base - L + 1 .. base with base = (n mod size) + size: member q
// is at a constant offset from a per-lane base, with no wrap-around
// arithmetic.
constexpr int CS = 16;   // row stride of the coefficient ring (users KP..15 stay zero)

struct Lds {
  float* gram;   // [R][2R]  K(r_j, r_i) of window members (columns doubled)
  float* evkr;   // [W][W-1] kappa_G(r_j, d_v) for the entries v evicted while j is in the window
  float* e;      // [W][KP]  running predictions f(r_j)
  float* c;      // [2W][CS] mu q_j beta_jk of the current step (rows doubled)
  float* bwin;   // [W][KP]  training symbols b_j of the window members
  float* ikjj;   // [W]      1 / kappa(r_j, r_j) (0 where kappa(r_j, r_j) <= 0)
  float* rwin;   // [2R][M2P] window members' vectors and r_{n+1} (rows doubled)
  float* part;   // [KP][kWaves] per-wave partial sums of f_n(r_n)
  float* aev;    // [KP]     coefficients of the evicted entry
  float* omega;  // [W]      position weights
  float* qs;     // [W+1]    mu / (omega_0 + .. + omega_{L-1}) for |J_n| = L
  float* vb;     // [W][KP]  beta of the current step (violation weights)
  float* vd;     // [W][KP]  slab distances of the current step (violation weights)
  int* stw;      // [W][KP]  set kinds of the window members (typed training)
  float* alds;   // [KP][cap] Gaussian coefficients, k-major (model-buffer path with SLOTS == 0)
};

__host__ __device__ inline size_t lds_floats(int W, int KP, int M2P) {
  const size_t R = W + 1;
  return 2 * R * R + (size_t)W * (W > 1 ? W - 1 : 1) + 2 * (size_t)W * KP + 2 * (size_t)W * CS + W +
         2 * R * M2P + kWaves * KP + KP + W + (W + 1) + 3 * (size_t)W * KP;
}

// LDS budget of one training workgroup (one per CU; static LDS aside).
constexpr size_t kLdsFloatsMax = 36864;     // 144 KiB

__device__ inline Lds carve(float* base, int W, int KP, int M2P) {
  Lds s;
  const int R = W + 1;
  float* p = base;
  s.gram = p; p += 2 * R * R;
  s.evkr = p; p += W * (W > 1 ? W - 1 : 1);
  s.e = p; p += W * KP;
  s.c = p; p += 2 * W * CS;
  s.bwin = p; p += W * KP;
  s.ikjj = p; p += W;
  s.rwin = p; p += 2 * R * M2P;
  s.part = p; p += kWaves * KP;
  s.aev = p; p += KP;
  s.omega = p; p += W;
  s.qs = p; p += W + 1;
  s.vb = p; p += W * KP;
  s.vd = p; p += W * KP;
  s.stw = reinterpret_cast<int*>(p); p += W * KP;
  s.alds = p;
  return s;
}

// Component m of r_n (zero in the padding m >= M2):
// r_{2t} = r1(t) = x_t, r_{2t+1} = r2(t) = [x_{t,M..2M-1}; -x_{t,0..M-1}].
template <class Ptr>
__device__ __forceinline__ float sample_comp(Ptr rx, int M2, int M, int n, int m) {
  if (m >= M2) return 0.0f;
  const auto src = rx + (size_t)(n >> 1) * M2;
  if ((n & 1) == 0) return src[m];
  return m < M ? src[m + M] : -src[m - M];
}

// a - b mod `mod` for 0 <= a < mod, 0 <= b < mod (ring index without division)
__device__ __forceinline__ int ring_sub(int a, int b, int mod) {
  const int r = a - b;
  return r < 0 ? r + mod : r;
}

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) int32_t gint;
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* to_global(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// NST steps of a member product from member q0 on: every operand load
// first, then the products, in straight-line code so that the loads issue
// back to back.  FULL: every member of the block is below L, so the loads
// are offsets from one per-lane address; otherwise members past L enter as
// zeros, read at member 0's address.
template <int SA, int SB, int NST, bool FULL>
__device__ __forceinline__ floatx4 member_block(floatx4 acc, int q0, int L, int grp, const float* a0,
                                                const float* b0) {
  float av[NST], bv[NST];
  if constexpr (FULL) {
    const int qlo = q0 + grp + 4 * (NST - 1);
    const float* pa = a0 - qlo * SA;
    const float* pb = b0 - qlo * SB;
#pragma unroll
    for (int st = 0; st < NST; ++st) {
      av[st] = pa[4 * (NST - 1 - st) * SA];
      bv[st] = pb[4 * (NST - 1 - st) * SB];
    }
  } else {
#pragma unroll
    for (int st = 0; st < NST; ++st) {
      const int q = q0 + 4 * st + grp;
      const bool ok = q < L;
      const int qc = ok ? q : 0;
      const float x = a0[-qc * SA], y = b0[-qc * SB];
      av[st] = ok ? x : 0.0f;
      bv[st] = ok ? y : 0.0f;
    }
  }
#pragma unroll
  for (int st = 0; st < NST; ++st) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[st], bv[st], acc, 0, 0, 0);
  return acc;
}

// acc += sum over window members q < L of a0[-q SA] b0[-q SB] on one 16 x 16
// tile of v_mfma_f32_16x16x4_f32 (a0, b0: this lane's A and B operands for
// the newest member; lane group grp supplies member 4 step + grp of each
// step).  Blocks of 8 steps (32 members), or 4 for a remainder of 16 or
// fewer.
template <int SA, int SB>
__device__ __forceinline__ floatx4 member_product(floatx4 acc, int L, int grp, const float* a0,
                                                  const float* b0) {
  for (int q0 = 0; q0 < L; q0 += 32) {
    const int rem = L - q0;
    if (rem >= 32)
      acc = member_block<SA, SB, 8, true>(acc, q0, L, grp, a0, b0);
    else if (rem > 16)
      acc = member_block<SA, SB, 8, false>(acc, q0, L, grp, a0, b0);
    else if (rem == 16)
      acc = member_block<SA, SB, 4, true>(acc, q0, L, grp, a0, b0);
    else
      acc = member_block<SA, SB, 4, false>(acc, q0, L, grp, a0, b0);
  }
  return acc;
}

// Training of one detector by one workgroup of kThreads threads.  lds_raw
// holds lds_floats(W, KP, M2P) floats.  ROWS (with SLOTS > 0): the kernel
// values of each step come from the precomputed rows j.glag and j.kw instead
// of being evaluated against a dictionary held here; the dictionary is
// written from the pilots at the end.
template <int M2P, int KP, int SLOTS, bool ROWS = false>
__device__ __forceinline__ void train_body(const TrainJob& j, const TrainCommon& cm, float* lds_raw,
                                           int* block_flags_p) {
  static_assert(!ROWS || SLOTS > 0, "rows training keeps the coefficients in registers");
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int W = cm.W, R = W + 1, cap = j.cap, K = j.K, M2 = j.M2, M = j.M2 / 2;
  // This job trains users k0 .. k0 + K - 1 of a detector with Kt users (the
  // users are independent given the shared kernel values); the group with
  // k0 = 0 also writes the dictionary and the state words.
  const int Kt = j.Kt, k0 = j.k0;
  const bool lead = k0 == 0;
  const int T = 2 * j.P;
  const int EVS = W > 1 ? W - 1 : 1;
  Lds s = carve(lds_raw, W, KP, M2P);
  // The job's arrays are global memory.  Saying so makes their accesses
  // global (not flat) instructions, which the LDS wait counter does not
  // track: the loads issued ahead of their use are then not drained by the
  // LDS waits of every phase.
  const gfloat* rx = to_global(j.rx);
  const gfloat* sym = to_global(j.sym);
  gfloat* const dict = to_global(j.dict);
  gfloat* const alpha = to_global(j.alpha);
  gfloat* const wout = to_global(j.w);
  gint* const state = to_global(j.state);
  const gfloat* const glag = to_global(j.glag);
  const gfloat* const kwg = to_global(j.kw);
  // Set kinds of the samples (generic engine) or hyperslabs throughout; the
  // rows training (the batch path) takes hyperslabs only and compiles
  // without them.  The kinds are read like the targets, unconditionally:
  // without kinds the read goes to the symbol array (in bounds at the same
  // byte index, the value unused), so no load of the step loop sits behind
  // a branch.
  constexpr bool kKinds = !ROWS;
  const bool typed = kKinds && j.st != nullptr;
  const auto stg = to_global(typed ? j.st : reinterpret_cast<const uint8_t*>(j.sym));
  int& block_flags = *block_flags_p;

  for (int i = tid; i < W * KP; i += kThreads) {
    s.e[i] = 0.0f;
    s.bwin[i] = 0.0f;
  }
  for (int i = tid; i < 2 * W * CS; i += kThreads) s.c[i] = 0.0f;
  // Position weights and the scale table qs[L] = mu / (omega_0 + .. +
  // omega_{L-1}), thread p for L = p + 1.  The weights are read at constant
  // indices (straight from the kernel arguments, no private copy); adding
  // the zeros past p leaves the left-to-right prefix sum unchanged.
  if (tid < W) {
    float acc = 0.0f, om = 0.0f;
#pragma unroll
    for (int i = 0; i < APSM_MAX_WINDOW; ++i) {
      const float o = cm.omega[i];
      acc += i <= tid ? o : 0.0f;
      om = i == tid ? o : om;
    }
    s.omega[tid] = om;
    s.qs[tid + 1] = cm.mu / acc;
  }
  if (tid == 0) s.qs[0] = 0.0f;

  // Linear coefficients w = wL v, v[k][m] held as matrix-core accumulators:
  // wave t < M2P/16 holds the 16 x 16 tile of components 16 t .. 16 t + 15
  // (users 0..15), its lane l and register i holding v[4 (l / 16) + i][16 t +
  // l % 16].  The wave both updates the tile (phase D) and uses it for
  // f_n(r_n) (phase A).
  // The Gram-times-coefficient tiles of phase D go to the waves after them.
  constexpr int NWT = M2P / 16;
  const bool wowner = wave < NWT;
  const int col = lane & 15;                // tile column of this lane
  const int grp = lane >> 4;                // tile rows 4 grp .. 4 grp + 3 of this lane
  const int wm = 16 * wave + col;           // component of this lane's weight-tile column
  const int etile = (wave - NWT) & (kWaves - 1);
  floatx4 wacc = {0.0f, 0.0f, 0.0f, 0.0f};
  // Initial filter: f_0 = 0, or the model's linear part (w = wL v) for a
  // linear start or a continued training.
  if (cm.init != kInitZero && wowner) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = 4 * grp + v;
      wacc[v] = (k < K && wm < M2) ? wout[(k0 + k) * M2 + wm] / cm.wl : 0.0f;
    }
  }
  // A continued training resumes the dictionary ring after the n0 samples
  // the model has seen; its window starts afresh.
  const int n0 = cm.init == kInitContinue ? __builtin_amdgcn_readfirstlane(state[2]) : 0;
  const int size0 = n0 < cap ? n0 : cap;      // entries in use at the start

  // Register-resident slots (SLOTS > 0): slot tid + kThreads * u.
  constexpr int DS = SLOTS > 0 && !ROWS ? SLOTS : 1;     // slots whose vectors are held here
  float dreg[DS][ROWS ? 1 : M2P];
  float dnorm[DS];
  float areg[SLOTS > 0 ? SLOTS : 1][KP];
  if constexpr (SLOTS > 0) {
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) {
#pragma unroll
      for (int k = 0; k < KP; ++k) areg[u][k] = 0.0f;
    }
    if constexpr (!ROWS) {
#pragma unroll
      for (int u = 0; u < SLOTS; ++u) {
        const int slot = tid + kThreads * u;
        const bool used = slot < size0;
        float n4[4] = {0.0f, 0.0f, 0.0f, 0.0f};    // grouped as ||r_n||^2 in phase A
#pragma unroll
        for (int m = 0; m < M2P; ++m) {
          dreg[u][m] = (used && m < M2) ? dict[(size_t)m * cap + slot] : 0.0f;
          n4[m & 3] = fmaf(dreg[u][m], dreg[u][m], n4[m & 3]);
        }
        dnorm[u] = (n4[0] + n4[1]) + (n4[2] + n4[3]);
#pragma unroll
        for (int k = 0; k < KP; ++k) areg[u][k] = (used && k < K) ? alpha[(size_t)slot * Kt + k0 + k] : 0.0f;
      }
    }
  } else if constexpr (SLOTS == 0) {
    // Dictionary in the model buffer, coefficients in LDS (those of a
    // continued model loaded, else an empty dictionary).
    for (int i = tid; i < cap * KP; i += kThreads) {
      const int k = i / cap, slot = i - k * cap;
      s.alds[i] = (slot < size0 && k < K) ? alpha[(size_t)slot * Kt + k0 + k] : 0.0f;
    }
  } else {
    // Dictionary and coefficients in the model buffers (a continued model's
    // are used in place; otherwise start from an empty dictionary).
    if (cm.init != kInitContinue)
      for (size_t i = tid; i < (size_t)cap * K; i += kThreads) alpha[(i / K) * Kt + k0 + i % K] = 0.0f;
  }
  if (tid == 0) block_flags = 0;
  int flags = 0;

  // Global inputs are read one step ahead, so their latency overlaps the
  // previous step: component tid of r_{n+1} (stored into the vector ring in
  // phase C) and b_{k,n+1} for thread k.  Every load of the step loop is
  // unconditional (clamped indices; the sign of an r2 component and the
  // user mask are applied where the value is stored), so that the waits the
  // compiler places for each value cover only that value's load.
  float comp_nx = 0.0f, comp_sg = 0.0f, bv = 0.0f, bv_nx = 0.0f;
  int stv = kSetSlab, stv_nx = kSetSlab;
  if (tid < M2P) {
    const float c0 = sample_comp(rx, M2, M, 0, tid);
    s.rwin[tid] = c0;
    s.rwin[R * M2P + tid] = c0;
  }
  bv = sym[(k0 + (tid < K ? tid : 0)) * 2];
  if constexpr (kKinds) stv = stg[(k0 + (tid < K ? tid : 0)) * 2];

  // Rows training: the kernel values of the even steps are loaded into
  // kr0 / kw0, those of the odd steps into kr1 / kw1, each two steps ahead
  // of its use.  Thread t reads, per slot, the lag that slot has at that
  // step, and for t < W the window Gram entry of lag t.
  float kr0[ROWS ? SLOTS : 1], kr1[ROWS ? SLOTS : 1];
  float kw0 = 0.0f, kw1 = 0.0f;
  auto rows_load = [&](int m, int sm, float* kr, float& kwv) {
    const gfloat* grow = glag + (size_t)m * cap;
#pragma unroll
    for (int u = 0; u < (ROWS ? SLOTS : 1); ++u) {
      const int slot = tid + kThreads * u;
      kr[u] = grow[ring_sub(sm, slot < cap ? slot : 0, cap)];
    }
    kwv = kwg[(size_t)m * W + (tid < W ? tid : 0)];
  };
  int sn2 = 0;                              // (n + 2) % cap
  if constexpr (ROWS) {
    rows_load(0, 0, kr0, kw0);
    rows_load(T > 1 ? 1 : 0, 1 % cap, kr1, kw1);
    sn2 = 2 % cap;
  }
  __syncthreads();

  int sn = n0 % cap, nw = 0, nr = 0;        // (n0 + n) % cap, n % W, n % R
  // One training step; kr / kwv: the prefetched kernel values of this step
  // (rows training), refilled with those of step n + 2 once used.
  auto step = [&](const int n, float* kr, float& kwv) {
    {
      const int n1 = n + 1 < T ? n + 1 : n;   // the last step reloads its own sample (unused)
      const int m = tid < M2 ? tid : 0;
      const bool odd = (n1 & 1) != 0;
      comp_nx = rx[(size_t)(n1 >> 1) * M2 + (odd ? (m < M ? m + M : m - M) : m)];
      comp_sg = tid < M2 ? (odd && m >= M ? -1.0f : 1.0f) : 0.0f;
      bv_nx = sym[((size_t)(n1 >> 1) * Kt + k0 + (tid < K ? tid : 0)) * 2 + (n1 & 1)];
      if constexpr (kKinds) stv_nx = stg[((size_t)(n1 >> 1) * Kt + k0 + (tid < K ? tid : 0)) * 2 + (n1 & 1)];
    }

    // ------------------------------------------------------------ phase A
    const float* rrow = s.rwin + nr * M2P;  // r_n
    float rn[SLOTS > 0 && !ROWS ? M2P : 1];
    float nn = 0.0f;
    if constexpr (ROWS) {
    } else if constexpr (SLOTS > 0) {
      // ||r_n||^2 summed in the same four groups (m mod 4) and order as the
      // products r_n . d below, so that for the entry r_n itself
      // 2 r_n.d - ||r_n||^2 - ||d||^2 is exactly 0: kappa_G(r_n, r_n) = 1 and the
      // Gram diagonal equals the wL ||r_n||^2 + wG of the projection.
      float n4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int m = 0; m < M2P; ++m) {
        rn[m] = rrow[m];
        n4[m & 3] = fmaf(rn[m], rn[m], n4[m & 3]);
      }
      nn = (n4[0] + n4[1]) + (n4[2] + n4[3]);
    } else {
      float n4[4] = {0.0f, 0.0f, 0.0f, 0.0f};        // grouped as above
      for (int m = 0; m < M2; ++m) n4[m & 3] = fmaf(rrow[m], rrow[m], n4[m & 3]);
      nn = (n4[0] + n4[1]) + (n4[2] + n4[3]);
    }
    const int ng = n0 + n;                  // global index of r_n (dictionary ring)
    const bool evicting = ng >= cap;
    const int L = n + 1 < W ? n + 1 : W;    // |J_n| (the window is local)
    const int evlo = ng - cap + 1;          // oldest entry in the dictionary after the append
    if (tid < KP) {
      s.bwin[nw * KP + tid] = tid < K ? bv : 0.0f;
      if constexpr (kKinds) s.stw[nw * KP + tid] = stv;
    }
    if constexpr (ROWS) {
      // Gram entries of r_n against the window members, one lag per thread
      if (tid < L) {
        const int ir = ring_sub(nr, tid, R);
        s.gram[nr * 2 * R + ir] = kwv;
        s.gram[nr * 2 * R + ir + R] = kwv;
        s.gram[ir * 2 * R + nr] = kwv;
        s.gram[ir * 2 * R + nr + R] = kwv;
      }
      if (tid == 0) s.ikjj[nw] = kwv > 0.0f ? 1.0f / kwv : 0.0f;   // lag 0: K(r_n, r_n)
    } else if (tid == 0) {
      const float kjj = fmaf(cm.wl, nn, cm.wg);
      s.ikjj[nw] = kjj > 0.0f ? 1.0f / kjj : 0.0f;
    }

    float part[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) part[k] = 0.0f;

    if constexpr (ROWS) {
#pragma unroll
      for (int u = 0; u < SLOTS; ++u) {
        const int slot = tid + kThreads * u;
        if (slot == sn) {                    // append (and evict)
          if (evicting) {
#pragma unroll
            for (int k = 0; k < KP; ++k) s.aev[k] = areg[u][k];
          }
#pragma unroll
          for (int k = 0; k < KP; ++k) areg[u][k] = 0.0f;
        }
        if (slot < cap && slot <= ng) {
          const int back = ring_sub(sn, slot, cap);   // this slot holds sample ng - back
          const float kg = kr[u];
#pragma unroll
          for (int k = 0; k < KP; ++k) part[k] = fmaf(areg[u][k], kg, part[k]);
          const int mv = ng - back - evlo;
          if (mv >= 0 && mv <= W - 2) s.evkr[nw * EVS + mv] = kg;
        }
      }
      // this buffer's next use is step n + 2
      rows_load(n + 2 < T ? n + 2 : n, sn2, kr, kwv);   // past the end: a valid row, unused
      sn2 = sn2 + 1 == cap ? 0 : sn2 + 1;
    } else if constexpr (SLOTS > 0) {
#pragma unroll
      for (int u = 0; u < SLOTS; ++u) {
        const int slot = tid + kThreads * u;
        if (slot == sn) {                    // append (and evict)
          if (evicting) {
#pragma unroll
            for (int k = 0; k < KP; ++k) s.aev[k] = areg[u][k];
          }
#pragma unroll
          for (int m = 0; m < M2P; ++m) dreg[u][m] = rn[m];
          dnorm[u] = nn;
#pragma unroll
          for (int k = 0; k < KP; ++k) areg[u][k] = 0.0f;
        }
        if (slot < cap && slot <= ng) {
          const int back = ring_sub(sn, slot, cap);   // this slot holds sample ng - back
          float d4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int m = 0; m < M2P; ++m) d4[m & 3] = fmaf(rn[m], dreg[u][m], d4[m & 3]);
          const float dot = (d4[0] + d4[1]) + (d4[2] + d4[3]);
          const float kg = __builtin_amdgcn_exp2f(j.c2 * (2.0f * dot - nn - dnorm[u]));
#pragma unroll
          for (int k = 0; k < KP; ++k) part[k] = fmaf(areg[u][k], kg, part[k]);
          if (back < L) {
            const int ir = ring_sub(nr, back, R);
            const float g = fmaf(cm.wl, dot, cm.wg * kg);
            s.gram[nr * 2 * R + ir] = g;
            s.gram[nr * 2 * R + ir + R] = g;
            s.gram[ir * 2 * R + nr] = g;
            s.gram[ir * 2 * R + nr + R] = g;
          }
          const int mv = ng - back - evlo;
          if (mv >= 0 && mv <= W - 2) s.evkr[nw * EVS + mv] = kg;
        }
      }
    } else {
      // Model-buffer path: SB of this thread's slots at a time, MB components
      // of each loaded before any is used, so that up to 64 loads are in
      // flight at once (the dictionary is component-major: lanes read
      // consecutive slots, coalesced).
      constexpr int SB0 = M2P >= 64 ? 1 : 64 / M2P;
      constexpr int SB = KP == 16 && SB0 > 2 ? 2 : SB0;   // 16 users: bounded by their coefficient registers
      constexpr int MB = M2P >= 64 ? 64 : M2P;
      const int nslot = (ng + 1 < cap ? ng + 1 : cap);      // slots in use after the append
      if (tid == (sn & (kThreads - 1))) {                   // append (and evict)
        if constexpr (SLOTS == 0) {
          if (evicting)
            for (int k = 0; k < KP; ++k) s.aev[k] = s.alds[k * cap + sn];
          for (int k = 0; k < KP; ++k) s.alds[k * cap + sn] = 0.0f;
        } else {
          auto arow = alpha + (size_t)sn * Kt + k0;
          if (evicting)
            for (int k = 0; k < K; ++k) s.aev[k] = arow[k];
          for (int k = 0; k < K; ++k) arow[k] = 0.0f;
        }
        for (int m = 0; m < M2; ++m) dict[(size_t)m * cap + sn] = rrow[m];
      }
      for (int base = tid; base < nslot; base += SB * kThreads) {
        float dot4[SB][4], dn4[SB][4], av[SB][KP];
#pragma unroll
        for (int b = 0; b < SB; ++b) {
          const int slot = base + b * kThreads;
          const bool ok = slot < nslot;
#pragma unroll
          for (int q = 0; q < 4; ++q) { dot4[b][q] = 0.0f; dn4[b][q] = 0.0f; }
          if constexpr (SLOTS == 0) {
#pragma unroll
            for (int k = 0; k < KP; ++k) av[b][k] = ok ? s.alds[k * cap + slot] : 0.0f;
          } else {
            const auto arow = alpha + (size_t)(ok ? slot : 0) * Kt + k0;
#pragma unroll
            for (int k = 0; k < KP; ++k) av[b][k] = (ok && k < K) ? arow[k] : 0.0f;
          }
        }
#pragma unroll 1
        for (int m0 = 0; m0 < M2P; m0 += MB) {
          // Unconditional loads (clamped addresses) so that they issue back to
          // back; padded components (m >= M2) are masked out after the load,
          // and slots past the ones in use are discarded below.
          float dv[SB][MB];
#pragma unroll
          for (int b = 0; b < SB; ++b) {
            const int slot = base + b * kThreads;
            const auto dcol = dict + (slot < nslot ? slot : 0);
#pragma unroll
            for (int m = 0; m < MB; ++m) {
              const int mm = m0 + m < M2 ? m0 + m : M2 - 1;
              dv[b][m] = dcol[(size_t)mm * cap];
            }
          }
#pragma unroll
          for (int b = 0; b < SB; ++b)
#pragma unroll
            for (int m = 0; m < MB; ++m) {
              const float d = m0 + m < M2 ? dv[b][m] : 0.0f;
              dot4[b][m & 3] = fmaf(rrow[m0 + m], d, dot4[b][m & 3]);
              dn4[b][m & 3] = fmaf(d, d, dn4[b][m & 3]);
            }
        }
#pragma unroll
        for (int b = 0; b < SB; ++b) {
          const int slot = base + b * kThreads;
          if (slot >= nslot) continue;
          const float dot = (dot4[b][0] + dot4[b][1]) + (dot4[b][2] + dot4[b][3]);
          const float dn = (dn4[b][0] + dn4[b][1]) + (dn4[b][2] + dn4[b][3]);
          const float kg = __builtin_amdgcn_exp2f(j.c2 * (2.0f * dot - nn - dn));
#pragma unroll
          for (int k = 0; k < KP; ++k) part[k] = fmaf(av[b][k], kg, part[k]);
          const int back = ring_sub(sn, slot, cap);
          if (back < L) {
            const int ir = ring_sub(nr, back, R);
            const float g = fmaf(cm.wl, dot, cm.wg * kg);
            s.gram[nr * 2 * R + ir] = g;
            s.gram[nr * 2 * R + ir + R] = g;
            s.gram[ir * 2 * R + nr] = g;
            s.gram[ir * 2 * R + nr + R] = g;
          }
          const int mv = ng - back - evlo;
          if (mv >= 0 && mv <= W - 2) s.evkr[nw * EVS + mv] = kg;
        }
      }
    }
    // the linear part last: the weight tile is the accumulator of the
    // previous step's matrix-core products, which the slot work above
    // leaves time to complete
    if (wowner) {
      const float rm = cm.wl * rrow[wm];
#pragma unroll
      for (int k = 0; k < KP; ++k) part[k] += (grp == (k >> 2)) ? wacc[k & 3] * rm : 0.0f;
    }
    {
      const float v = wave_sum_scatter<KP>(part, lane);
      if (scatter_writer<KP>(lane)) s.part[scatter_user<KP>(lane) * kWaves + wave] = v;
    }
    __syncthreads();

    // ------------------------------------------------------------ phase C
    // Every operand is loaded before the first use (one LDS round trip).
    // Position weights: c = mu q_j beta at once.  Violation weights (q_kj
    // proportional to member j's distance to its slab, per user): beta and
    // the distance are parked in LDS and c is formed after a barrier, once
    // the distances of all members are there.
    // Position weights: c = mu q_j beta at once.  Violation or active-set
    // weights, or the extrapolated relaxation: beta and the distance to the
    // set are parked in LDS and c is formed after a barrier (see below).
    const bool vweights = cm.weights != kWeightsPosition;
    const bool extra = cm.extrapolate != 0;
    const bool two_pass = vweights || extra;
    const float qscale = s.qs[L];
    // c of member p (ring row jw, dictionary slot `slot`) and user k: the
    // coefficient ring and, on the model-buffer paths, the Gaussian
    // coefficient (one (member, user) pair per thread; the barrier after
    // phase C orders it before every later read)
    auto commit = [&](int p, int k, int jw, int slot, float c, float aold) {
      if (k < K) {
        if constexpr (SLOTS == 0) s.alds[k * cap + slot] = fmaf(c, cm.wg, aold);
        if constexpr (SLOTS < 0) alpha[(size_t)slot * Kt + k0 + k] = fmaf(c, cm.wg, aold);
      }
      s.c[jw * CS + k] = c;
      s.c[(jw + W) * CS + k] = c;
    };
    for (int t = tid; t < L * KP; t += kThreads) {
      const int p = t / KP, k = t - p * KP;
      const int jw = ring_sub(nw, p, W);
      const int slot = ring_sub(sn, p, cap);    // dictionary slot of member n - p
      float pw[kWaves];
#pragma unroll
      for (int w = 0; w < kWaves; ++w) pw[w] = s.part[k * kWaves + w];
      const float eold = s.e[jw * KP + k];
      const float ev = s.evkr[jw * EVS + (p > 0 ? p - 1 : 0)];
      const float aev = s.aev[k];
      const float bw = s.bwin[jw * KP + k];
      const float ik = s.ikjj[jw];
      const float om = s.omega[p];
      float aold = 0.0f;
      if constexpr (SLOTS == 0) aold = s.alds[k * cap + slot];
      if constexpr (SLOTS < 0) aold = alpha[(size_t)slot * Kt + k0 + (k < K ? k : 0)];

      // new member: the reduced partial sums; older members: the running
      // value less the evicted entry's Gaussian term (selects, no branch)
      float esum = 0.0f;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) esum += pw[w];
      const float eupd = evicting ? eold - aev * ev : eold;
      const float e = p == 0 ? esum : eupd;
      const float x = e - bw;
      // e minus the nearest value the member's set admits: eqn:beta's soft
      // threshold for a hyperslab; one-sided for a halfspace; all of x for
      // a hyperplane
      float res;
      if (typed) {
        const int kind = s.stw[jw * KP + k];
        res = kind == kSetPlane   ? x
              : kind == kSetUpper ? fmaxf(x - cm.eps, 0.0f)
              : kind == kSetLower ? fminf(x + cm.eps, 0.0f)
                                  : soft_threshold(x, cm.eps);
      } else {
        res = soft_threshold(x, cm.eps);
      }
      const float beta = -res * ik;
      if (k < K) {
        s.e[jw * KP + k] = e;
        if (!isfinite(x)) flags |= 1;
      }
      if (two_pass) {
        s.vb[p * KP + k] = beta;
        // active-set weights: violated by more than 1e-5 (a member that its
        // own projection left on the boundary stays out, whatever the rounding)
        const float dist = cm.weights == kWeightsActive ? (fabsf(res) > 1e-5f ? 1.0f : 0.0f) : fabsf(res);
        s.vd[p * KP + k] = k < K ? dist : 0.0f;
      } else {
        commit(p, k, jw, slot, k < K ? qscale * om * beta : 0.0f, aold);
      }
    }
    if (extra) {
      // Extrapolated relaxation, per user k: c_j = mu M q_j beta_j with
      // M = sum_j q_j beta_j^2 K_jj / sum_{j,l} u_j K_jl u_l, u = q beta
      // (1 where the denominator is not positive).  u is parked in this
      // step's rows of the coefficient ring (the commit overwrites them);
      // the per-member terms replace beta and the distance in LDS and one
      // thread per user sums them in member order.
      __syncthreads();
      for (int t = tid; t < L * KP; t += kThreads) {
        const int p = t / KP, k = t - p * KP;
        float q = 0.0f;
        if (k < K) {
          if (vweights) {
            float tot = 0.0f;
            for (int i = 0; i < L; ++i) tot += s.vd[i * KP + k];
            q = tot > 0.0f ? s.vd[p * KP + k] / tot : 0.0f;
          } else {
            q = qscale * s.omega[p] / cm.mu;
          }
        }
        s.c[ring_sub(nw, p, W) * CS + k] = q * s.vb[p * KP + k];
      }
      __syncthreads();
      for (int t = tid; t < L * KP; t += kThreads) {
        const int p = t / KP, k = t - p * KP;
        const float* grow = s.gram + ring_sub(nr, p, R) * 2 * R + nr + R;   // K(r_{n-p}, r_{n-l}) at grow[-l]
        float kt = 0.0f;
        for (int l = 0; l < L; ++l) kt = fmaf(grow[-l], s.c[ring_sub(nw, l, W) * CS + k], kt);
        const float u = s.c[ring_sub(nw, p, W) * CS + k];
        s.vd[p * KP + k] = u * s.vb[p * KP + k] * grow[-p];
        s.vb[p * KP + k] = u * kt;
      }
      __syncthreads();
      if (tid < KP) {
        float num = 0.0f, den = 0.0f;
        for (int p = 0; p < L; ++p) {
          num += s.vd[p * KP + tid];
          den += s.vb[p * KP + tid];
        }
        s.part[tid] = den > 0.0f ? num / den : 1.0f;
      }
      __syncthreads();
      for (int t = tid; t < L * KP; t += kThreads) {
        const int p = t / KP, k = t - p * KP;
        const int jw = ring_sub(nw, p, W);
        const int slot = ring_sub(sn, p, cap);
        float aold = 0.0f;
        if constexpr (SLOTS == 0) aold = s.alds[k * cap + slot];
        if constexpr (SLOTS < 0) aold = alpha[(size_t)slot * Kt + k0 + (k < K ? k : 0)];
        const float c = k < K ? cm.mu * s.part[k] * s.c[jw * CS + k] : 0.0f;
        commit(p, k, jw, slot, c, aold);
      }
    } else if (vweights) {
      __syncthreads();
      for (int t = tid; t < L * KP; t += kThreads) {
        const int p = t / KP, k = t - p * KP;
        const int jw = ring_sub(nw, p, W);
        const int slot = ring_sub(sn, p, cap);
        float tot = 0.0f;
        for (int i = 0; i < L; ++i) tot += s.vd[i * KP + k];
        float aold = 0.0f;
        if constexpr (SLOTS == 0) aold = s.alds[k * cap + slot];
        if constexpr (SLOTS < 0) aold = alpha[(size_t)slot * Kt + k0 + (k < K ? k : 0)];
        const float c = (k < K && tot > 0.0f) ? cm.mu * (s.vd[p * KP + k] / tot) * s.vb[p * KP + k] : 0.0f;
        commit(p, k, jw, slot, c, aold);
      }
    }
    if (tid < M2P && n + 1 < T) {           // r_{n+1} into its ring row (no member of J_n)
      const int nr1 = nr + 1 == R ? 0 : nr + 1;
      s.rwin[nr1 * M2P + tid] = comp_sg * comp_nx;
      s.rwin[(nr1 + R) * M2P + tid] = comp_sg * comp_nx;
    }
    __syncthreads();

    // ------------------------------------------------------------ phase D
    const float* cbase = s.c + (nw + W) * CS;       // member n - q at cbase - q * CS
    if (wowner) {
      // v[k][m] += sum_q c_{q,k} r_q[m] with w = wL v: A = coefficients
      // (rows k), B = member vectors
      wacc = member_product<CS, M2P>(wacc, L, grp, cbase + col, s.rwin + (nr + R) * M2P + wm);
    }
    if (etile < ((L + 15) >> 4)) {
      // e[i][k] += sum_q K(r_i, r_q) c_{q,k}: A = Gram rows of members
      // 16 etile .. 16 etile + 15 (columns doubled along the member index
      // q), B = coefficients
      const int ia = 16 * etile + col;
      const float* grow = s.gram + ring_sub(nr, ia < L ? ia : 0, R) * 2 * R + nr + R;
      floatx4 acc;
      int eidx[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * etile + 4 * grp + v;
        eidx[v] = (i < L && col < KP) ? ring_sub(nw, i, W) * KP + col : -1;
        acc[v] = s.e[eidx[v] >= 0 ? eidx[v] : 0];
      }
      acc = member_product<1, CS>(acc, L, grp, grow, cbase + col);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (eidx[v] >= 0) s.e[eidx[v]] = acc[v];
    }
    if constexpr (SLOTS > 0) {
#pragma unroll
      for (int u = 0; u < SLOTS; ++u) {
        const int slot = tid + kThreads * u;
        if (slot < cap && slot <= ng) {
          const int back = ring_sub(sn, slot, cap);
          if (back < L) {
            const float* cj = cbase - back * CS;
#pragma unroll
            for (int k = 0; k < KP; ++k) areg[u][k] = fmaf(cj[k], cm.wg, areg[u][k]);
          }
        }
      }
    }
    // Phase A of the next step touches only ring rows that no window member
    // of this step uses (the Gram and vector rings have W + 1 rows; the
    // W-rows rings are read only in phase C), so no barrier is needed here.

    bv = bv_nx;
    stv = stv_nx;
    sn = sn + 1 == cap ? 0 : sn + 1;
    nw = nw + 1 == W ? 0 : nw + 1;
    nr = nr + 1 == R ? 0 : nr + 1;
  };
  if constexpr (ROWS) {
    // two steps per iteration, each with its own buffer, so that a buffer is
    // refilled right after its use and next read two steps later
    for (int n = 0; n < T; n += 2) {
      step(n, kr0, kw0);
      if (n + 1 < T) step(n + 1, kr1, kw1);
    }
  } else {
    for (int n = 0; n < T; ++n) step(n, kr0, kw0);
  }
  __syncthreads();

  // ------------------------------------------------------------ write back
  if constexpr (SLOTS > 0) {
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) {
      const int slot = tid + kThreads * u;
      if (slot < cap) {
        if constexpr (ROWS) {
          // the slot holds sample T-1 - lag (lag of the slot after the last step), if written
          const int lag = ring_sub((T - 1) % cap, slot, cap);
          const int i = T - 1 - lag;
          if (lead)
            for (int mm = 0; mm < M2; ++mm)
              dict[(size_t)mm * cap + slot] = i >= 0 ? sample_comp(rx, M2, M, i, mm) : 0.0f;
        } else {
#pragma unroll
          for (int mm = 0; mm < M2P; ++mm)
            if (mm < M2) dict[(size_t)mm * cap + slot] = dreg[u][mm];
        }
        auto arow = alpha + (size_t)slot * Kt + k0;
#pragma unroll
        for (int k = 0; k < KP; ++k)
          if (k < K) arow[k] = areg[u][k];
      }
    }
  } else {
    // Slots never written (n0 + T < cap) are cleared so detection may sum them.
    for (int slot = n0 + T + tid; slot < cap; slot += kThreads)
      for (int m = 0; m < M2; ++m) dict[(size_t)m * cap + slot] = 0.0f;
    if constexpr (SLOTS == 0)
      for (int i = tid; i < cap * K; i += kThreads) {
        const int slot = i / K, k = i - slot * K;
        alpha[(size_t)slot * Kt + k0 + k] = s.alds[k * cap + slot];
      }
  }
  if (wowner) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = 4 * grp + v;
      if (k < K && wm < M2) wout[(k0 + k) * M2 + wm] = cm.wl * wacc[v];
    }
  }
  if (flags) atomicOr(&block_flags, flags);
  __syncthreads();
  if (tid == 0) {
    if (lead) {
      const int Tg = n0 + T;                // samples seen in all
      state[0] = Tg < cap ? Tg : cap;
      state[1] = Tg % cap;
      state[2] = Tg;
    }
    // A detector trained as one job overwrites its flags word; the groups of
    // a split detector OR theirs into it (cleared by the kernel-rows launch).
    if (K == Kt) state[3] = block_flags;
    else atomicOr(j.state + 3, block_flags);
  }
}

// Detectors of one shape, described in the kernel arguments.
template <int M2P, int KP, int SLOTS>
__global__ __launch_bounds__(kThreads) void train_kernel(TrainArgs a) {
  extern __shared__ float lds_raw[];
  __shared__ int block_flags;
  const int b = blockIdx.x;
  TrainJob j;
  j.rx = a.rx + (size_t)b * a.P * a.M2;
  j.sym = a.sym + (size_t)b * a.P * a.K * 2;
  j.st = a.st ? a.st + (size_t)b * a.P * a.K * 2 : nullptr;
  j.dict = a.dict[b];
  j.alpha = a.alpha[b];
  j.w = a.w[b];
  j.state = a.state[b];
  j.P = a.P;
  j.M2 = a.M2;
  j.K = a.K;
  j.Kt = a.K;
  j.k0 = 0;
  j.cap = a.cap;
  j.c2 = a.c2;
  j.variant = 0;
  train_body<M2P, KP, SLOTS>(j, a.cm, lds_raw, &block_flags);
}

// Specialisation for a shape: SLOTS > 0 keeps SLOTS dictionary slots per
// thread in registers (SLOTS * (M2P + KP) <= 128 floats); SLOTS = 0 keeps
// the dictionary in the model buffer and the coefficients in LDS; SLOTS = -1
// keeps both in the model buffers (capacities whose coefficients do not fit
// the LDS budget).
__host__ __device__ constexpr int kp_for(int K) { return K <= 4 ? 4 : K <= 8 ? 8 : 16; }
__host__ __device__ constexpr int m2p_for(int M2) { return M2 <= 16 ? 16 : M2 <= 32 ? 32 : M2 <= 64 ? 64 : 128; }

__host__ __device__ inline int slots_for(int M2P, int KP, int W, int cap) {
  const int need = (cap + kThreads - 1) / kThreads;
  const int s = need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 0;
  // dictionary plus coefficient registers of the slots within 128 per thread
  // (two waves per SIMD at 512 threads leave 256 registers per thread)
  if (s > 0 && s * (M2P + KP) <= 128) return s;
  return lds_floats(W, KP, M2P) + (size_t)cap * KP <= kLdsFloatsMax ? 0 : -1;
}

__host__ __device__ inline size_t lds_bytes_for(int W, int KP, int M2P, int slots, int cap) {
  return (lds_floats(W, KP, M2P) + (slots == 0 ? (size_t)cap * KP : 0)) * sizeof(float);
}

// Every specialisation (M2P, KP, SLOTS) with its variant number.
#define APSM_TRAIN_VARIANTS_M(X, base, M2P, KP)                                    \
  X(base + 0, M2P, KP, -1) X(base + 1, M2P, KP, 0) X(base + 2, M2P, KP, 1)         \
  X(base + 3, M2P, KP, 2) X(base + 4, M2P, KP, 4) X(base + 5, M2P, KP, 8)
#define APSM_TRAIN_VARIANTS(X)                                                      \
  APSM_TRAIN_VARIANTS_M(X, 0, 16, 4) APSM_TRAIN_VARIANTS_M(X, 6, 16, 8)            \
  APSM_TRAIN_VARIANTS_M(X, 12, 16, 16) APSM_TRAIN_VARIANTS_M(X, 18, 32, 4)         \
  APSM_TRAIN_VARIANTS_M(X, 24, 32, 8) APSM_TRAIN_VARIANTS_M(X, 30, 32, 16)         \
  APSM_TRAIN_VARIANTS_M(X, 36, 64, 4) APSM_TRAIN_VARIANTS_M(X, 42, 64, 8)          \
  APSM_TRAIN_VARIANTS_M(X, 48, 64, 16) APSM_TRAIN_VARIANTS_M(X, 54, 128, 4)        \
  APSM_TRAIN_VARIANTS_M(X, 60, 128, 8) APSM_TRAIN_VARIANTS_M(X, 66, 128, 16)

__host__ __device__ constexpr int variant_of(int M2P, int KP, int SLOTS) {
  const int mi = M2P == 16 ? 0 : M2P == 32 ? 1 : M2P == 64 ? 2 : 3;
  const int ki = KP == 4 ? 0 : KP == 8 ? 1 : 2;
  const int si = SLOTS < 0 ? 0 : SLOTS == 0 ? 1 : SLOTS == 1 ? 2 : SLOTS == 2 ? 3 : SLOTS == 4 ? 4 : 5;
  return (mi * 3 + ki) * 6 + si;
}

// The table kernel holds the register-resident specialisations only where
// they fit the register file on their own (no spill space needed); other
// jobs take the model-buffer path.  One function holding the heavier ones as
// well would spill for all of them.
__host__ __device__ constexpr bool in_table(int M2P, int KP, int SLOTS) {
  return SLOTS <= 0 || (SLOTS * (M2P + KP) <= 128 && !(M2P == 64 && KP == 16));
}

// Detectors of shapes with 2M <= 64, one job per workgroup from a device
// table; each job runs the specialisation its variant names.  (The 2M = 128
// specialisations, held in the same function, would make it spill for every
// job: such detectors are trained by their own launches.)
__global__ __launch_bounds__(kThreads) void train_table_kernel(const TrainJob* jobs, TrainCommon cm) {
  extern __shared__ float lds_raw[];
  __shared__ int block_flags;
  const TrainJob j = jobs[blockIdx.x];
  switch (j.variant) {
#define APSM_TRAIN_CASE(id, M2P, KP, SLOTS)                                         \
  case id:                                                                          \
    if constexpr (M2P <= 64 && in_table(M2P, KP, SLOTS)) train_body<M2P, KP, SLOTS>(j, cm, lds_raw, &block_flags); \
    break;
    APSM_TRAIN_VARIANTS(APSM_TRAIN_CASE)
#undef APSM_TRAIN_CASE
    default:
      break;
  }
}

// ---- training from precomputed kernel rows

// Every rows specialisation (M2P, KP, SLOTS in 1, 2, 4, 8) with its number.
#define APSM_ROWS_VARIANTS_M(X, base, M2P, KP) \
  X(base + 0, M2P, KP, 1) X(base + 1, M2P, KP, 2) X(base + 2, M2P, KP, 4) X(base + 3, M2P, KP, 8)
#define APSM_ROWS_VARIANTS(X)                                                     \
  APSM_ROWS_VARIANTS_M(X, 0, 16, 4) APSM_ROWS_VARIANTS_M(X, 4, 16, 8)            \
  APSM_ROWS_VARIANTS_M(X, 8, 16, 16) APSM_ROWS_VARIANTS_M(X, 12, 32, 4)          \
  APSM_ROWS_VARIANTS_M(X, 16, 32, 8) APSM_ROWS_VARIANTS_M(X, 20, 32, 16)         \
  APSM_ROWS_VARIANTS_M(X, 24, 64, 4) APSM_ROWS_VARIANTS_M(X, 28, 64, 8)          \
  APSM_ROWS_VARIANTS_M(X, 32, 64, 16) APSM_ROWS_VARIANTS_M(X, 36, 128, 4)        \
  APSM_ROWS_VARIANTS_M(X, 40, 128, 8) APSM_ROWS_VARIANTS_M(X, 44, 128, 16)       \
  X(48, 16, 4, 16) X(49, 32, 4, 16) X(50, 64, 4, 16) X(51, 128, 4, 16)

__global__ __launch_bounds__(kThreads) void train_rows_kernel(const TrainJob* jobs, TrainCommon cm) {
  extern __shared__ float lds_raw[];
  __shared__ int block_flags;
  const TrainJob j = jobs[blockIdx.x];
  switch (j.variant) {
#define APSM_ROWS_CASE(id, M2P, KP, SLOTS) \
  case id: train_body<M2P, KP, SLOTS, true>(j, cm, lds_raw, &block_flags); break;
    APSM_ROWS_VARIANTS(APSM_ROWS_CASE)
#undef APSM_ROWS_CASE
    default:
      break;
  }
}

// Kernel rows: item (job, n0, l0) writes, for the steps n0 <= n < n0 + 128
// and the lags l0 <= l < l0 + 128,
//   glag[n][l] = kappa_G(r_n, r_{n-l})   (0 for l > n)
// and for l < W the window Gram entry kw[n][l] = wL r_n.r_{n-l} + wG kappa_G(r_n, r_{n-l}).
// The products r_n.r_i of the tile form a 128 x 255 band of a Gram matrix:
// wave w computes the 16 steps n0 + 16 w .. n0 + 16 w + 15 against the nine
// 16-sample column tiles that its lags reach, on v_mfma_f32_16x16x4_f32
// (steps as rows, samples as columns).  Lane (c, g) of a column tile holds
// components g Q .. g Q + Q - 1 (Q = M2R / 4) of its step (A operand, in
// registers) and of its sample (B operand, read from LDS four at a time), so
// MFMA s contracts component g Q + s over the four lane groups.  The 256
// samples the workgroup needs are staged in LDS with their squared norms;
// kappa_G = exp2(-c2 max(0, ||r_n||^2 + ||r_i||^2 - 2 r_n.r_i)), and exactly 1
// at lag 0 (with r_n.r_n taken as ||r_n||^2).
constexpr int kRowsTile = 128;              // steps per workgroup
constexpr int kRowsLags = 128;              // lags per workgroup
constexpr int kRowsThreads = 512;           // eight waves, 16 steps each
constexpr int kRowsSamples = 256;           // kRowsTile + kRowsLags - 1, padded to 16 column tiles

__host__ __device__ constexpr int rows_m2r(int M2) { return M2 <= 16 ? 16 : M2 <= 32 ? 32 : M2 <= 64 ? 64 : 128; }
size_t kernel_rows_lds_floats(int M2) { return (size_t)kRowsSamples * (rows_m2r(M2) + 4) + kRowsSamples; }

template <int M2R>
__global__ __launch_bounds__(kRowsThreads) void kernel_rows_kernel(const TrainJob* jobs, const int4* items,
                                                                   TrainCommon cm) {
  constexpr int Q = M2R / 4, STR = M2R + 4;  // STR = 4 (mod 64): conflict-free column-tile reads
  extern __shared__ float rows_lds[];
  float* xs = rows_lds;                      // [kRowsSamples][STR] samples ilo ..
  float* xn = rows_lds + kRowsSamples * STR; // their squared norms
  const int4 it = items[blockIdx.x];
  const TrainJob& j = jobs[it.x];
  const int n0 = it.y, l0 = it.z;
  const int M2 = j.M2, M = M2 / 2, cap = j.cap, W = cm.W, T = 2 * j.P;
  const int ilo = n0 - l0 - (kRowsLags - 1);
  // the training groups of a detector OR their flags into a cleared word
  if (n0 == 0 && l0 == 0 && threadIdx.x == 0) to_global(j.state)[3] = 0;
  const auto rx = to_global(j.rx);
  // component m of training vector i (0 outside the sequence or the width):
  // a clamped, unconditional load and a sign/mask applied afterwards
  auto comp = [&](int i, int m) {
    const bool ok = i >= 0 && i < T && m < M2, odd = (i & 1) != 0;
    const int ic = ok ? i : 0, mc = m < M2 ? m : 0;
    const float sg = ok ? (odd && mc >= M ? -1.0f : 1.0f) : 0.0f;
    return sg * rx[(size_t)(ic >> 1) * M2 + (odd ? (mc < M ? mc + M : mc - M) : mc)];
  };
  {
    constexpr int B = 8;                     // loads in flight per thread
    constexpr int N = kRowsSamples * M2R;
    for (int e0 = threadIdx.x; e0 < N; e0 += B * kRowsThreads) {
      float v[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int e = e0 + u * kRowsThreads;
        const int ec = e < N ? e : e0;
        v[u] = comp(ilo + ec / M2R, ec % M2R);
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int e = e0 + u * kRowsThreads;
        if (e < N) xs[(e / M2R) * STR + e % M2R] = v[u];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < kRowsSamples) {
    const float* x = xs + threadIdx.x * STR;
    float n4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int m = 0; m < M2R; ++m) n4[m & 3] = fmaf(x[m], x[m], n4[m & 3]);
    xn[threadIdx.x] = (n4[0] + n4[1]) + (n4[2] + n4[3]);
  }

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  // A operand: step n0 + 16 w + c, components g Q .. g Q + Q - 1
  float a[Q];
  float an = 0.0f;
#pragma unroll
  for (int s = 0; s < Q; ++s) {
    a[s] = comp(n0 + 16 * w + c, g * Q + s);
    an = fmaf(a[s], a[s], an);
  }
  an += __shfl_xor(an, 16);
  an += __shfl_xor(an, 32);                  // ||r_{n0+16w+c}||^2 in every lane of column c
  float nn[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) nn[i] = __shfl(an, 4 * g + i);   // steps 16 w + 4 g + i
  __syncthreads();

  floatx4 acc[9];
#pragma unroll
  for (int u = 0; u < 9; ++u) acc[u] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int s0 = 0; s0 < Q; s0 += 4) {
#pragma unroll
    for (int u = 0; u < 9; ++u) {
      const floatx4 b4 = *reinterpret_cast<const floatx4*>(xs + (16 * (w + u) + c) * STR + g * Q + s0);
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s0 + t], b4[t], acc[u], 0, 0, 0);
    }
  }

  // outputs: acc[u] lane (c, g) row i = step n0 + 16 w + 4 g + i against sample
  // ilo + 16 (w + u) + c, i.e. lag l0 + 127 + 4 g + i - 16 u - c
  auto glag = to_global(j.glag);
  auto kwg = to_global(j.kw);
#pragma unroll
  for (int u = 0; u < 9; ++u) {
    const int q = 16 * (w + u) + c;          // staged sample
    const float xq = xn[q];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * w + 4 * g + i, n = n0 + r;
      const int lr = kRowsLags - 1 + 4 * g + i - 16 * u - c;   // lag - l0
      const int lag = l0 + lr;
      if (lr < 0 || lr >= kRowsLags || lag >= cap || n >= T) continue;
      const bool inseq = n - lag >= 0;
      const float dot = lag == 0 ? nn[i] : acc[u][i];
      const float d2 = fmaxf(nn[i] + xq - 2.0f * dot, 0.0f);
      const float kg = !inseq ? 0.0f : lag == 0 ? 1.0f : __builtin_amdgcn_exp2f(-j.c2 * d2);
      glag[(size_t)n * cap + lag] = kg;
      if (lag < W) kwg[(size_t)n * W + lag] = inseq ? fmaf(cm.wl, dot, cm.wg * kg) : 0.0f;
    }
  }
}

template <int M2P, int KP, int SLOTS>
hipError_t launch_one(const TrainArgs& a, hipStream_t stream) {
  const size_t bytes = lds_bytes_for(a.cm.W, KP, M2P, SLOTS, a.cap);
  auto kern = train_kernel<M2P, KP, SLOTS>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(a.n_inst), dim3(kThreads), bytes, stream, a);
  return hipGetLastError();
}

template <int M2P, int KP>
hipError_t pick_slots(const TrainArgs& a, hipStream_t stream) {
  switch (slots_for(M2P, KP, a.cm.W, a.cap)) {
    case 1: if constexpr (1 * (M2P + KP) <= 128) return launch_one<M2P, KP, 1>(a, stream); break;
    case 2: if constexpr (2 * (M2P + KP) <= 128) return launch_one<M2P, KP, 2>(a, stream); break;
    case 4: if constexpr (4 * (M2P + KP) <= 128) return launch_one<M2P, KP, 4>(a, stream); break;
    case 8: if constexpr (8 * (M2P + KP) <= 128) return launch_one<M2P, KP, 8>(a, stream); break;
    case 0: return launch_one<M2P, KP, 0>(a, stream);
    default: break;
  }
  return launch_one<M2P, KP, -1>(a, stream);
}

template <int M2P>
hipError_t pick_k(const TrainArgs& a, hipStream_t stream) {
  if (a.K <= 4) return pick_slots<M2P, 4>(a, stream);
  if (a.K <= 8) return pick_slots<M2P, 8>(a, stream);
  return pick_slots<M2P, 16>(a, stream);
}

}  // namespace

hipError_t launch_train(const TrainArgs& a, hipStream_t stream) {
  if (a.M2 <= 16) return pick_k<16>(a, stream);
  if (a.M2 <= 32) return pick_k<32>(a, stream);
  if (a.M2 <= 64) return pick_k<64>(a, stream);
  if (a.M2 <= 128) return pick_k<128>(a, stream);
  return hipErrorInvalidValue;
}

// Specialisation of the table kernel for a shape (register-resident slots
// that the table does not hold take the model-buffer path).
static int table_slots(int M2, int K, int W, int cap) {
  const int M2P = m2p_for(M2), KP = kp_for(K);
  const int slots = slots_for(M2P, KP, W, cap);
  if (in_table(M2P, KP, slots)) return slots;
  return lds_floats(W, KP, M2P) + (size_t)cap * KP <= kLdsFloatsMax ? 0 : -1;
}

bool train_in_table(int M2) { return M2 <= 64; }

int train_rows_variant(int M2, int K, int cap) {
  const int need = (cap + kThreads - 1) / kThreads;
  if (M2 > 128 || K > 16 || need > 16 || (need > 8 && K > 4)) return -1;
  const int M2P = m2p_for(M2), KP = kp_for(K);
  const int mi = M2P == 16 ? 0 : M2P == 32 ? 1 : M2P == 64 ? 2 : 3;
  if (need > 8) return 48 + mi;               // 16 slots per thread, four users
  const int ki = KP == 4 ? 0 : KP == 8 ? 1 : 2;
  const int si = need <= 1 ? 0 : need <= 2 ? 1 : need <= 4 ? 2 : 3;
  return (mi * 3 + ki) * 4 + si;
}

int train_rows_max_users(int cap) { return (cap + kThreads - 1) / kThreads > 8 ? 4 : 16; }

size_t train_rows_lds_bytes(int W, int M2, int K) { return lds_floats(W, kp_for(K), m2p_for(M2)) * sizeof(float); }

int kernel_rows_tile_steps() { return kRowsTile; }
int kernel_rows_tile_lags() { return kRowsLags; }

template <int M2R>
static hipError_t launch_rows_m(const TrainJob* jobs, const int4* items, int n_items, const TrainCommon& cm,
                                hipStream_t stream) {
  const size_t bytes = kernel_rows_lds_floats(M2R) * sizeof(float);
  auto kern = kernel_rows_kernel<M2R>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(n_items), dim3(kRowsThreads), bytes, stream, jobs, items, cm);
  return hipGetLastError();
}

// Every job of one launch runs with the width of the widest (max_M2): the
// components past a job's 2M are zeros.
hipError_t launch_kernel_rows(const TrainJob* jobs, const int4* items, int n_items, int max_M2,
                              const TrainCommon& cm, hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  switch (rows_m2r(max_M2)) {
    case 16: return launch_rows_m<16>(jobs, items, n_items, cm, stream);
    case 32: return launch_rows_m<32>(jobs, items, n_items, cm, stream);
    case 64: return launch_rows_m<64>(jobs, items, n_items, cm, stream);
    default: return launch_rows_m<128>(jobs, items, n_items, cm, stream);
  }
}

hipError_t launch_train_rows(const TrainJob* jobs, int n, const TrainCommon& cm, size_t lds_bytes,
                             hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(train_rows_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(train_rows_kernel, dim3(n), dim3(kThreads), lds_bytes, stream, jobs, cm);
  return hipGetLastError();
}

int train_variant(int M2, int K, int W, int cap) {
  return variant_of(m2p_for(M2), kp_for(K), table_slots(M2, K, W, cap));
}

size_t train_lds_bytes(int W, int M2, int K, int cap) {
  return lds_bytes_for(W, kp_for(K), m2p_for(M2), table_slots(M2, K, W, cap), cap);
}

hipError_t launch_train_table(const TrainJob* jobs, int n, const TrainCommon& cm, size_t lds_bytes,
                              hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(train_table_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(train_table_kernel, dim3(n), dim3(kThreads), lds_bytes, stream, jobs, cm);
  return hipGetLastError();
}

}  // namespace apsm
