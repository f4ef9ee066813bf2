// Differentiable unrolled APSM: forward passes, validation loss and the
// hand-written adjoint (reverse sweep) with pass checkpointing.
//
// Forward (Sec. II-D eqn:apsm with eqn:beta, repeated): an iteration is one
// pass of the windowed parallel projections over the T = 2P real training
// samples; pass 1 is the training of Sec. II-D with an unbounded dictionary
// (every training sample owns a Gaussian coefficient, zero until its own
// step), later passes project onto the same hyperslabs again.  The window
// restarts with each pass; q_j = omega[n-j] / sum_{s<|J_n|} omega[s].  The
// frozen filters are then evaluated on validation vectors (Sec. III-B) and
// L = mean over instances, users and symbols of |g_k - b_k|^2.
//
// Step n of a pass, for window members j (slot s = n - j) and users k:
//   e_jk = w_k . r_j + sum_i alpha_ik G_ij,  G_ij = exp(-D_ij / (2 sigma^2))
//   x = e - b,  beta = -sign(x) max(|x| - eps, 0) / kappa_jj,
//   c = mu q_s beta,  w_k += wL sum_j c_jk r_j,  alpha_jk += wG c_jk.
// Adjoint of that step, from (wbar, abar) of the state after it:
//   cbar_jk = wL wbar_k . r_j + wG abar_jk
//   betabar = mu q_s cbar,  mubar += q_s beta cbar,  qbar_s += mu sum_k beta cbar
//   xbar = -betabar [|x| > eps] / kappa_jj,  epsbar += betabar sign(x) [|x| > eps] / kappa_jj
//   sigmabar += xbar_jk h_jk,  h_jk = sum_i alpha_ik G_ij D_ij / sigma^3 (taped)
//   omegabar_p += (qbar_p - sum_s qbar_s q_s) / Z
//   wbar_k += sum_j xbar_jk r_j,  abar_ik += sum_j xbar_jk G_ij.
// The reverse sweep needs only x and h of each step (the tape), recorded by
// re-running the forward of one checkpoint segment at a time.
//
// One workgroup per instance runs the sequential passes; G and D of the
// training samples are computed once per forward call and read per step
// along the window's columns (contiguous, since window members are
// consecutive samples).  Per-instance gradient parts are accumulated in
// double and reduced over instances in a fixed order (deterministic, and
// independent of the checkpoint interval).
#include "apsm_internal.h"

namespace apsm {
namespace {

constexpr int kT = 256;                // threads per workgroup (set-up, validation, reductions)

// Threads of the sequential pass and reverse kernels: the per-step work is
// spread over as many lanes as the LDS of the partial sums allows.
template <int KP>
constexpr int seq_threads() { return KP <= 8 ? 1024 : 512; }

// The Gaussian coefficients (forward) or their adjoints (reverse), [T][KP],
// are kept in LDS after the kernel's other dynamic arrays (`before` floats,
// the offset rounded up to 16 bytes for the vector reads) when the whole
// fits this budget of dynamic LDS, else in the workspace.
constexpr size_t kDynLdsFloats = 36864;      // 144 KiB
__host__ __device__ inline size_t coef_lds_offset(size_t floats_before) { return (floats_before + 3) / 4 * 4; }
__host__ __device__ inline bool coef_in_lds(int T, int KP, size_t before) {
  return coef_lds_offset(before) + (size_t)T * KP <= kDynLdsFloats;
}

__device__ __forceinline__ float comp(const float* rx, int M2, int n, int m) {
  // component m of real sample n: r_{2t} = r1(t), r_{2t+1} = r2(t) = [Im; -Re]
  const int M = M2 >> 1;
  const float* src = rx + (size_t)(n >> 1) * M2;
  if ((n & 1) == 0) return src[m];
  return m < M ? src[m + M] : -src[m - M];
}

__device__ __forceinline__ float target(const float* sym, int K, int n, int k) {
  return sym[((size_t)(n >> 1) * K + k) * 2 + (n & 1)];
}

struct Inst {
  float* G;       // [T][T]
  float* Dm;      // [T][T]
  float* ck;      // [NC][K*M2P + T*KP]
  float* st;      // [K*M2P + T*KP]  state after the forward passes: w then alpha
  float* sc;      // [K*M2P + T*KP]  state of the segment re-runs of the reverse sweep
  float* tx;      // [E][T][W][KP]
  float* th;      // [E][T][W][KP]
  float* adj;     // [K*M2P + T*KP]  wbar, then the adjoint of alpha from the validation loss
  float* X;       // [T][KP]         step adjoints accumulated by sample (reverse sweep)
  float* fbar;    // [Sr][KP]
  float* lpart;   // [nvb]
  float* spart;   // [nib]
  double* gpart;  // [4 + APSM_MAX_WINDOW]: sigma_raw, eps, mu, pad, omega[]
};

__device__ Inst inst_of(const UnrolledArgs& a, int b) {
  unsigned char* base = static_cast<unsigned char*>(a.ws) + (size_t)b * a.inst_bytes;
  Inst I;
  I.G = reinterpret_cast<float*>(base + a.off_G);
  I.Dm = reinterpret_cast<float*>(base + a.off_D);
  I.ck = reinterpret_cast<float*>(base + a.off_ck);
  I.st = reinterpret_cast<float*>(base + a.off_st);
  I.sc = reinterpret_cast<float*>(base + a.off_sc);
  I.tx = reinterpret_cast<float*>(base + a.off_tx);
  I.th = reinterpret_cast<float*>(base + a.off_th);
  I.adj = reinterpret_cast<float*>(base + a.off_adj);
  I.X = reinterpret_cast<float*>(base + a.off_X);
  I.fbar = reinterpret_cast<float*>(base + a.off_fbar);
  I.lpart = reinterpret_cast<float*>(base + a.off_lpart);
  I.spart = reinterpret_cast<float*>(base + a.off_spart);
  I.gpart = reinterpret_cast<double*>(base + a.off_gpart);
  return I;
}

// ---------------------------------------------------------------- Gram
// G_ij and D_ij of the training samples, 16 x 16 pairs per workgroup.
__global__ __launch_bounds__(kT) void unr_gram_kernel(UnrolledArgs a) {
  __shared__ float ri[16][APSM_MAX_M2 + 1], rj[16][APSM_MAX_M2 + 1];
  const int b = blockIdx.z;
  const Inst I = inst_of(a, b);
  const float* rx = a.rx_pilot + (size_t)b * a.P * a.M2;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  for (int e = threadIdx.x; e < 16 * a.M2; e += kT) {
    const int r = e / a.M2, m = e - r * a.M2;
    ri[r][m] = i0 + r < a.T ? comp(rx, a.M2, i0 + r, m) : 0.0f;
    rj[r][m] = j0 + r < a.T ? comp(rx, a.M2, j0 + r, m) : 0.0f;
  }
  __syncthreads();
  const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;
  const int i = i0 + ti, j = j0 + tj;
  if (i >= a.T || j >= a.T) return;
  float d = 0.0f;
  for (int m = 0; m < a.M2; ++m) {
    const float t = ri[ti][m] - rj[tj][m];
    d = fmaf(t, t, d);
  }
  const float sigma = a.theta[0];
  const float c = 1.0f / (2.0f * sigma * sigma);
  I.G[(size_t)i * a.T + j] = expf(-d * c);
  I.Dm[(size_t)i * a.T + j] = d;
}

// ---------------------------------------------------------------- passes
// Runs passes [p0, p1) of one instance.  The state starts from zero (p0 = 0)
// or from checkpoint p0 / E.  With TAPE, x and h of every step are recorded
// (pass p at tape slot p - p0); otherwise checkpoints are written at the
// start of every pass p with p % E == 0.
//
// The window predictions are kept up to date incrementally, as in the
// training kernel: only the member entering at step n is evaluated against
// the whole expansion (one row of G, and of G D for the sigma sums); every
// member's value then changes by the step's update evaluated at it, from
// the pairwise linear products, G and D among the members (LDS rings).  Each
// pass restarts the window, so a pass depends only on the state at its start
// (the checkpoints), whatever the checkpoint interval.
template <int KP, int NT, bool TAPE>
__global__ __launch_bounds__(NT) void unr_pass_kernel(UnrolledArgs a, int p0, int p1) {
  constexpr int NWV = NT / 64;
  extern __shared__ __attribute__((aligned(16))) float lds[];
  const int b = blockIdx.x;
  const Inst I = inst_of(a, b);
  const int T = a.T, M2 = a.M2, M2P = a.M2P, K = a.K, W = a.W, R = W + 1;
  const float* rx = a.rx_pilot + (size_t)b * a.P * M2;
  const float* sym = a.sym_pilot + (size_t)b * a.P * K * 2;
  float* wl = lds;                          // [K][M2P]
  float* part = wl + K * M2P;               // [NWV][KP] the entering member's prediction, per wave
  float* parth = part + NWV * KP;           // [NWV][KP] its sigma sums
  float* cbuf = parth + NWV * KP;           // [W][KP] coefficients of the step, by position s
  float* ew = cbuf + W * KP;                // [W][KP] f_n(r_j) of the members, by j % W
  float* hw = ew + W * KP;                  // [W][KP] sum_i alpha_ik G_ij D_ij, by j % W
  float* rw = hw + W * KP;                  // [W + 1][M2P] member vectors and r_{n+1}, by j % (W + 1)
  float* lg = rw + R * M2P;                 // [W][W] r_i . r_j of members, by (i % W, j % W)
  float* gg = lg + W * W;                   // [W][W] G_ij
  float* dd = gg + W * W;                   // [W][W] D_ij
  float* om = dd + W * W;                   // [W] omega
  float* zs = om + W;                       // [W + 1] prefix sums of omega
  const int SW = K * M2P + T * KP;
  float* const state = TAPE ? I.sc : I.st;
  // [T][KP]: in LDS when it fits (written back to the state at the end)
  const size_t before = (size_t)K * M2P + 2 * NWV * KP + 3 * W * KP + (size_t)R * M2P + 3 * W * W + 2 * W + 1;
  const bool alds = coef_in_lds(T, KP, before);
  float* alpha = alds ? lds + coef_lds_offset(before) : state + K * M2P;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  const float eps = a.theta[1], mu = a.theta[2];
  for (int s = tid; s < W; s += NT) om[s] = a.theta[3 + s];
  if (tid == 0) {
    float z = 0.0f;
    zs[0] = 0.0f;
    for (int s = 0; s < W; ++s) { z += a.theta[3 + s]; zs[s + 1] = z; }
  }
  // initial state
  const float* src = p0 == 0 ? nullptr : I.ck + (size_t)(p0 / a.E) * SW;
  for (int e = tid; e < K * M2P; e += NT) wl[e] = src ? src[e] : 0.0f;
  for (int e = tid; e < T * KP; e += NT) alpha[e] = src ? src[K * M2P + e] : 0.0f;
  __syncthreads();

  for (int p = p0; p < p1; ++p) {
    if (!TAPE && p % a.E == 0) {
      float* dst = I.ck + (size_t)(p / a.E) * SW;
      for (int e = tid; e < K * M2P; e += NT) dst[e] = wl[e];
      for (int e = tid; e < T * KP; e += NT) dst[K * M2P + e] = alpha[e];
    }
    if (tid < M2P) rw[tid] = tid < M2 ? comp(rx, M2, 0, tid) : 0.0f;   // r_0
    __syncthreads();
    for (int n = 0; n < T; ++n) {
      const int L = n + 1 < W ? n + 1 : W;
      const int jr = n % W, vr = n % R;
      // phase 1: the entering member r_n against the expansion (per-wave sums)
      {
        float pe[KP], ph[KP];
#pragma unroll
        for (int k = 0; k < KP; ++k) { pe[k] = 0.0f; ph[k] = 0.0f; }
        const float* grow = I.G + (size_t)n * T;
        const float* drow = I.Dm + (size_t)n * T;
        for (int i = tid; i < T; i += NT) {
          const float g = grow[i];
          const float4* ar = reinterpret_cast<const float4*>(alpha + (size_t)i * KP);
          const float gd = TAPE ? g * drow[i] : 0.0f;
#pragma unroll
          for (int q = 0; q < KP / 4; ++q) {
            const float4 v = ar[q];
            pe[4 * q] = fmaf(v.x, g, pe[4 * q]);
            pe[4 * q + 1] = fmaf(v.y, g, pe[4 * q + 1]);
            pe[4 * q + 2] = fmaf(v.z, g, pe[4 * q + 2]);
            pe[4 * q + 3] = fmaf(v.w, g, pe[4 * q + 3]);
            if constexpr (TAPE) {
              ph[4 * q] = fmaf(v.x, gd, ph[4 * q]);
              ph[4 * q + 1] = fmaf(v.y, gd, ph[4 * q + 1]);
              ph[4 * q + 2] = fmaf(v.z, gd, ph[4 * q + 2]);
              ph[4 * q + 3] = fmaf(v.w, gd, ph[4 * q + 3]);
            }
          }
        }
#pragma unroll
        for (int k = 0; k < KP; ++k) {
          for (int off = 32; off > 0; off >>= 1) {
            pe[k] += __shfl_xor(pe[k], off);
            if constexpr (TAPE) ph[k] += __shfl_xor(ph[k], off);
          }
        }
        if (lane == 0) {
#pragma unroll
          for (int k = 0; k < KP; ++k) {
            part[wave * KP + k] = pe[k];
            parth[wave * KP + k] = ph[k];
          }
        }
      }
      // the entering member's pairs with the members (itself included)
      for (int s = tid; s < L; s += NT) {
        const int j = n - s, jm = j % W;
        const float* r1 = rw + vr * M2P;
        const float* r2 = rw + (j % R) * M2P;
        float d = 0.0f;
        for (int m = 0; m < M2; ++m) d = fmaf(r1[m], r2[m], d);
        const float g = I.G[(size_t)n * T + j], dv = I.Dm[(size_t)n * T + j];
        lg[jr * W + jm] = d;
        lg[jm * W + jr] = d;
        gg[jr * W + jm] = g;
        gg[jm * W + jr] = g;
        dd[jr * W + jm] = dv;
        dd[jm * W + jr] = dv;
      }
      __syncthreads();
      // phase 2: predictions, projection coefficients, tape
      const float Z = zs[L];
      for (int t = tid; t < L * KP; t += NT) {
        const int s = t / KP, k = t - s * KP;
        float c = 0.0f;
        if (k < K) {
          const int j = n - s, jm = j % W;
          float e, h;
          if (s == 0) {
            e = 0.0f;
            h = 0.0f;
            for (int w = 0; w < NWV; ++w) {
              e += part[w * KP + k];
              h += parth[w * KP + k];
            }
            float lin = 0.0f;
            for (int m = 0; m < M2; ++m) lin = fmaf(wl[k * M2P + m], rw[vr * M2P + m], lin);
            e += lin;
            ew[jm * KP + k] = e;
            hw[jm * KP + k] = h;
          } else {
            e = ew[jm * KP + k];
            h = hw[jm * KP + k];
          }
          const float x = e - target(sym, K, j, k);
          const float kjj = a.wl * lg[jm * W + jm] + a.wg;
          const float mag = fabsf(x) - eps;
          const float beta = (mag > 0.0f && kjj > 0.0f) ? -copysignf(mag, x) / kjj : 0.0f;
          c = mu * (om[s] / Z) * beta;
          if constexpr (TAPE) {
            const size_t o = (((size_t)(p - p0) * T + n) * W + s) * KP + k;
            I.tx[o] = x;
            I.th[o] = h;
          }
        }
        cbuf[s * KP + k] = c;
      }
      __syncthreads();
      // phase 3: state update (every coefficient from the same f_n) and the
      // members' running values after it (those that stay in the window)
      for (int e = tid; e < K * M2; e += NT) {
        const int k = e / M2, m = e - k * M2;
        float acc = 0.0f;
        for (int s = 0; s < L; ++s) acc = fmaf(cbuf[s * KP + k], rw[((n - s) % R) * M2P + m], acc);
        wl[k * M2P + m] = fmaf(a.wl, acc, wl[k * M2P + m]);
      }
      for (int t = tid; t < L * KP; t += NT) {
        const int s = t / KP, k = t - s * KP;
        if (k < K) alpha[(size_t)(n - s) * KP + k] = fmaf(a.wg, cbuf[s * KP + k], alpha[(size_t)(n - s) * KP + k]);
        if (k < K && s < W - 1) {
          const int im = (n - s) % W;
          float de = 0.0f, dh = 0.0f;
          for (int s2 = 0; s2 < L; ++s2) {
            const int jm2 = (n - s2) % W;
            const float c = cbuf[s2 * KP + k];
            const float gv = gg[im * W + jm2];
            de = fmaf(c, fmaf(a.wl, lg[im * W + jm2], a.wg * gv), de);
            if constexpr (TAPE) dh = fmaf(c * a.wg, gv * dd[im * W + jm2], dh);
          }
          ew[im * KP + k] += de;
          if constexpr (TAPE) hw[im * KP + k] += dh;
        }
      }
      if (n + 1 < T && tid < M2P) rw[((n + 1) % R) * M2P + tid] = tid < M2 ? comp(rx, M2, n + 1, tid) : 0.0f;
      __syncthreads();
    }
  }
  for (int e = tid; e < K * M2P; e += NT) state[e] = wl[e];
  if (alds)
    for (int e = tid; e < T * KP; e += NT) state[K * M2P + e] = alpha[e];
}

// ---------------------------------------------------------------- validation
// f on the validation vectors (real vector v = 2t + l of symbol t), the
// squared-error partial sums and dL/df = 2 (f - b) / N.
template <int KP, int M2P>
__global__ __launch_bounds__(kT) void unr_val_fwd_kernel(UnrolledArgs a) {
  __shared__ float dv[64][M2P + 1];
  __shared__ float da[64][KP];
  __shared__ float red[kT];
  const int b = blockIdx.y;
  const Inst I = inst_of(a, b);
  const int T = a.T, M2 = a.M2, WS = a.M2P, K = a.K, Sr = 2 * a.S;
  const float* rx = a.rx_pilot + (size_t)b * a.P * M2;
  const float* rv = a.rx_val + (size_t)b * a.S * M2;
  const float* sv = a.sym_val + (size_t)b * a.S * K * 2;
  const float* w = I.st;
  const float* alpha = I.st + K * WS;
  const float sigma = a.theta[0];
  const float c = 1.0f / (2.0f * sigma * sigma);
  const int v = blockIdx.x * kT + threadIdx.x;
  const bool valid = v < Sr;
  const int vv = valid ? v : 0;
  float x[M2P];
  float f[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) f[k] = 0.0f;
#pragma unroll
  for (int m = 0; m < M2P; ++m) x[m] = m < M2 ? comp(rv, M2, vv, m) : 0.0f;
  for (int i0 = 0; i0 < T; i0 += 64) {
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * M2P; e += kT) {
      const int r = e / M2P, m = e - r * M2P;
      dv[r][m] = (i0 + r < T && m < M2) ? comp(rx, M2, i0 + r, m) : 0.0f;
    }
    for (int e = threadIdx.x; e < 64 * KP; e += kT) {
      const int r = e / KP, k = e - r * KP;
      da[r][k] = i0 + r < T ? alpha[(size_t)(i0 + r) * KP + k] : 0.0f;
    }
    __syncthreads();
    const int n = T - i0 < 64 ? T - i0 : 64;
    for (int r = 0; r < n; ++r) {
      float d = 0.0f;
#pragma unroll
      for (int m = 0; m < M2P; ++m) {
        const float t = x[m] - dv[r][m];
        d = fmaf(t, t, d);
      }
      const float g = expf(-d * c);
#pragma unroll
      for (int k = 0; k < KP; ++k) f[k] = fmaf(da[r][k], g, f[k]);
    }
  }
  float sq = 0.0f;
  for (int k = 0; k < K; ++k) {
    float lin = 0.0f;
#pragma unroll
    for (int m = 0; m < M2P; ++m) lin = fmaf(m < M2 ? w[k * WS + m] : 0.0f, x[m], lin);
    const float err = f[k] + lin - target(sv, K, vv, k);
    if (valid) {
      sq = fmaf(err, err, sq);
      I.fbar[(size_t)v * KP + k] = 2.0f * err * a.inv_count;
    }
  }
  red[threadIdx.x] = valid ? sq : 0.0f;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) I.lpart[blockIdx.x] = red[0];
}

// Adjoint of the validation evaluation: abar_i = sum_v fbar_v G(r_i, v),
// sigma part sum_v sum_k fbar_vk alpha_ik G D (times 1/sigma^3 later), and
// (block row nib) wbar = sum_v fbar_v v.  64 entries per workgroup, four
// lanes per entry over the vectors of each staged tile.
template <int KP, int M2P>
__global__ __launch_bounds__(kT) void unr_val_bwd_kernel(UnrolledArgs a) {
  __shared__ float vt[64][M2P + 1];
  __shared__ float fb[64][KP];
  __shared__ float red[kT][KP + 1];
  const int b = blockIdx.y;
  const Inst I = inst_of(a, b);
  const int T = a.T, M2 = a.M2, WS = a.M2P, K = a.K, Sr = 2 * a.S;
  const float* rx = a.rx_pilot + (size_t)b * a.P * M2;
  const float* rv = a.rx_val + (size_t)b * a.S * M2;
  const float* alpha = I.st + K * WS;
  float* wbar = I.adj;
  float* abar = I.adj + K * WS;
  const int nib = (T + 63) / 64;
  if ((int)blockIdx.x == nib) {
    // wbar_k,m = sum_v fbar_vk v_m
    for (int e = threadIdx.x; e < K * WS; e += kT) {
      const int k = e / WS, m = e - k * WS;
      float acc = 0.0f;
      if (m < M2)
        for (int v = 0; v < Sr; ++v) acc = fmaf(I.fbar[(size_t)v * KP + k], comp(rv, M2, v, m), acc);
      wbar[e] = acc;
    }
    return;
  }
  const float sigma = a.theta[0];
  const float c = 1.0f / (2.0f * sigma * sigma);
  const int li = threadIdx.x >> 2, lane = threadIdx.x & 3;
  const int i = blockIdx.x * 64 + li;
  const bool valid = i < T;
  float r[M2P];
#pragma unroll
  for (int m = 0; m < M2P; ++m) r[m] = (valid && m < M2) ? comp(rx, M2, i, m) : 0.0f;
  float al[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) al[k] = valid ? alpha[(size_t)i * KP + k] : 0.0f;
  float ab[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) ab[k] = 0.0f;
  float sg = 0.0f;
  for (int v0 = 0; v0 < Sr; v0 += 64) {
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * M2P; e += kT) {
      const int q = e / M2P, m = e - q * M2P;
      vt[q][m] = (v0 + q < Sr && m < M2) ? comp(rv, M2, v0 + q, m) : 0.0f;
    }
    for (int e = threadIdx.x; e < 64 * KP; e += kT) {
      const int q = e / KP, k = e - q * KP;
      fb[q][k] = v0 + q < Sr ? I.fbar[(size_t)(v0 + q) * KP + k] : 0.0f;
    }
    __syncthreads();
    for (int q = lane; q < 64; q += 4) {
      float d = 0.0f;
#pragma unroll
      for (int m = 0; m < M2P; ++m) {
        const float t = r[m] - vt[q][m];
        d = fmaf(t, t, d);
      }
      const float g = expf(-d * c);
      float s = 0.0f;
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        ab[k] = fmaf(fb[q][k], g, ab[k]);
        s = fmaf(fb[q][k], al[k], s);
      }
      sg = fmaf(s, g * d, sg);
    }
  }
  // fixed-order reduction over the four lanes of each entry
#pragma unroll
  for (int k = 0; k < KP; ++k) red[threadIdx.x][k] = ab[k];
  red[threadIdx.x][KP] = sg;
  __syncthreads();
  if (lane == 0 && valid) {
#pragma unroll
    for (int k = 0; k < KP; ++k)
      abar[(size_t)i * KP + k] = ((red[threadIdx.x][k] + red[threadIdx.x + 1][k]) + red[threadIdx.x + 2][k]) +
                                 red[threadIdx.x + 3][k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float tot = 0.0f;
    for (int q = 0; q < kT; ++q) tot += red[q][KP];
    I.spart[blockIdx.x] = tot;
  }
}

// ---------------------------------------------------------------- reverse
// Reverse sweep over passes [p0, p1) (tape slot p - p0), updating the
// adjoint state and adding this segment's gradient parts to gpart.
//
// The adjoint of alpha is needed only at the window members.  It is kept
// as abar = abar0 + G X, abar0 the validation loss's part (unchanged) and
// X_i the step adjoints xbar accumulated by sample i; a member entering the
// window (in reverse order) is evaluated with one row of G, and the members'
// values then change by the step's xbar through the G block among them.  X
// carries over between segments in the workspace.
template <int KP, int NT>
__global__ __launch_bounds__(NT) void unr_reverse_kernel(UnrolledArgs a, int p0, int p1) {
  constexpr int NWV = NT / 64;
  extern __shared__ __attribute__((aligned(16))) float lds[];
  const int b = blockIdx.x;
  const Inst I = inst_of(a, b);
  const int T = a.T, M2 = a.M2, M2P = a.M2P, K = a.K, W = a.W;
  const float* rx = a.rx_pilot + (size_t)b * a.P * M2;
  float* wb = lds;                         // [K][M2P] wbar
  float* eb = wb + K * M2P;                // [W][KP] xbar (= ebar), by position s
  float* qb = eb + W * KP;                 // [W][KP] qbar parts
  float* abw = qb + W * KP;                // [W][KP] abar of the members, by j % W
  float* red = abw + W * KP;               // [NWV][KP] per-wave sums of a row
  float* rw = red + NWV * KP;              // [W + 1][M2P] member vectors, by j % (W + 1)
  float* nw = rw + (W + 1) * M2P;          // [W + 1] their squared norms
  float* om = nw + W + 1;                  // [W]
  float* zs = om + W;                      // [W + 1]
  __shared__ double dred[NT];
  const float* abar0 = I.adj + K * M2P;
  // X [T][KP]: in LDS when it fits (loaded here, written back at the end)
  const size_t before = (size_t)K * M2P + 3 * W * KP + NWV * KP + (size_t)(W + 1) * (M2P + 1) + 2 * W + 1;
  const bool xl = coef_in_lds(T, KP, before);
  float* X = xl ? lds + coef_lds_offset(before) : I.X;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (xl)
    for (int e = tid; e < T * KP; e += NT) X[e] = I.X[e];
  const float eps = a.theta[1], mu = a.theta[2];
  for (int s = tid; s < W; s += NT) om[s] = a.theta[3 + s];
  if (tid == 0) {
    float z = 0.0f;
    zs[0] = 0.0f;
    for (int s = 0; s < W; ++s) { z += a.theta[3 + s]; zs[s + 1] = z; }
  }
  for (int e = tid; e < K * M2P; e += NT) wb[e] = I.adj[e];
  __syncthreads();
  double g_sig = 0.0, g_eps = 0.0, g_mu = 0.0, g_om = 0.0;   // g_om: lane s of wave 0
  for (int p = p1 - 1; p >= p0; --p) {
    for (int n = T - 1; n >= 0; --n) {
      const int L = n + 1 < W ? n + 1 : W;
      const float Z = zs[L];
      // members entering the window: all of them at the pass's last step,
      // afterwards n - W + 1 (none once the window reaches sample 0)
      const int j_lo = n == T - 1 ? n - L + 1 : n - W + 1;
      const int j_hi = n == T - 1 ? n : n - W + 1;
      for (int j = j_lo < 0 ? 0 : j_lo; j <= j_hi; ++j) {
        if (tid < M2P) rw[(j % (W + 1)) * M2P + tid] = tid < M2 ? comp(rx, M2, j, tid) : 0.0f;
        float acc[KP];
#pragma unroll
        for (int k = 0; k < KP; ++k) acc[k] = 0.0f;
        const float* grow = I.G + (size_t)j * T;
        for (int i = tid; i < T; i += NT) {
          const float g = grow[i];
          const float4* xr = reinterpret_cast<const float4*>(X + (size_t)i * KP);
#pragma unroll
          for (int q = 0; q < KP / 4; ++q) {
            const float4 v = xr[q];
            acc[4 * q] = fmaf(v.x, g, acc[4 * q]);
            acc[4 * q + 1] = fmaf(v.y, g, acc[4 * q + 1]);
            acc[4 * q + 2] = fmaf(v.z, g, acc[4 * q + 2]);
            acc[4 * q + 3] = fmaf(v.w, g, acc[4 * q + 3]);
          }
        }
#pragma unroll
        for (int k = 0; k < KP; ++k)
          for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off);
        if (lane == 0) {
#pragma unroll
          for (int k = 0; k < KP; ++k) red[wave * KP + k] = acc[k];
        }
        __syncthreads();
        if (tid < KP) {
          float v = 0.0f;
          for (int w = 0; w < NWV; ++w) v += red[w * KP + tid];
          abw[(j % W) * KP + tid] = abar0[(size_t)j * KP + tid] + v;
        }
        if (tid == 64) {                   // its squared norm (wave 1; the vector was written before the barrier)
          const float* r = rw + (j % (W + 1)) * M2P;
          float nr = 0.0f;
          for (int m = 0; m < M2; ++m) nr = fmaf(r[m], r[m], nr);
          nw[j % (W + 1)] = nr;
        }
        __syncthreads();
      }
      for (int t = tid; t < L * KP; t += NT) {
        const int s = t / KP, k = t - s * KP;
        float xb = 0.0f, qp = 0.0f;
        if (k < K) {
          const int j = n - s;
          const float* r = rw + (j % (W + 1)) * M2P;
          float dot = 0.0f;
          for (int m = 0; m < M2; ++m) dot = fmaf(wb[k * M2P + m], r[m], dot);
          const float nrm = nw[j % (W + 1)];
          const float cb = a.wl * dot + a.wg * abw[(j % W) * KP + k];
          const size_t o = (((size_t)(p - p0) * T + n) * W + s) * KP + k;
          const float x = I.tx[o], h = I.th[o];
          const float kjj = a.wl * nrm + a.wg;
          const float mag = fabsf(x) - eps;
          const bool act = mag > 0.0f && kjj > 0.0f;
          const float beta = act ? -copysignf(mag, x) / kjj : 0.0f;
          const float q = om[s] / Z;
          const float bb = mu * q * cb;
          g_mu += (double)(q * beta * cb);
          qp = mu * beta * cb;
          xb = act ? -bb / kjj : 0.0f;
          if (act) g_eps += (double)((x > 0.0f ? bb : -bb) / kjj);
          g_sig += (double)xb * (double)h;
        }
        eb[s * KP + k] = xb;
        qb[s * KP + k] = qp;
      }
      __syncthreads();
      // omega: lane s of wave 0 (W <= 64)
      if (tid < 64) {
        float qs = 0.0f, qq = 0.0f;
        if (tid < L) {
          for (int k = 0; k < K; ++k) qs += qb[tid * KP + k];
          qq = qs * (om[tid] / Z);
        }
        for (int off = 32; off > 0; off >>= 1) qq += __shfl_xor(qq, off);
        if (tid < L) g_om += (double)((qs - qq) / Z);
      }
      for (int e = tid; e < K * M2; e += NT) {
        const int k = e / M2, m = e - k * M2;
        float acc = 0.0f;
        for (int s = 0; s < L; ++s) acc = fmaf(eb[s * KP + k], rw[((n - s) % (W + 1)) * M2P + m], acc);
        wb[k * M2P + m] += acc;
      }
      // the step's xbar into X; the members that stay (all but n) by the G block
      for (int t = tid; t < L * KP; t += NT) {
        const int s = t / KP, k = t - s * KP;
        const int j = n - s;
        X[(size_t)j * KP + k] += eb[s * KP + k];
        if (s >= 1) {
          const float* grow = I.G + (size_t)j * T + n;     // G_{j, n - s2} at grow[-s2]
          float acc = 0.0f;
          for (int s2 = 0; s2 < L; ++s2) acc = fmaf(eb[s2 * KP + k], grow[-s2], acc);
          abw[(j % W) * KP + k] += acc;
        }
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < K * M2P; e += NT) I.adj[e] = wb[e];
  if (xl)
    for (int e = tid; e < T * KP; e += NT) I.X[e] = X[e];
  // fixed-order block sums of the scalar parts
  double* gp = I.gpart;
  const double parts[3] = {g_sig, g_eps, g_mu};
  for (int q = 0; q < 3; ++q) {
    dred[tid] = parts[q];
    __syncthreads();
    for (int s2 = NT / 2; s2 > 0; s2 >>= 1) {
      if (tid < s2) dred[tid] += dred[tid + s2];
      __syncthreads();
    }
    if (tid == 0) gp[q] += dred[0];
    __syncthreads();
  }
  if (tid < W) gp[4 + tid] += g_om;
}

// ---------------------------------------------------------------- reductions
__global__ __launch_bounds__(kT) void unr_zero_gpart_kernel(UnrolledArgs a) {
  const Inst I = inst_of(a, blockIdx.x);
  for (int e = threadIdx.x; e < 4 + APSM_MAX_WINDOW; e += kT) I.gpart[e] = 0.0;
  for (int e = threadIdx.x; e < a.T * a.KP; e += kT) I.X[e] = 0.0f;
}

__global__ __launch_bounds__(kT) void unr_loss_kernel(UnrolledArgs a, float* loss) {
  __shared__ double red[kT];
  double acc = 0.0;
  const int nvb = (2 * a.S + kT - 1) / kT;
  for (int b = threadIdx.x; b < a.n; b += kT) {
    const Inst I = inst_of(a, b);
    double s = 0.0;
    for (int q = 0; q < nvb; ++q) s += (double)I.lpart[q];
    acc += s;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(red[0] * (double)a.inv_count);
}

// grad = upstream * (sum over instances of the parts); sigma gets 1/sigma^3.
__global__ __launch_bounds__(kT) void unr_grad_kernel(UnrolledArgs a, float* grad, const float* upstream) {
  const int q = threadIdx.x;
  const int nq = 3 + a.W;
  if (q >= nq) return;
  const int nib = (a.T + 63) / 64;
  double acc = 0.0;
  for (int b = 0; b < a.n; ++b) {
    const Inst I = inst_of(a, b);
    if (q == 0) {
      double s = I.gpart[0];
      for (int t = 0; t < nib; ++t) s += (double)I.spart[t];
      acc += s;
    } else if (q < 3) {
      acc += I.gpart[q];
    } else {
      acc += I.gpart[4 + (q - 3)];
    }
  }
  if (q == 0) {
    const double sg = a.theta[0];
    acc /= sg * sg * sg;
  }
  const double up = upstream ? (double)upstream[0] : 1.0;
  grad[q] = (float)(acc * up);
}

template <int KP>
hipError_t forward_k(const UnrolledArgs& a, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(unr_gram_kernel, dim3((a.T + 15) / 16, (a.T + 15) / 16, a.n), dim3(kT), 0, s, a);
  constexpr int NT = seq_threads<KP>();
  const size_t lds = unrolled_pass_lds(a);
  auto pk = unr_pass_kernel<KP, NT, false>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(pk),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pk, dim3(a.n), dim3(NT), lds, s, a, 0, a.passes);
  const dim3 gv((2 * a.S + kT - 1) / kT, a.n);
  if (a.M2 <= 16) hipLaunchKernelGGL((unr_val_fwd_kernel<KP, 16>), gv, dim3(kT), 0, s, a);
  else if (a.M2 <= 32) hipLaunchKernelGGL((unr_val_fwd_kernel<KP, 32>), gv, dim3(kT), 0, s, a);
  else if (a.M2 <= 64) hipLaunchKernelGGL((unr_val_fwd_kernel<KP, 64>), gv, dim3(kT), 0, s, a);
  else hipLaunchKernelGGL((unr_val_fwd_kernel<KP, 128>), gv, dim3(kT), 0, s, a);
  hipLaunchKernelGGL(unr_loss_kernel, dim3(1), dim3(kT), 0, s, a, loss);
  return hipGetLastError();
}

template <int KP>
hipError_t backward_k(const UnrolledArgs& a, float* grad, const float* upstream, hipStream_t s) {
  hipLaunchKernelGGL(unr_zero_gpart_kernel, dim3(a.n), dim3(kT), 0, s, a);
  const dim3 gb((a.T + 63) / 64 + 1, a.n);
  if (a.M2 <= 16) hipLaunchKernelGGL((unr_val_bwd_kernel<KP, 16>), gb, dim3(kT), 0, s, a);
  else if (a.M2 <= 32) hipLaunchKernelGGL((unr_val_bwd_kernel<KP, 32>), gb, dim3(kT), 0, s, a);
  else if (a.M2 <= 64) hipLaunchKernelGGL((unr_val_bwd_kernel<KP, 64>), gb, dim3(kT), 0, s, a);
  else hipLaunchKernelGGL((unr_val_bwd_kernel<KP, 128>), gb, dim3(kT), 0, s, a);
  constexpr int NT = seq_threads<KP>();
  const size_t lds_p = unrolled_pass_lds(a);
  const size_t lds_r = unrolled_reverse_lds(a);
  auto pk = unr_pass_kernel<KP, NT, true>;
  auto rk = unr_reverse_kernel<KP, NT>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(pk),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_p);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(rk), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_r);
  if (e != hipSuccess) return e;
  const int nseg = (a.passes + a.E - 1) / a.E;
  for (int sgm = nseg - 1; sgm >= 0; --sgm) {
    const int p0 = sgm * a.E;
    const int p1 = p0 + a.E < a.passes ? p0 + a.E : a.passes;
    hipLaunchKernelGGL(pk, dim3(a.n), dim3(NT), lds_p, s, a, p0, p1);
    hipLaunchKernelGGL(rk, dim3(a.n), dim3(NT), lds_r, s, a, p0, p1);
  }
  hipLaunchKernelGGL(unr_grad_kernel, dim3(1), dim3(kT), 0, s, a, grad, upstream);
  return hipGetLastError();
}

}  // namespace

size_t unrolled_pass_lds(const UnrolledArgs& a) {
  const int nwv = (a.KP <= 8 ? seq_threads<8>() : seq_threads<16>()) / 64;
  const size_t W = a.W;
  const size_t before = (size_t)a.K * a.M2P + 2 * (size_t)nwv * a.KP + 3 * W * a.KP + (W + 1) * a.M2P +
                        3 * W * W + 2 * W + 1;
  return sizeof(float) * (coef_in_lds(a.T, a.KP, before) ? coef_lds_offset(before) + (size_t)a.T * a.KP : before);
}

size_t unrolled_reverse_lds(const UnrolledArgs& a) {
  const int nwv = (a.KP <= 8 ? seq_threads<8>() : seq_threads<16>()) / 64;
  const size_t before = (size_t)a.K * a.M2P + 3 * (size_t)a.W * a.KP + (size_t)nwv * a.KP +
                        (size_t)(a.W + 1) * (a.M2P + 1) + 2 * a.W + 1;
  return sizeof(float) * (coef_in_lds(a.T, a.KP, before) ? coef_lds_offset(before) + (size_t)a.T * a.KP : before);
}

hipError_t launch_unrolled_forward(const UnrolledArgs& a, float* loss, hipStream_t s) {
  if (a.KP == 4) return forward_k<4>(a, loss, s);
  if (a.KP == 8) return forward_k<8>(a, loss, s);
  return forward_k<16>(a, loss, s);
}

hipError_t launch_unrolled_backward(const UnrolledArgs& a, float* grad, const float* upstream, hipStream_t s) {
  if (a.KP == 4) return backward_k<4>(a, grad, upstream, s);
  if (a.KP == 8) return backward_k<8>(a, grad, upstream, s);
  return backward_k<16>(a, grad, upstream, s);
}

}  // namespace apsm
