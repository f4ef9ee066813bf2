/*
 * apsm.h - C ABI of the MI355X (gfx950) APSM partially linear multiuser
 * detector library (libapsm.so).
 *
 * The method is the one of Mehlhose et al., "GPU-accelerated partially linear
 * multiuser detection for 5G and beyond URLLC systems" (arXiv 2201.05024):
 * per user k a real filter f_k in the sum RKHS H = H_L + H_G (Sec. II-B,
 * Fact 1),
 *
 *     f_k(x) = w_k^T x + sum_i alpha[i][k] * exp(-||x - d_i||^2 / (2 sigma^2)),
 *
 * trained by windowed parallel hyperslab projections (Sec. II-D, eqn:apsm,
 * eqn:beta) and evaluated on every received vector for detection (Sec. III-B)
 * with g_k(r) = f_k(r1) + i f_k(r2) (Sec. II-D real split).
 *
 * Conventions shared by every entry point:
 *  - Array pointers are DEVICE pointers unless the comment says HOST.
 *  - A complex vector r in C^M is stored as M2 = 2M float32 values
 *    [Re r_0 .. Re r_{M-1}, Im r_0 .. Im r_{M-1}] (this is r1 of Sec. II-D;
 *    r2 = [Im r; -Re r] is formed inside the kernels and never stored).
 *  - A complex symbol is stored as two float32 values (Re, Im).
 *  - A decided symbol is one uint8 label (gray(i_re) << b) | gray(i_im), b the
 *    bits per axis (1 for QPSK, 2 for 16-QAM), i_re / i_im the per-axis level
 *    index in increasing amplitude order, gray the binary-reflected Gray code.
 *    Constellations have unit average energy: QPSK levels +-1/sqrt2, 16-QAM
 *    levels {-3,-1,1,3}/sqrt10; a value exactly on a threshold takes the
 *    higher level.
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 *    NULL is the null stream).  Arguments are validated on the host before
 *    anything is launched: a call that returns an error launched nothing.
 *  - The caller allocates and owns every device buffer.  The library never
 *    allocates device memory.
 *  - No C++ exception crosses this interface.  Calls on different streams are
 *    independent; calls that write the same buffers must be ordered by the
 *    caller.
 */
#ifndef APSM_H
#define APSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------- */
#define APSM_OK                 0
#define APSM_ERR_INVALID_ARG    1  /* null pointer, non-finite or out-of-range parameter */
#define APSM_ERR_SHAPE          2  /* sizes inconsistent with each other or the model    */
#define APSM_ERR_UNSUPPORTED    3  /* valid but beyond this build's limits (see below)   */
#define APSM_ERR_HIP            4  /* a HIP launch failed; see apsm_last_hip_error()     */
#define APSM_ERR_WORKSPACE      5  /* workspace NULL, smaller than required or not
                                      256-byte aligned                                   */
#define APSM_ERR_NONFINITE      6  /* apsm_get_status: a model status flag reports
                                      non-finite values (see APSM_FLAG_*)                */

/* Status flags in state[3] of a model (apsm_model_t).  Training overwrites
 * the word with its own flags; detection ORs its flag in (atomically, so
 * concurrent detections with one model are safe) and leaves every other
 * model field untouched.  A caller may clear the word by writing 0. */
#define APSM_FLAG_TRAIN_NONFINITE   1  /* a training prediction error was not finite    */
#define APSM_FLAG_DETECT_NONFINITE  2  /* detection met a non-finite received vector
                                          component or produced a non-finite output    */

/* ---- limits of this build ------------------------------------------- */
#define APSM_MAX_M2       128      /* real input dimension 2M                       */
#define APSM_MAX_K        16       /* users per instance                            */
#define APSM_MAX_WINDOW   64       /* sliding-window size W                         */
#define APSM_MAX_DICT     65536    /* dictionary capacity                           */

/* Modulations for apsm_detect: the value is the number of bits per symbol. */
#define APSM_MOD_NONE   0          /* no decisions, soft outputs only               */
#define APSM_MOD_QPSK   2
#define APSM_MOD_QAM16  4

/* Initial filter of a training (apsm_params_t.init). */
#define APSM_INIT_ZERO      0      /* f_0 = 0: the model is reset                                */
#define APSM_INIT_LINEAR    1      /* f_0 = the model's linear part w (e.g. from apsm_linear_mmse),
                                      Gaussian dictionary emptied (needs w_lin > 0)              */
#define APSM_INIT_CONTINUE  2      /* continue the model as it is: its dictionary ring, Gaussian
                                      and linear coefficients and sample count (state[2]) carry on,
                                      the window J_n starts afresh with the new samples (needs
                                      w_lin > 0; one-detector training entry points only)        */

/* Set weights q_j of a training step (apsm_params_t.weights). */
#define APSM_WEIGHTS_POSITION   0  /* uniform 1/|J_n|, or the position weights pos_weights      */
#define APSM_WEIGHTS_VIOLATION  1  /* per user k, q_kj proportional to member j's distance
                                      max(|f_n(r_j) - b_kj| - eps, 0) to its slab (0 for all when
                                      none is violated); pos_weights must be NULL               */
#define APSM_WEIGHTS_ACTIVE     2  /* per user k, q_kj uniform over the members whose set f_n
                                      violates by more than 1e-5, 0 on the others (no update
                                      when none is); pos_weights must be NULL                   */

/* Kind of the closed convex set a training sample defines through the value
 * f(r_j) (apsm_params_t.set_types).  The hyperslab is the detector's set
 * (eqn:convex_set); the others make the training a generic projection engine
 * (Sec. I and Sec. VI: the GPU design serves other projection-based methods
 * in RKHSs).  Each projection moves f(r_j) to the nearest admitted value. */
#define APSM_SET_SLAB    0         /* |f(r_j) - b_j| <= eps                          */
#define APSM_SET_PLANE   1         /* f(r_j) = b_j (eps not used)                    */
#define APSM_SET_UPPER   2         /* f(r_j) <= b_j + eps                            */
#define APSM_SET_LOWER   3         /* f(r_j) >= b_j - eps                            */

/* Design parameters of the iteration (HOST struct).
 *  sigma2      Gaussian kernel width sigma^2 > 0 (Sec. II-A).
 *  eps         hyperslab half-width eps >= 0 (eqn:convex_set).
 *  mu          relaxation in (0, 2): f_{n+1} = f_n + mu * sum_j q_j beta_j kappa(r_j, .);
 *              mu = 1 is exactly eqn:apsm (the q_j sum to one).
 *  w_lin,
 *  w_gauss     weights of the sum space (Sec. II-B), >= 0 and not both 0.
 *  window      W >= 1: J_n = {n-W+1..n} for n >= W-1, else {0..n}.
 *  dict_cap    capacity of the Gaussian dictionary, >= window.  Sample r_n
 *              enters the dictionary at the start of step n; when it is full
 *              the oldest Gaussian term is dropped first (its linear part
 *              stays).  dict_cap >= 2P gives the paper's ever-growing
 *              dictionary exactly.
 *  init        APSM_INIT_*: the initial filter f_0 (Sec. II-D leaves it arbitrary;
 *              Sec. I: a conventional linear filter when channel information
 *              is available) or the continuation of a trained model.
 *  pos_weights HOST pointer to `window` positive floats omega (omega[0] for the
 *              newest set j = n), q_j = omega[n-j] / sum_{i in J_n} omega[n-i];
 *              NULL for uniform q_j = 1/|J_n| (eqn:apsm's weights, Sec. II-D).
 *  weights     APSM_WEIGHTS_*: position weights, weights proportional to the slab
 *              violation, or uniform over the violated sets (Sec. II-D: the q_j
 *              may prioritise sets adaptively).
 *  extrapolate 0, or 1 for the extrapolated relaxation: per user the step
 *              mu * M_n with M_n = sum_j q_j ||P_j f - f||^2 / ||sum_j q_j (P_j f - f)||^2
 *              >= 1 over the window's sets (1 where the denominator vanishes);
 *              mu stays in (0, 2).
 *  set_types   DEVICE pointer to uint8 APSM_SET_* kinds laid out as the pilot
 *              symbols, [P][K][2] (real, imaginary part; [n_inst][P][K][2] for
 *              apsm_train_batched), or NULL for hyperslabs everywhere.  With
 *              violation weights the distance is the one to the sample's set.
 *              Taken by apsm_train, apsm_train_batched and apsm_pocs; the
 *              other entry points return APSM_ERR_UNSUPPORTED for non-NULL. */
typedef struct apsm_params {
  float sigma2;
  float eps;
  float mu;
  float w_lin;
  float w_gauss;
  int32_t window;
  int32_t dict_cap;
  int32_t init;
  const float* pos_weights;
  int32_t weights;
  int32_t extrapolate;
  const uint8_t* set_types;
} apsm_params_t;

/* A trained detector: the whole filter state (Sec. III-B: dictionary plus
 * coefficients).  HOST struct of DEVICE pointers, all caller-allocated.
 *  dict   [M2][dict_cap]  Gaussian dictionary ring, component-major: component m of
 *                         the entry in slot i is dict[m * dict_cap + i] (so that the
 *                         training and packing kernels read it with coalesced
 *                         loads); slot of sample n is n % dict_cap; unused slots
 *                         hold zeros.
 *  alpha  [dict_cap][K]   Gaussian coefficients (wG * gamma_i of Sec. II-D); zero for
 *                         unused slots.
 *  w      [K][M2]         linear coefficients (wL * gamma^(L) of Sec. II-D).
 *  state  int32[4]        written by training: {entries in use, next slot,
 *                         training steps done, status flags (APSM_FLAG_*)};
 *                         detection only ORs APSM_FLAG_DETECT_NONFINITE into
 *                         the flags word.
 *  packed apsm_model_packed_bytes(M2, K, dict_cap) bytes (required): the
 *         same filter re-laid out for the detection kernels (written by
 *         apsm_train and by apsm_model_pack, read by apsm_detect); for
 *         2M <= 64 and K <= 8 it holds the layouts of both detection kernels.
 *         It does not depend on sigma2.
 * sigma2 travels with the call (apsm_detect) rather than in this struct. */
typedef struct apsm_model {
  int32_t M2;
  int32_t K;
  int32_t dict_cap;
  int32_t reserved;           /* must be 0 */
  float* dict;
  float* alpha;
  float* w;
  int32_t* state;
  void* packed;
} apsm_model_t;

/* Size in bytes of apsm_model_t.packed for this shape; 0 if the shape needs
 * no packed form.  Pure host function. */
size_t apsm_model_packed_bytes(int M2, int K, int dict_cap);

/* Rebuild model->packed from dict, alpha and state (e.g. after the caller
 * wrote or modified the model arrays directly).  apsm_train does this
 * itself.  Asynchronous on `stream`; no-op when the packed size is 0. */
int apsm_model_pack(const apsm_model_t* model, void* stream);

/* Training (Sec. II-D eqn:apsm with eqn:beta; Sec. III-B training phase).
 * Starts from the initial filter params->init names (f_0 = 0 resets the
 * model), runs the 2P steps n = 0..2P-1 of the real
 * training sequence r_{2t} = r1(t), r_{2t+1} = r2(t), b_{k,2t} = Re b_k(t),
 * b_{k,2t+1} = Im b_k(t), and packs the result (apsm_model_pack).
 *  params     HOST, see apsm_params_t.
 *  M2         2M, even, 2..APSM_MAX_M2;  K  1..APSM_MAX_K;  P >= 1 pilots.
 *  rx_pilot   [P][M2] received pilot vectors (r1 layout).
 *  sym_pilot  [P][K][2] transmitted pilot symbols (Re, Im).
 *  model      HOST struct; model->M2, K, dict_cap must equal M2, K,
 *             params->dict_cap.
 * Returns APSM_OK or an error code; the filter is ready once the stream
 * reaches the launch. */
int apsm_train(const apsm_params_t* params, int M2, int K, int P,
               const float* rx_pilot, const float* sym_pilot,
               const apsm_model_t* model, void* stream);

/* Training of n_inst detectors of one shape and one parameter set in one
 * launch (one workgroup per detector, so they train concurrently).  Detector
 * i reads rx_pilot + i*P*M2 and sym_pilot + i*P*K*2 (contiguous [n_inst][P][M2]
 * and [n_inst][P][K][2] arrays) and writes models[i].
 *  models     HOST array of n_inst model descriptors, each as for apsm_train.
 * Same results as n_inst apsm_train calls; n_inst = 0 is a no-op. */
int apsm_train_batched(const apsm_params_t* params, int M2, int K, int P, int n_inst,
                       const float* rx_pilot, const float* sym_pilot,
                       const apsm_model_t* models, void* stream);

/* Detection (Sec. III-B): for every received vector r(s), s = 0..S-1,
 * g_k = f_k(r1) + i f_k(r2) with the frozen filter `model` (read only, except
 * that APSM_FLAG_DETECT_NONFINITE is ORed into state[3] when a received
 * vector component or an output is not finite; outputs are still written).
 *  model      HOST struct of a trained model.
 *  sigma2     the kernel width the model was trained with (> 0).
 *  S          number of received vectors, >= 0 (0 launches nothing).
 *  rx         [S][M2] received vectors (r1 layout).
 *  soft       [S][K][2] (Re g_k, Im g_k) output, or NULL.
 *  hard       [S][K] uint8 labels output, or NULL; needs modulation != NONE.
 *  modulation APSM_MOD_NONE / APSM_MOD_QPSK / APSM_MOD_QAM16.
 *  truth      [S][K] uint8 transmitted labels, or NULL.
 *  err_count  [K] int64: the number of s with decided label != truth[s][k]
 *             is ADDED to err_count[k] (zero it first); NULL if truth is NULL.
 * At least one of soft / hard / err_count must be non-NULL. */
int apsm_detect(const apsm_model_t* model, float sigma2, int S,
                const float* rx, float* soft, uint8_t* hard, int modulation,
                const uint8_t* truth, int64_t* err_count, void* stream);

/* Linear MMSE receive filters from channel estimates, as the linear start
 * f_0 of a training (APSM_INIT_LINEAR; Sec. I: initialisation by a
 * conventional linear filter when channel information is available).  For
 * each of n_inst instances with channel H in C^{M x K} (column k: user k's
 * channel, including its power and any known scale of the received
 * vectors) and noise variance n0 per antenna:
 *     U = H (H^H H + n0 I)^{-1},   w_k = [Re u_k; Im u_k],
 * so that w_k . r1 + i w_k . r2 = u_k^H r (the real split of Sec. II-D).
 *  h      [n_inst][K][M2] DEVICE: column k of H as [Re h_k; Im h_k].
 *  n0     >= 0 (0 needs H of full column rank).
 *  w      [n_inst][K][M2] DEVICE output (e.g. model.w of a detector).
 * Asynchronous on `stream`. */
int apsm_linear_mmse(const float* h, float n0, int M2, int K, int n_inst, float* w, void* stream);

/* Decision-directed tracking (Sec. II-E, remark on focusing on detection:
 * gradual channel changes are tracked by running the iteration on the data
 * symbols).  For a block of S received vectors: detect them with the frozen
 * filter (as apsm_detect), replace the soft outputs by the decided
 * constellation points, then continue the training of `model` over the
 * block's real training sequence with those decisions as the targets (as
 * apsm_train with APSM_INIT_CONTINUE: the dictionary ring continues, the
 * window starts afresh) and repack the model.
 *  params     HOST; its init field is not used (tracking always continues);
 *             needs w_lin > 0 and dict_cap == model->dict_cap.
 *  modulation APSM_MOD_QPSK or APSM_MOD_QAM16.
 *  decided    [S][K][2] DEVICE output: the decided symbols (Re, Im) the block
 *             was tracked on.
 *  hard, truth, err_count  optional, as for apsm_detect (decisions of the
 *             frozen filter, before the block's update).
 * Asynchronous on `stream`. */
int apsm_track(const apsm_params_t* params, const apsm_model_t* model, int S, const float* rx, int modulation,
               float* decided, uint8_t* hard, const uint8_t* truth, int64_t* err_count, void* stream);

/* ---- generic projection engine: ball projection and cyclic POCS ------
 * The ball B = {f : ||f_k||_H <= radius} around f = 0 in the sum space H
 * with the norm of Fact 1 (Sec. II-B),
 *     ||f_k||^2 = ||w_k||^2 / w_lin + alpha_k^T G alpha_k / w_gauss,
 * G the Gaussian Gram matrix of the dictionary entries in use (a zero
 * weight leaves its part out).  The projection onto B scales user k's
 * w_k and alpha_k by radius / ||f_k|| when ||f_k|| > radius, else leaves
 * them unchanged.  The Gaussian part of the norm is evaluated by the
 * detection kernels on the model's own dictionary vectors. */

/* Workspace bytes for apsm_project_ball and apsm_pocs with this model shape
 * (pure host function; 0 for shapes beyond this build's limits). */
size_t apsm_ball_workspace_bytes(int M2, int K, int dict_cap);

/* Projection of every user's filter onto the ball, then repacking.
 *  model      a trained model (its packed form current).
 *  sigma2, w_lin, w_gauss
 *             the kernel width and sum-space weights the model was trained
 *             with (> 0, >= 0, >= 0, weights not both 0).
 *  radius     >= 0, finite.
 *  workspace  DEVICE, 256-byte aligned, >= apsm_ball_workspace_bytes bytes.
 *  norms      [K] DEVICE output or NULL: ||f_k||_H before the projection.
 * Asynchronous on `stream`. */
int apsm_project_ball(const apsm_model_t* model, float sigma2, float w_lin, float w_gauss, float radius,
                      void* workspace, size_t ws_bytes, float* norms, void* stream);

/* Cyclic projections (POCS) of one detector: `cycles` times, the windowed
 * parallel projections over the P pilots' sets (as apsm_train: from
 * params->init in the first cycle, continued in the later ones, the
 * samples re-entering the dictionary ring with new indices and the window
 * starting afresh), then the projection onto the ball of `radius`.
 *  params     HOST, as for apsm_train (set_types allowed); cycles > 1 needs
 *             w_lin > 0.
 *  cycles     >= 1.
 *  workspace  as for apsm_project_ball.
 * Asynchronous on `stream`. */
int apsm_pocs(const apsm_params_t* params, int M2, int K, int P, const float* rx_pilot, const float* sym_pilot,
              const apsm_model_t* model, float radius, int cycles, void* workspace, size_t ws_bytes,
              void* stream);

/* ---- batches of detectors with different shapes ----------------------
 * Many independent detectors (each its own user count K, input dimension
 * M2, pilot count, dictionary capacity, sigma^2, data size and modulation)
 * trained in one launch and detected in one launch, so that a batch of small
 * problems fills the GPU and its whole train -> detect -> error-count
 * sequence can be captured once in a HIP graph and replayed.  Each detector
 * gives exactly the results that apsm_train and apsm_detect give for it
 * alone.  Use:
 *   apsm_batch_create      describe the detectors (host only),
 *   apsm_batch_workspace_bytes / apsm_batch_bind
 *                          give the batch its device tables (caller-owned
 *                          workspace, written once, synchronously),
 *   apsm_batch_tune        optional: time the launch forms on this batch and
 *                          keep the fastest (synchronous; not while capturing),
 *   apsm_batch_train, apsm_batch_detect
 *                          asynchronous launches on `stream`, no allocation,
 *                          no host synchronisation (capturable),
 *   apsm_batch_destroy.
 * The buffers named in the items must stay valid while the batch is used. */
typedef struct apsm_batch_item {
  apsm_model_t model;          /* shape (M2, K, dict_cap) and arrays of this detector   */
  float sigma2;                /* its kernel width (> 0)                                 */
  int32_t P;                   /* pilots, >= 1 (training)                               */
  const float* rx_pilot;       /* [P][M2]                                                */
  const float* sym_pilot;      /* [P][K][2]                                              */
  int32_t S;                   /* received vectors to detect, >= 0                      */
  int32_t modulation;          /* APSM_MOD_*                                             */
  const float* rx;             /* [S][M2]                                                */
  float* soft;                 /* [S][K][2] or NULL                                      */
  uint8_t* hard;               /* [S][K] or NULL (needs modulation != NONE)              */
  const uint8_t* truth;        /* [S][K] or NULL                                         */
  int64_t* err_count;          /* [K], added to; NULL iff truth is NULL                  */
} apsm_batch_item_t;

typedef struct apsm_batch apsm_batch_t;   /* opaque host object */

/* Validate and describe n >= 1 detectors.  params (HOST) gives eps, mu, w_lin,
 * w_gauss, window and pos_weights shared by all of them; its sigma2 and
 * dict_cap are not used (each item has its own).  Every item must satisfy
 * what apsm_train and apsm_detect require of the same arguments, and
 * model.dict_cap >= window.  The buffers the batch writes (every item's model
 * arrays, soft, hard and err_count) must not overlap each other, and no
 * buffer it reads (pilots, rx, truth) may overlap one it writes: such a
 * batch is rejected with APSM_ERR_INVALID_ARG.  On success *out is a new
 * batch. */
int apsm_batch_create(const apsm_params_t* params, const apsm_batch_item_t* items, int n,
                      apsm_batch_t** out);

/* Bytes of device workspace the batch needs: job tables, the work-item
 * lists of detection, claim counters and the training kernel rows (for each
 * detector with dict_cap <= 8192: 2P x (dict_cap + window) floats, the
 * Gaussian kernel values of every pilot step against the dictionary entries
 * it sees, computed by one data-parallel launch before training). */
size_t apsm_batch_workspace_bytes(const apsm_batch_t* batch);

/* Write the batch's tables into `workspace` (DEVICE, at least
 * apsm_batch_workspace_bytes, 256-byte aligned, caller-owned; it must not be
 * used for anything else while the batch is used).  Synchronous: returns
 * after the copy on `stream` has completed.  APSM_ERR_WORKSPACE if the
 * workspace is NULL, too small or misaligned. */
int apsm_batch_bind(apsm_batch_t* batch, void* workspace, size_t bytes, void* stream);

/* Autotune batched detection on this GPU and record the choices in the
 * library's tuning cache (see apsm_tune_save): (1) for every shape class in
 * the batch that both detection kernels hold (2M <= 64 and K <= 8; class =
 * 2M padded to 16/32/64 and K), time the split-FP16 kernel (coefficient sums
 * on VALU) against the two-contraction kernel (coefficient sums on the matrix
 * cores) on the class's largest detector, keep the faster for the class (this
 * batch's jobs move to that kernel's launch; later batches and apsm_detect
 * calls of the class use it too); (2) time the launch forms (persistent
 * workgroups claiming work items from a counter, or one workgroup per item)
 * and keep the faster for this shape mix.  Runs detections several times:
 * soft and hard outputs are overwritten and err_count accumulates those
 * runs, so zero err_count afterwards.  Synchronous; not while capturing. */
int apsm_batch_tune(apsm_batch_t* batch, void* stream);

/* Set the launch form of this batch's detection (overrides the tuned or
 * default choice): persistent != 0 for a grid of workgroups that claim work
 * items until none is left, sized to occupy `cus` compute units (cus <= 0:
 * all of them; fewer leave whole CUs free for kernels on other streams, such
 * as the next batch's training), 0 for one workgroup per work item.  Outputs
 * do not depend on the form.  Host only; takes effect at the next
 * apsm_batch_detect. */
int apsm_batch_set_form(apsm_batch_t* batch, int persistent, int cus);

/* Train every detector of the batch (same results as apsm_train per item)
 * and pack the models; asynchronous on `stream`.  The same as
 * apsm_batch_kernel_rows followed by apsm_batch_train_prepared on `stream`. */
int apsm_batch_train(const apsm_batch_t* batch, void* stream);

/* The two parts of apsm_batch_train, for callers that schedule them on
 * different streams.  apsm_batch_kernel_rows computes the kernel rows of the
 * batch's pilots into the workspace (one data-parallel launch over the whole
 * GPU); apsm_batch_train_prepared trains and packs from them and must be
 * ordered after that launch (same stream, or an event), with the pilots
 * unchanged in between.  Calls of one batch must not overlap. */
int apsm_batch_kernel_rows(const apsm_batch_t* batch, void* stream);
int apsm_batch_train_prepared(const apsm_batch_t* batch, void* stream);

/* Detect every item's received vectors (same results as apsm_detect per
 * item); asynchronous on `stream`.  Calls of one batch must not overlap
 * (they share the claim counters in the workspace). */
int apsm_batch_detect(const apsm_batch_t* batch, void* stream);

/* Release the host object (not the workspace).  NULL is allowed. */
void apsm_batch_destroy(apsm_batch_t* batch);

/* ---- differentiable unrolled training ---------------------------------
 * A batch of n_inst detectors of one shape trained by `passes` unrolled
 * iterations, each one full pass of the windowed projections (Sec. II-D
 * eqn:apsm, eqn:beta) over the T = 2P real training samples: pass 1 is the
 * training of apsm_train with an unbounded dictionary (dict_cap >= 2P), later
 * passes project onto the same hyperslabs again, restarting the window; then
 * the filters are evaluated on S validation symbols (Sec. III-B) and
 *     L = mean over instances, users and symbols of |g_k - b_k|^2.
 * The parameters theta (DEVICE float[3 + window]) are shared by the batch:
 *     theta[0] = sigma   (Gaussian kernel exp(-||u-v||^2 / (2 sigma^2)), > 0)
 *     theta[1] = eps     (hyperslab half-width, >= 0)
 *     theta[2] = mu      (relaxation, f <- f + mu sum_j q_j beta_j kappa(r_j, .))
 *     theta[3 + p] = omega[p] > 0, q_j = omega[n-j] / sum_{i in J_n} omega[n-i].
 * theta lives in device memory and is not checked on the host.
 * apsm_unrolled_backward gives dL/dtheta with a hand-written adjoint (reverse
 * sweep over the steps); it re-runs the forward from checkpoints taken every
 * ckpt_every passes, one segment at a time, so memory holds the checkpoints
 * and one segment's record instead of every step.  The gradient does not
 * depend on ckpt_every (bit for bit).  At |x| = eps the slab is closed and
 * the threshold's derivative is taken as 0. */
typedef struct apsm_unrolled {
  int32_t n_inst;       /* detectors, >= 1                                      */
  int32_t P;            /* pilots per detector (T = 2P), 1..2048                */
  int32_t M2;           /* 2M, even, 2..APSM_MAX_M2                             */
  int32_t K;            /* users, 1..APSM_MAX_K                                 */
  int32_t S;            /* validation symbols per detector, >= 1               */
  int32_t passes;       /* unrolled iterations, >= 1                            */
  int32_t ckpt_every;   /* checkpoint interval in passes, >= 1                  */
  int32_t window;       /* W, 1..APSM_MAX_WINDOW                                */
  float w_lin, w_gauss; /* sum-space weights (as apsm_params_t)                 */
} apsm_unrolled_t;

/* Device workspace bytes for this shape (training Gram matrix and squared
 * distances, checkpoints, one segment's record, adjoint state). */
size_t apsm_unrolled_workspace_bytes(const apsm_unrolled_t* u);

/* Forward: loss (DEVICE float[1]) = L.  Inputs, contiguous DEVICE arrays:
 *  rx_pilot [n][P][M2], sym_pilot [n][P][K][2], rx_val [n][S][M2],
 *  sym_val [n][S][K][2].  workspace: >= apsm_unrolled_workspace_bytes,
 *  256-byte aligned (else APSM_ERR_WORKSPACE); keeps what the backward call
 *  needs. */
int apsm_unrolled_forward(const apsm_unrolled_t* u, const float* theta, const float* rx_pilot,
                          const float* sym_pilot, const float* rx_val, const float* sym_val,
                          void* workspace, size_t ws_bytes, float* loss, void* stream);

/* Backward: grad (DEVICE float[3 + window]) = upstream * dL/dtheta, with
 * upstream a DEVICE float (NULL for 1).  Same arguments as the forward call
 * it follows (same theta and inputs, same workspace); may be repeated. */
int apsm_unrolled_backward(const apsm_unrolled_t* u, const float* theta, const float* rx_pilot,
                           const float* sym_pilot, const float* rx_val, const float* sym_val,
                           void* workspace, size_t ws_bytes, const float* upstream, float* grad,
                           void* stream);

/* ---- training without device allocation ------------------------------
 * For callers that cannot allocate device memory or pass a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Trains one detector exactly as apsm_batch_train trains a
 * one-item batch (the kernel rows of every pilot step, then training from
 * them, then packing: bit-identical results), with the job table and the
 * kernel rows in a static device array of the library instead of a
 * workspace.  Arguments, validation and results as for apsm_train; the
 * shape must have dict_cap <= 4096 (else APSM_ERR_UNSUPPORTED) and need at
 * most APSM_NOALLOC_SCRATCH_BYTES of scratch: about 2P * (dict_cap + window)
 * * 4 bytes (else APSM_ERR_WORKSPACE).  Allocates nothing (no hipMalloc or
 * allocating library call); asynchronous on `stream`.  Each GPU holds its
 * own copy of the array, from the first call on that GPU until the process
 * ends; every call on one GPU uses the same copy, so calls that overlap in
 * time on one GPU (different streams, or threads) race: the caller orders
 * them. */
#define APSM_NOALLOC_SCRATCH_BYTES (64u << 20)
int apsm_train_noalloc(const apsm_params_t* params, int M2, int K, int P,
                       const float* rx_pilot, const float* sym_pilot,
                       const apsm_model_t* model, void* stream);

/* Synchronous copy of model->state into host_state[4]; waits for all work on
 * the device.  Returns APSM_ERR_NONFINITE (with host_state filled) when the
 * flags word host_state[3] is nonzero, APSM_OK otherwise. */
int apsm_get_status(const apsm_model_t* model, int32_t* host_state);

/* Tuning cache: the choices of apsm_batch_tune, keyed by GPU architecture
 * name, HIP runtime version and shape class (detection kernel) or batch
 * shape mix (launch form).  apsm_tune_save writes the cache to `path` (HOST
 * string) as a JSON object of string pairs; apsm_tune_load merges such a
 * file into it (entries measured on another architecture or runtime are kept
 * but never match).  APSM_ERR_INVALID_ARG if the file cannot be written, read
 * or parsed (nothing is merged then).  Thread-safe. */
int apsm_tune_save(const char* path);
int apsm_tune_load(const char* path);

/* Release what the library keeps on the host between calls: the launch-form
 * and kernel choices cached by apsm_batch_tune (the tuning cache).  Device memory is not touched
 * (the library holds none besides its static scratch array).  Safe to call at
 * any time from one thread while no other library call runs; later calls
 * work as after loading the library. */
void apsm_shutdown(void);

/* Static description of an error code; never NULL. */
const char* apsm_strerror(int code);

/* Text of the last HIP error seen by this thread's calls ("" if none). */
const char* apsm_last_hip_error(void);

/* Library version, e.g. "0.1.0". */
const char* apsm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* APSM_H */
