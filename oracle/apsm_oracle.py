"""FP64 CPU oracle of APSM partially linear multiuser detection.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this module:
only the test suite, the smoke check and the benchmark's CPU-baseline leg use
it.  It shares no code with the HIP library; both consume the same float32
input arrays (from the seeded generator), which this module upcasts to float64.

Everything here is written as the plain definitions of the paper (Mehlhose et
al., "GPU-accelerated partially linear multiuser detection for 5G and beyond
URLLC systems", arXiv 2201.05024), step by step and in its notation:

* kernels kappa_L, kappa_G ............................ Sec. II-A
* sum space H = H_L + H_G, kappa = wL kappa_L + wG kappa_G and its
  inner product ........................................ Sec. II-B, Fact 1, eqn:sum_inner_product
* real split r1 = [Re r; Im r], r2 = [Im r; -Re r], b -> (Re b, Im b),
  g(r) = f(r1) + i f(r2), time index n = 2t + l - 1 .... Sec. II-D
* hyperslab C_n = {f : |<f, kappa(r_n, .)> - b_n| <= eps}  eqn:convex_set
* f_{n+1} = sum_{j in J_n} q_j P_{C_j}(f_n), P_{C_j}(f) = f + beta_j kappa(r_j, .)
                                                       eqn:apsm
* beta_j (three cases) ................................. eqn:beta
* J_n = {n-W+1..n} (n >= W-1), else {0..n} ............. Sec. II-D, after eqn:beta
* linear part collapsed onto 2M coefficients, Gaussian dictionary of received
  vectors ............................................. Sec. II-D, last paragraph
* detection f_n(r) = <f_n, kappa(r, .)>, model frozen .. Sec. III-B

Readings where the paper is silent (each listed in the design notes):

* step size mu: f_{n+1} = f_n + mu * sum_j q_j beta_j kappa(r_j, .); mu = 1 is
  exactly eqn:apsm because the q_j sum to one;
* f_0 = 0;
* q_j uniform 1/|J_n| over all window members, or q_j = omega_{n-j} /
  sum_{i in J_n} omega_{n-i} for per-position weights omega;
* r_n enters the Gaussian dictionary (coefficient 0) at the start of step n;
  with a dictionary cap D_cap >= W the oldest Gaussian term is evicted first
  (FIFO); its linear part stays, since it lives in the 2M linear coefficients;
* constellation: unit average energy, per-axis nearest level, a tie on a
  threshold goes to the higher level.

Parity status: every function below is pinned by the CPU tests (closed forms,
special cases reducing to set-membership NLMS and kernel interpolation, Fejer
monotonicity in the H-norm, a brute-force term-list form, hand-derived golden
values).  Absolute symbol error rates are parity unpinned relative to the
paper, which prints none.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np


# --------------------------------------------------------------------------
# Kernels and the sum space (Sec. II-A, II-B)
# --------------------------------------------------------------------------

def kappa_lin(u: np.ndarray, v: np.ndarray) -> float:
    """Linear kernel kappa_L(u, v) = u^T v (Sec. II-A)."""
    return float(np.dot(u, v))


def kappa_gauss(u: np.ndarray, v: np.ndarray, sigma2: float) -> float:
    """Gaussian kernel exp(-||u - v||^2 / (2 sigma^2)) (Sec. II-A)."""
    d = np.asarray(u, dtype=np.float64) - np.asarray(v, dtype=np.float64)
    return math.exp(-float(np.dot(d, d)) / (2.0 * sigma2))


def kappa_sum(u, v, sigma2: float, w_lin: float, w_gauss: float) -> float:
    """Reproducing kernel of the weighted sum space (Fact 1)."""
    return w_lin * kappa_lin(u, v) + w_gauss * kappa_gauss(u, v, sigma2)


def gram(points: np.ndarray, sigma2: float, w_lin: float, w_gauss: float) -> np.ndarray:
    """Gram matrix [kappa(p_i, p_j)] of the sum kernel, by the definition."""
    n = len(points)
    G = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            G[i, j] = kappa_sum(points[i], points[j], sigma2, w_lin, w_gauss)
    return G


def gauss_gram(points: np.ndarray, sigma2: float) -> np.ndarray:
    n = len(points)
    G = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            G[i, j] = kappa_gauss(points[i], points[j], sigma2)
    return G


# --------------------------------------------------------------------------
# Real split (Sec. II-D)
# --------------------------------------------------------------------------

def real_split(r: np.ndarray):
    """r in C^M -> (r1, r2) in R^{2M}: r1 = [Re r; Im r], r2 = [Im r; -Re r]."""
    r = np.asarray(r, dtype=np.complex128)
    r1 = np.concatenate([r.real, r.imag], axis=-1)
    r2 = np.concatenate([r.imag, -r.real], axis=-1)
    return r1, r2


def training_sequence(rx_pilot: np.ndarray, sym_pilot: np.ndarray):
    """Interleave pilots into the real training sequence (r_n, b_n).

    rx_pilot: [P][M] complex; sym_pilot: [P][K] complex.
    n = 2t + l - 1 with l in {1, 2}: r_{2t} = r1(t), r_{2t+1} = r2(t),
    b_{k,2t} = Re b_k(t), b_{k,2t+1} = Im b_k(t).
    Returns R [2P][2M] and B [2P][K], float64.
    """
    rx_pilot = np.asarray(rx_pilot, dtype=np.complex128)
    sym_pilot = np.asarray(sym_pilot, dtype=np.complex128)
    P, M = rx_pilot.shape
    K = sym_pilot.shape[1]
    R = np.empty((2 * P, 2 * M))
    B = np.empty((2 * P, K))
    for t in range(P):
        r1, r2 = real_split(rx_pilot[t])
        R[2 * t] = r1
        R[2 * t + 1] = r2
        B[2 * t] = sym_pilot[t].real
        B[2 * t + 1] = sym_pilot[t].imag
    return R, B


# --------------------------------------------------------------------------
# The filter: f = f_L + f_G, linear part on the Euclidean basis, Gaussian part
# on a dictionary of received vectors (Sec. II-D, last paragraph)
# --------------------------------------------------------------------------

# Distance to its set above which a member counts as violated for the
# active-set weights (a reading; see APSMParams.weight_mode).
ACTIVE_MARGIN = 1e-5


@dataclass
class APSMParams:
    sigma2: float = 0.5
    eps: float = 0.05
    mu: float = 1.0
    window: int = 16
    w_lin: float = 0.5
    w_gauss: float = 0.5
    dict_cap: Optional[int] = None          # None: the dictionary grows without bound
    pos_weights: Optional[np.ndarray] = None  # omega[0..W-1], omega[0] for j = n
    # "position": q_j from the position weights (uniform 1/|J_n| without them);
    # "violation": per user k, q_kj = d_kj / sum_{i in J_n} d_ki with d_kj =
    # max(|f_n(r_j) - b_kj| - eps, 0) the distance of f_n(r_j) to its slab
    # (0 for every member when none is violated);
    # "active": per user k, q_kj = 1 / |A_k| on the members A_k whose set
    # f_n violates by more than ACTIVE_MARGIN, 0 elsewhere (no update when
    # none is); the margin keeps a member that its own projection left on
    # the boundary out of the set, whatever the rounding
    weight_mode: str = "position"
    # Extrapolated relaxation: per user the step mu * M_n with
    # M_n = sum_j q_j ||P_j f - f||^2 / ||sum_j q_j (P_j f - f)||^2 >= 1
    # (1 where the denominator vanishes)
    extrapolate: bool = False


class Filter:
    """K real filters f_k sharing one Gaussian dictionary.

    f_k(x) = w_k^T x + sum_i alpha[i][k] kappa_G(d_i, x)
    w_k holds wL * gamma^(L) (the linear dictionary coefficients) and
    alpha[i][k] holds wG * gamma_i (the Gaussian dictionary coefficients).
    Dictionary rows are kept oldest first, each tagged with the training
    index n it came from.
    """

    def __init__(self, K: int, M2: int, sigma2: float):
        self.K = K
        self.M2 = M2
        self.sigma2 = float(sigma2)
        self.w = np.zeros((K, M2))            # f_0 = 0
        self.dict_vec = np.zeros((0, M2))
        self.alpha = np.zeros((0, K))
        self.dict_idx: List[int] = []

    def copy(self) -> "Filter":
        g = Filter(self.K, self.M2, self.sigma2)
        g.w = self.w.copy()
        g.dict_vec = self.dict_vec.copy()
        g.alpha = self.alpha.copy()
        g.dict_idx = list(self.dict_idx)
        return g

    def append(self, x: np.ndarray, n: int):
        self.dict_vec = np.vstack([self.dict_vec, np.asarray(x, dtype=np.float64)[None, :]])
        self.alpha = np.vstack([self.alpha, np.zeros((1, self.K))])
        self.dict_idx.append(n)

    def evict_oldest(self):
        self.dict_vec = self.dict_vec[1:]
        self.alpha = self.alpha[1:]
        self.dict_idx.pop(0)

    def evaluate(self, x: np.ndarray) -> np.ndarray:
        """(f_1(x), .., f_K(x)) = <f, kappa(x, .)> by the reproducing property."""
        return evaluate_many(self, np.asarray(x, dtype=np.float64)[None, :])[0]

    def slot_of(self, n: int) -> int:
        return self.dict_idx.index(n)

    def h_norm2_diff(self, other: "Filter", w_lin: float, w_gauss: float) -> np.ndarray:
        """||f_k - g_k||_H^2 per user, with Fact 1's inner product:
        ||h||^2 = ||v||^2 / wL + a^T G a / wG for h(x) = v^T x + sum_i a_i kappa_G(p_i, x)."""
        pts = np.vstack([self.dict_vec, other.dict_vec])
        coef = np.vstack([self.alpha, -other.alpha])       # [npts][K]
        dv = self.w - other.w
        lin = np.sum(dv * dv, axis=1) / w_lin
        if len(pts) == 0:
            return lin
        G = gauss_gram(pts, self.sigma2)
        gau = np.einsum("ik,ij,jk->k", coef, G, coef) / w_gauss
        return lin + gau


def soft_threshold(x: float, eps: float) -> float:
    return math.copysign(max(abs(x) - eps, 0.0), x)


def beta(e: float, b: float, eps: float, kjj: float) -> float:
    """Projection coefficient of eqn:beta, by its three cases (closed slab)."""
    if kjj == 0.0:
        return 0.0
    x = e - b
    if x < -eps:
        return (b - e - eps) / kjj
    if x > eps:
        return (b - e + eps) / kjj
    return 0.0


# Kinds of the set a training sample defines in H through the value f(r_j)
# (the generic engine: Sec. I and Sec. VI, the same machinery for other
# projection-based methods).  Each is {f : f(r_j) in [lo, hi]}, a closed
# convex set; the hyperslab of eqn:convex_set is the default.
SET_SLAB = 0        # |f(r) - b| <= eps
SET_PLANE = 1       # f(r) = b (a hyperplane; eps is not used)
SET_UPPER = 2       # f(r) <= b + eps (a halfspace)
SET_LOWER = 3       # f(r) >= b - eps (a halfspace)


def set_interval(kind: int, b: float, eps: float):
    """[lo, hi] of the values f(r_j) the set of this kind admits."""
    if kind == SET_SLAB:
        return b - eps, b + eps
    if kind == SET_PLANE:
        return b, b
    if kind == SET_UPPER:
        return -math.inf, b + eps
    if kind == SET_LOWER:
        return b - eps, math.inf
    raise ValueError(kind)


def beta_set(e: float, b: float, eps: float, kjj: float, kind: int) -> float:
    """Projection onto {f : f(r_j) in [lo, hi]}: P(f) = f + beta kappa(r_j, .)
    moves f(r_j) to the nearest point of [lo, hi], so beta = (clip(e) - e) /
    kappa(r_j, r_j) (0 when f(r_j) is already inside)."""
    if kjj == 0.0:
        return 0.0
    lo, hi = set_interval(kind, b, eps)
    return (min(max(e, lo), hi) - e) / kjj


def window(n: int, W: int) -> range:
    """J_n = {n-W+1, .., n} if n >= W-1, else {0, .., n}."""
    return range(n - W + 1, n + 1) if n >= W - 1 else range(0, n + 1)


def set_weights(n: int, J: range, p: APSMParams) -> dict:
    if p.pos_weights is None:
        return {j: 1.0 / len(J) for j in J}
    om = np.asarray(p.pos_weights, dtype=np.float64)
    tot = sum(om[n - j] for j in J)
    return {j: om[n - j] / tot for j in J}


class Trainer:
    """Windowed parallel hyperslab projections (eqn:apsm), one step at a time.

    f0: the initial filter (Sec. II-D leaves f_0 arbitrary; default f_0 = 0).
    n0: global index of the first sample of R when continuing a filter that
    has already seen n0 samples: the samples enter its dictionary as
    n0, n0 + 1, .. (FIFO eviction continues across the boundary), while the
    window J_n starts afresh inside R.
    types: optional [T][K] set kinds (SET_*) per sample and user; None gives
    the hyperslabs of eqn:convex_set with the three cases of eqn:beta."""

    def __init__(self, R: np.ndarray, B: np.ndarray, p: APSMParams,
                 f0: Optional[Filter] = None, n0: int = 0, types: Optional[np.ndarray] = None):
        self.R = np.asarray(R, dtype=np.float64)
        self.B = np.asarray(B, dtype=np.float64)
        self.types = None if types is None else np.asarray(types, dtype=np.int64)
        self.p = p
        if p.dict_cap is not None and p.dict_cap < p.window:
            raise ValueError("dictionary cap must be at least the window size")
        if p.weight_mode not in ("position", "violation", "active"):
            raise ValueError(p.weight_mode)
        T, M2 = self.R.shape
        K = self.B.shape[1]
        self.f = f0.copy() if f0 is not None else Filter(K, M2, p.sigma2)
        self.n = 0
        self.n0 = n0

    def step(self):
        """One step n: returns (J_n, e, beta) for inspection."""
        p, f, n = self.p, self.f, self.n
        r_n = self.R[n]
        # r_n joins the Gaussian dictionary with coefficient 0; with a cap,
        # the oldest Gaussian term leaves first.
        if p.dict_cap is not None and len(f.dict_vec) == p.dict_cap:
            f.evict_oldest()
        f.append(r_n, self.n0 + n)

        J = window(n, p.window)
        q = set_weights(n, J, p)
        # All W projections act on the same f_n (eqn:apsm), so every
        # prediction and every beta is taken before any coefficient changes.
        E = evaluate_many(f, self.R[list(J)])
        e = {j: E[i] for i, j in enumerate(J)}
        bet = {}
        for j in J:
            kjj = kappa_sum(self.R[j], self.R[j], p.sigma2, p.w_lin, p.w_gauss)
            if self.types is None:
                bet[j] = np.array([beta(e[j][k], self.B[j, k], p.eps, kjj) for k in range(f.K)])
            else:
                bet[j] = np.array([beta_set(e[j][k], self.B[j, k], p.eps, kjj, self.types[j, k])
                                   for k in range(f.K)])
        if p.weight_mode in ("violation", "active"):
            # q_kj proportional to the distance of f_n(r_j) to set C_kj, or
            # uniform over the violated sets (the paper leaves the weights
            # free to prioritise sets adaptively)
            if self.types is None:
                dist = {j: np.maximum(np.abs(e[j] - self.B[j]) - p.eps, 0.0) for j in J}
            else:
                dist = {}
                for j in J:
                    iv = [set_interval(self.types[j, k], self.B[j, k], p.eps) for k in range(f.K)]
                    dist[j] = np.array([abs(min(max(e[j][k], lo), hi) - e[j][k]) for k, (lo, hi) in enumerate(iv)])
            if p.weight_mode == "active":
                dist = {j: (dist[j] > ACTIVE_MARGIN).astype(np.float64) for j in J}
            tot = sum(dist.values())
            qk = {j: np.divide(dist[j], tot, out=np.zeros(f.K), where=tot > 0) for j in J}
        else:
            qk = {j: np.full(f.K, q[j]) for j in J}
        M = np.ones(f.K)
        if p.extrapolate:
            # P_j f - f = beta_j kappa(r_j, .), of squared norm beta_j^2
            # kappa(r_j, r_j); the norm of the combination through the Gram
            # matrix of the members
            Jl = list(J)
            Gm = gram(self.R[Jl], p.sigma2, p.w_lin, p.w_gauss)
            Q = np.array([qk[j] for j in Jl])                   # [L][K]
            Bt = np.array([bet[j] for j in Jl])
            num = np.einsum("jk,jk,j->k", Q, Bt * Bt, np.diag(Gm))
            den = np.einsum("jk,jl,lk->k", Q * Bt, Gm, Q * Bt)
            M = np.where(den > 0.0, num / np.where(den > 0.0, den, 1.0), 1.0)
        for j in J:
            c = p.mu * M * qk[j] * bet[j]                  # [K]
            # P_{C_j} adds beta_j (wL kappa_L(r_j, .) + wG kappa_G(r_j, .)).
            f.w += np.outer(c * p.w_lin, self.R[j])
            f.alpha[f.slot_of(self.n0 + j)] += c * p.w_gauss
        self.n += 1
        return J, e, bet


def train(R: np.ndarray, B: np.ndarray, p: APSMParams,
          on_step: Optional[Callable] = None) -> Filter:
    tr = Trainer(R, B, p)
    for _ in range(len(R)):
        out = tr.step()
        if on_step is not None:
            on_step(tr, out)
    return tr.f


def sample_types(set_types_pairs: np.ndarray) -> np.ndarray:
    """[P][K][2] set kinds (real part, imaginary part of each pilot symbol) ->
    [T][K] in the order of the training sequence (n = 2t + l - 1)."""
    st = np.asarray(set_types_pairs)
    P, K, _ = st.shape
    out = np.empty((2 * P, K), dtype=np.int64)
    out[0::2] = st[..., 0]
    out[1::2] = st[..., 1]
    return out


def train_from_pilots(rx_pilot_planar: np.ndarray, sym_pilot_pairs: np.ndarray,
                      p: APSMParams, f0: Optional[Filter] = None, n0: int = 0,
                      set_types: Optional[np.ndarray] = None) -> Filter:
    """Planar float arrays as stored for the library -> Filter: training from
    f0 (default f_0 = 0) whose dictionary has seen n0 samples before;
    set_types [P][K][2] (SET_*) or None for hyperslabs."""
    rx = _planar_to_complex(rx_pilot_planar)
    sym = np.asarray(sym_pilot_pairs, dtype=np.float64)
    sym = sym[..., 0] + 1j * sym[..., 1]
    R, B = training_sequence(rx, sym)
    tr = Trainer(R, B, p, f0=f0, n0=n0, types=None if set_types is None else sample_types(set_types))
    for _ in range(len(R)):
        tr.step()
    return tr.f


# --------------------------------------------------------------------------
# Initialisation by a conventional linear filter when channel information is
# available (Sec. I; Sec. II-D: f_0 in eqn:apsm is arbitrary, and may be a
# linear filter of H_L).  The linear filter is the textbook MMSE receiver
# (a reading: the paper names no particular one).
# --------------------------------------------------------------------------

def linear_mmse(H: np.ndarray, n0: float) -> np.ndarray:
    """Linear MMSE receive filters for the model r = H x + n of Sec. II-C with
    unit-power symbols and noise CN(0, n0 I): U = H (H^H H + n0 I)^{-1}, user
    k's estimate u_k^H r (column k of U)."""
    H = np.asarray(H, dtype=np.complex128)
    K = H.shape[1]
    G = H.conj().T @ H + n0 * np.eye(K)
    return H @ np.linalg.inv(G)


def filter_from_linear(U: np.ndarray, sigma2: float) -> Filter:
    """The filter whose detection g_k(r) = f_k(r1) + i f_k(r2) equals u_k^H r:
    f_k(x) = w_k^T x with w_k = [Re u_k; Im u_k] (real split of Sec. II-D), an
    empty Gaussian dictionary."""
    U = np.asarray(U, dtype=np.complex128)
    M, K = U.shape
    f = Filter(K, 2 * M, sigma2)
    f.w = np.concatenate([U.real.T, U.imag.T], axis=1)
    return f


# --------------------------------------------------------------------------
# Decision-directed tracking (Sec. II-E: the filter keeps adapting on the
# detected data symbols)
# --------------------------------------------------------------------------

def decided_symbols(soft: np.ndarray, modulation: str) -> np.ndarray:
    """soft [..., 2] -> the decided constellation points, complex."""
    lv = axis_levels(modulation)
    return lv[slice_axis(soft[..., 0], modulation)] + 1j * lv[slice_axis(soft[..., 1], modulation)]


def decision_directed(f: Filter, rx_planar: np.ndarray, modulation: str, p: APSMParams,
                      n0: int) -> tuple:
    """One block of tracking: detect the block with the frozen filter f
    (Sec. III-B), take the slicer's decisions as the targets b, and continue
    the iteration over the block's real training sequence (its samples enter
    the dictionary as n0, n0 + 1, ..; the window starts afresh).  Returns
    (the updated filter, the soft outputs the decisions came from)."""
    soft = detect_planar(f, rx_planar)
    bhat = decided_symbols(soft, modulation)
    R, B = training_sequence(_planar_to_complex(rx_planar), bhat)
    tr = Trainer(R, B, p, f0=f, n0=n0)
    for _ in range(len(R)):
        tr.step()
    return tr.f, soft


def _planar_to_complex(x):
    x = np.asarray(x, dtype=np.float64)
    M = x.shape[-1] // 2
    return x[..., :M] + 1j * x[..., M:]


# --------------------------------------------------------------------------
# Detection (Sec. III-B): f is frozen; g(r) = f(r1) + i f(r2)
# --------------------------------------------------------------------------

def evaluate_many(f: Filter, X: np.ndarray, chunk: int = 256) -> np.ndarray:
    """f_k(x) for every row of X [n][2M]; the Gaussian sum is taken over the
    explicit differences x - d_i, chunked over samples to bound memory."""
    X = np.asarray(X, dtype=np.float64)
    out = X @ f.w.T
    if len(f.dict_vec) == 0:
        return out
    Dm = f.dict_vec                                 # [D][2M]
    A = f.alpha                                     # [D][K]
    for s in range(0, len(X), chunk):
        diff = X[s:s + chunk, None, :] - Dm[None, :, :]
        kg = np.exp(-np.sum(diff * diff, axis=2) / (2.0 * f.sigma2))
        out[s:s + chunk] += kg @ A
    return out


def detect(f: Filter, rx: np.ndarray, chunk: int = 256) -> np.ndarray:
    """rx: [S][M] complex -> g [S][K] complex."""
    r1, r2 = real_split(rx)
    return evaluate_many(f, r1, chunk) + 1j * evaluate_many(f, r2, chunk)


def detect_planar(f: Filter, rx_planar: np.ndarray, chunk: int = 256) -> np.ndarray:
    """Planar float rows [S][2M] -> soft outputs [S][K][2] (Re g, Im g)."""
    g = detect(f, _planar_to_complex(rx_planar), chunk)
    return np.stack([g.real, g.imag], axis=-1)


# --------------------------------------------------------------------------
# Decisions and symbol error rate
# --------------------------------------------------------------------------

def axis_levels(modulation: str) -> np.ndarray:
    if modulation == "qpsk":
        return np.array([-1.0, 1.0]) / math.sqrt(2.0)
    if modulation == "qam16":
        return np.array([-3.0, -1.0, 1.0, 3.0]) / math.sqrt(10.0)
    raise ValueError(modulation)


def axis_thresholds(modulation: str) -> np.ndarray:
    lv = axis_levels(modulation)
    return (lv[1:] + lv[:-1]) / 2.0


def slice_axis(x: np.ndarray, modulation: str) -> np.ndarray:
    """Nearest level index per axis; exactly on a threshold -> the higher level."""
    th = axis_thresholds(modulation)
    x = np.asarray(x, dtype=np.float64)
    idx = np.zeros(x.shape, dtype=np.int64)
    for t in th:
        idx += (x >= t)
    return idx


def _gray(i):
    return i ^ (i >> 1)


def decide(soft: np.ndarray, modulation: str) -> np.ndarray:
    """soft [..., 2] (Re, Im) -> uint8 labels (gray(i_re) << b) | gray(i_im)."""
    bits = {"qpsk": 1, "qam16": 2}[modulation]
    ire = slice_axis(soft[..., 0], modulation)
    iim = slice_axis(soft[..., 1], modulation)
    return ((_gray(ire) << bits) | _gray(iim)).astype(np.uint8)


def symbol_errors(labels: np.ndarray, truth: np.ndarray) -> np.ndarray:
    """Per-user count of decided labels that differ from the transmitted ones."""
    return np.sum(np.asarray(labels) != np.asarray(truth), axis=0).astype(np.int64)


def boundary_distance(soft: np.ndarray, modulation: str) -> np.ndarray:
    """Distance of each (Re, Im) soft value to the nearest decision threshold,
    min over the two axes: [..., 2] -> [...]."""
    th = axis_thresholds(modulation)
    d = np.min(np.abs(soft[..., None] - th), axis=-1)
    return np.min(d, axis=-1)


# --------------------------------------------------------------------------
# Brute-force term-list form (tiny inputs only)
# --------------------------------------------------------------------------

class TermListTrainer:
    """The same iteration with nothing merged: every projection is kept as its
    own term (sample index j, coefficient c) of c * kappa(r_j, .).  Evaluation
    sums wL r_j^T x over all terms and wG kappa_G(r_j, x) over the terms whose
    sample is still in the Gaussian dictionary (the last D_cap samples)."""

    def __init__(self, R, B, p: APSMParams):
        self.R = np.asarray(R, dtype=np.float64)
        self.B = np.asarray(B, dtype=np.float64)
        self.p = p
        self.K = self.B.shape[1]
        self.terms = []            # (j, c[K])
        self.n = 0

    def _in_dict(self, j: int) -> bool:
        cap = self.p.dict_cap
        return cap is None or j > self.n - 1 - cap

    def evaluate(self, x):
        p = self.p
        out = np.zeros(self.K)
        for j, c in self.terms:
            v = p.w_lin * float(np.dot(self.R[j], x))
            if self._in_dict(j):
                v += p.w_gauss * kappa_gauss(self.R[j], x, p.sigma2)
            out += c * v
        return out

    def step(self):
        p, n = self.p, self.n
        self.n += 1              # r_n is now in the dictionary (and the oldest may be out)
        J = window(n, p.window)
        q = set_weights(n, J, p)
        new = []
        for j in J:
            e = self.evaluate(self.R[j])
            kjj = p.w_lin * float(np.dot(self.R[j], self.R[j])) + p.w_gauss
            bet = np.array([beta(e[k], self.B[j, k], p.eps, kjj) for k in range(self.K)])
            new.append((j, p.mu * q[j] * bet))
        self.terms.extend(new)
