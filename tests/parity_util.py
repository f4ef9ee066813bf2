"""Helpers shared by the GPU parity tests: seeded inputs, oracle runs and the
comparison rules.

Tolerance (float32 kernels against the FP64 oracle):
  |f_gpu - f_ref| <= 1e-4 * max(|f_ref|, a_min) per soft output, with a_min
  the smallest per-axis constellation amplitude (1/sqrt2 for QPSK, 1/sqrt10
  for 16-QAM), so values near zero are judged on the constellation's scale.
Decisions: identical labels for every sample whose oracle soft value is at
least 1e-5 away from every decision threshold; mismatches inside that band
are allowed (the two sides round differently) and are reported.
"""
import math

import numpy as np

import oracle as O

REL_TOL = 1e-4
BAND = 1e-5
A_MIN = {"qpsk": 1 / math.sqrt(2), "qam16": 1 / math.sqrt(10)}


def oracle_params(p):
    """paper_2201_05024_amd.Params -> oracle.APSMParams."""
    return O.APSMParams(sigma2=p.sigma2, eps=p.eps, mu=p.mu, window=p.window, w_lin=p.w_lin,
                        w_gauss=p.w_gauss, dict_cap=p.dict_cap,
                        pos_weights=None if p.pos_weights is None else np.asarray(p.pos_weights))


def oracle_model_to_ring(f, cap):
    """Place an oracle Filter's dictionary into the library's ring (sample n
    in slot n % cap) as float64 arrays, d [cap][M2] (the library stores its
    transpose, component-major) and alpha [cap][K]."""
    M2, K = f.M2, f.K
    d = np.zeros((cap, M2))
    a = np.zeros((cap, K))
    for n, vec, al in zip(f.dict_idx, f.dict_vec, f.alpha):
        d[n % cap] = vec
        a[n % cap] = al
    return d, a


def ring_to_oracle_model(dict_, alpha, w, sigma2, size):
    """Library ring arrays (dict_ as [cap][M2], i.e. the transpose of the
    library's component-major array) -> oracle Filter (slot order; the sum is
    order-free)."""
    f = O.Filter(w.shape[0], w.shape[1], sigma2)
    f.w = np.asarray(w, dtype=np.float64)
    f.dict_vec = np.asarray(dict_[:size], dtype=np.float64)
    f.alpha = np.asarray(alpha[:size], dtype=np.float64)
    f.dict_idx = list(range(size))
    return f


def rounded(f):
    """The oracle model rounded to float32 (and back), for detection-only parity."""
    g = f.copy()
    g.w = g.w.astype(np.float32).astype(np.float64)
    g.dict_vec = g.dict_vec.astype(np.float32).astype(np.float64)
    g.alpha = g.alpha.astype(np.float32).astype(np.float64)
    return g


def compare_soft(soft_gpu, soft_ref, modulation):
    """Returns (max scaled error, fraction of outputs within tolerance)."""
    soft_gpu = np.asarray(soft_gpu, dtype=np.float64)
    scale = np.maximum(np.abs(soft_ref), A_MIN[modulation])
    err = np.abs(soft_gpu - soft_ref) / scale
    return float(err.max()) if err.size else 0.0, err


def compare_hard(hard_gpu, soft_ref, modulation):
    """Returns (mismatches outside the band, mismatches inside the band)."""
    ref_lab = O.decide(soft_ref, modulation)
    near = O.boundary_distance(soft_ref, modulation) < BAND
    diff = np.asarray(hard_gpu) != ref_lab
    return int(np.sum(diff & ~near)), int(np.sum(diff & near))
