"""FP64 oracle of the generic projection engine: projections in the sum RKHS
H = H_L + H_G beyond the hyperslabs of the detector.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper presents its GPU design as applicable to other projection-based
methods in RKHSs (Sec. I, Sec. VI).  The sets here, each a closed convex set
of H, with their projections:

* per training sample, {f : f(r_j) in [lo, hi]}: hyperslab, hyperplane and
  the two halfspaces (apsm_oracle.SET_*, trained by Trainer with `types`);
* the ball B = {f : ||f||_H <= rho} around f = 0, whose projection scales f
  by rho / ||f||_H when f lies outside, with the norm of Fact 1:
  ||f||^2 = ||w||^2 / wL + alpha^T G alpha / wG for f(x) = w^T x +
  sum_i alpha_i kappa_G(d_i, x) (G the Gaussian Gram matrix of the
  dictionary; a zero weight leaves its part out, its coefficients being 0);
* cyclic projections (POCS): each cycle continues the windowed parallel
  projections over the sample block, then projects onto the ball.

Parity status: pinned by tests/test_oracle_engine.py (the norm against the
quadratic form of the unmerged term list, the ball's defining properties,
interval projections landing on their boundaries, Fejer monotonicity of the
cycles for a point inside every set).
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from .apsm_oracle import APSMParams, Filter, gauss_gram, train_from_pilots


def h_norm(f: Filter, w_lin: float, w_gauss: float) -> np.ndarray:
    """||f_k||_H per user (Fact 1's inner product)."""
    lin = np.sum(f.w * f.w, axis=1) / w_lin if w_lin > 0 else np.zeros(f.K)
    if w_gauss > 0 and len(f.dict_vec):
        G = gauss_gram(f.dict_vec, f.sigma2)
        gau = np.einsum("ik,ij,jk->k", f.alpha, G, f.alpha) / w_gauss
    else:
        gau = np.zeros(f.K)
    return np.sqrt(lin + gau)


def project_ball(f: Filter, radius: float, w_lin: float, w_gauss: float) -> Filter:
    """P_B(f) per user: f_k unchanged if ||f_k|| <= rho, else rho f_k / ||f_k||."""
    nrm = h_norm(f, w_lin, w_gauss)
    scale = np.where(nrm > radius, radius / np.where(nrm > 0, nrm, 1.0), 1.0)
    g = f.copy()
    g.w = g.w * scale[:, None]
    g.alpha = g.alpha * scale[None, :]
    return g


def pocs(rx_pilot_planar: np.ndarray, sym_pilot_pairs: np.ndarray, p: APSMParams, radius: float,
         cycles: int, f0: Optional[Filter] = None, n0: int = 0,
         set_types: Optional[np.ndarray] = None) -> Filter:
    """`cycles` times: the windowed parallel projections over the block (its
    samples entering the dictionary with global indices n0, n0 + T, .. and a
    fresh window each cycle), then the projection onto the ball."""
    f = f0
    n = n0
    T = 2 * np.asarray(rx_pilot_planar).shape[0]
    for _ in range(cycles):
        f = train_from_pilots(rx_pilot_planar, sym_pilot_pairs, p, f0=f, n0=n, set_types=set_types)
        n += T
        f = project_ball(f, radius, p.w_lin, p.w_gauss)
    return f
