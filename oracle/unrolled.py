"""FP64 reference of unrolled APSM training and of its gradient.

TEST INFRASTRUCTURE ONLY (like the rest of this package): used by the test
suite, never by the library or its binding.  Shares no code with the HIP
path.

What is computed (the differentiable form of the detector):

* Forward.  An "iteration" is one full pass of the windowed parallel hyperslab
  projections (Sec. II-D, eqn:apsm with the coefficients of eqn:beta) over the
  T = 2P real training samples r_0..r_{T-1} with targets b_{k,n} (real split
  of Sec. II-D).  Pass 1 is exactly the training of Sec. II-D with an
  unbounded dictionary: r_n enters the Gaussian dictionary at the start of
  step n with coefficient 0.  Later passes project again onto the same
  hyperslabs C_n; all their samples are in the dictionary already, so only
  coefficients change.  The window J_n = {n-W+1..n} (or {0..n}) restarts with
  every pass.  Each step uses q_j = omega_{n-j} / sum_{i in J_n} omega_{n-i}
  and the relaxation mu: f <- f + mu sum_j q_j beta_j kappa(r_j, .).
  After the passes the frozen filters are evaluated on validation vectors
  (Sec. III-B, g = f(r1) + i f(r2)) and the loss is
      L = mean over instances, users and validation symbols of |g_k - b_k|^2.
* Parameters theta = (sigma, eps, mu, omega_0..omega_{W-1}); the Gaussian
  kernel is exp(-||u - v||^2 / (2 sigma^2)) (Sec. II-A).
* Gradient: reverse-mode automatic differentiation (torch.autograd, float64)
  of the forward exactly as written below, step by step.  At |x| = eps the
  slab is closed (beta = 0) and the derivative of the threshold is taken as 0.

Coefficients are held for every training sample from the start, zero until
the sample's own step in pass 1; an entry with zero coefficient adds nothing
to any evaluation, so this is the growing dictionary of Sec. II-D.

Pins (tests/test_unrolled_oracle.py): pass 1 equals the step-by-step trainer
of apsm_oracle; the gradient equals central finite differences of the
forward; the loss is invariant to scaling omega (so its omega-gradient is
orthogonal to omega); a one-step case against its closed-form derivative.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np
import torch

from .apsm_oracle import training_sequence, window


def real_validation(rx_val_planar: np.ndarray, sym_val_pairs: np.ndarray):
    """Validation symbols in the planar storage -> real vectors and targets,
    r1(t) then r2(t) for each t (Sec. II-D real split): Rv [2S][2M], Bv [2S][K]."""
    x = np.asarray(rx_val_planar, dtype=np.float64)
    M = x.shape[-1] // 2
    rx = x[..., :M] + 1j * x[..., M:]
    sym = np.asarray(sym_val_pairs, dtype=np.float64)
    sym = sym[..., 0] + 1j * sym[..., 1]
    Rv, Bv = training_sequence(rx, sym)
    return Rv, Bv


def real_training(rx_pilot_planar: np.ndarray, sym_pilot_pairs: np.ndarray):
    return real_validation(rx_pilot_planar, sym_pilot_pairs)


def _sqdist(X, Y):
    """||x_a - y_b||^2 for all pairs, written out as a difference (no norm trick)."""
    d = X[:, None, :] - Y[None, :, :]
    return (d * d).sum(-1)


def unrolled_state(theta, R, B, passes: int, w_lin: float, w_gauss: float):
    """Run the passes.  theta: float64 tensor [3 + W]; R [T][M2], B [T][K]
    (torch float64).  Returns (w [K][M2], alpha [T][K])."""
    sigma, eps, mu, om = theta[0], theta[1], theta[2], theta[3:]
    W = om.shape[0]
    T, M2 = R.shape
    K = B.shape[1]
    G = torch.exp(-_sqdist(R, R) / (2.0 * sigma * sigma))
    kjj = w_lin * (R * R).sum(1) + w_gauss          # kappa(r_j, r_j), kappa_G(r, r) = 1
    w = torch.zeros(K, M2, dtype=torch.float64)
    alpha = torch.zeros(T, K, dtype=torch.float64)
    for _ in range(passes):
        for n in range(T):
            J = list(window(n, W))
            Jt = torch.tensor(J)
            # predictions f_n(r_j) of every window member, all from the same f_n
            e = R[Jt] @ w.T + G[Jt] @ alpha
            x = e - B[Jt]
            beta = -torch.sign(x) * torch.relu(x.abs() - eps) / kjj[Jt, None]
            om_J = om[torch.tensor([n - j for j in J])]
            q = om_J / om_J.sum()
            c = mu * q[:, None] * beta                 # [|J|][K]
            w = w + w_lin * (c.T @ R[Jt])
            alpha = alpha.index_add(0, Jt, w_gauss * c)
    return w, alpha


def unrolled_sq_error(theta, R, B, Rv, Bv, passes: int, w_lin: float, w_gauss: float):
    """Sum over the validation vectors and users of (f_k(r) - b_k)^2 for one
    instance (its two real vectors per symbol give |g_k - b_k|^2)."""
    w, alpha = unrolled_state(theta, R, B, passes, w_lin, w_gauss)
    sigma = theta[0]
    Gv = torch.exp(-_sqdist(Rv, R) / (2.0 * sigma * sigma))
    f = Rv @ w.T + Gv @ alpha
    return ((f - Bv) ** 2).sum()


def loss_and_grad(theta: Sequence[float], instances, passes: int, w_lin: float = 0.5,
                  w_gauss: float = 0.5):
    """instances: list of (rx_pilot_planar, sym_pilot_pairs, rx_val_planar,
    sym_val_pairs) float arrays as stored for the library.  Returns
    (L, dL/dtheta) in float64, L the mean over instances, users and
    validation symbols of |g - b|^2."""
    th = torch.tensor(np.asarray(theta, dtype=np.float64), requires_grad=True)
    total = torch.zeros((), dtype=torch.float64)
    count = 0
    for rxp, symp, rxv, symv in instances:
        R, B = real_training(rxp, symp)
        Rv, Bv = real_validation(rxv, symv)
        R, B, Rv, Bv = (torch.from_numpy(a) for a in (R, B, Rv, Bv))
        total = total + unrolled_sq_error(th, R, B, Rv, Bv, passes, w_lin, w_gauss)
        count += Bv.shape[0] // 2 * Bv.shape[1]
    L = total / count
    L.backward()
    return float(L.detach()), th.grad.detach().numpy().copy()


def loss_only(theta: Sequence[float], instances, passes: int, w_lin: float = 0.5, w_gauss: float = 0.5):
    with torch.no_grad():
        th = torch.tensor(np.asarray(theta, dtype=np.float64))
        total, count = 0.0, 0
        for rxp, symp, rxv, symv in instances:
            R, B = real_training(rxp, symp)
            Rv, Bv = real_validation(rxv, symv)
            R, B, Rv, Bv = (torch.from_numpy(a) for a in (R, B, Rv, Bv))
            total += float(unrolled_sq_error(th, R, B, Rv, Bv, passes, w_lin, w_gauss))
            count += Bv.shape[0] // 2 * Bv.shape[1]
    return total / count


def final_state(theta: Sequence[float], rx_pilot_planar, sym_pilot_pairs, passes: int,
                w_lin: float = 0.5, w_gauss: float = 0.5):
    """(w, alpha) after the passes, float64 numpy (alpha row n = sample n)."""
    with torch.no_grad():
        th = torch.tensor(np.asarray(theta, dtype=np.float64))
        R, B = real_training(rx_pilot_planar, sym_pilot_pairs)
        w, a = unrolled_state(th, torch.from_numpy(R), torch.from_numpy(B), passes, w_lin, w_gauss)
    return w.numpy(), a.numpy()
