"""Pins of the FP64 unrolled-APSM reference (oracle/unrolled.py) against
things other than itself: the step-by-step trainer of the oracle (pass 1, and
pass 2 as a second training run started from the first), central finite
differences of the forward (the definition of the derivative), and the
invariances the parameterisation fixes."""
import numpy as np
import pytest

import oracle as O
import synth
from oracle import unrolled as U

torch = pytest.importorskip("torch")


def small_instances(n=2, K=2, M=2, P=6, S=5, seed=77):
    out = []
    for i in range(n):
        inst = synth.make_instance(synth.InstanceSpec(K=K, M=M, P=P, S=S, snr_db=8.0, seed=seed + i))
        out.append((inst.rx_pilot, inst.sym_pilot, inst.rx_data, inst.sym_data))
    return out


THETA = [0.7, 0.05, 0.9, 1.0, 0.8, 0.6, 0.5]     # sigma, eps, mu, omega[0..3]


def test_pass_one_is_the_trainer():
    rxp, symp, _, _ = small_instances(1, K=3, M=4, P=20)[0]
    th = [0.6, 0.05, 1.2, 1.0, 0.5, 0.25]
    w, a = U.final_state(th, rxp, symp, passes=1)
    p = O.APSMParams(sigma2=0.36, eps=0.05, mu=1.2, window=3, pos_weights=np.array(th[3:]))
    f = O.train_from_pilots(rxp, symp, p)
    np.testing.assert_allclose(w, f.w, rtol=0, atol=1e-12)
    assert f.dict_idx == list(range(40))
    np.testing.assert_allclose(a, f.alpha, rtol=0, atol=1e-12)


def test_pass_two_is_a_second_training_run_from_pass_one():
    """A second pass projects onto the same hyperslabs starting from the
    first pass's filter; the trainer started from that filter (it re-appends
    each sample with coefficient 0, which leaves every function value as it
    is) gives the same filter function."""
    rxp, symp, rxv, _ = small_instances(1, K=2, M=3, P=15)[0]
    th = [0.8, 0.02, 1.0, 1.0, 1.0, 1.0, 1.0]
    w2, a2 = U.final_state(th, rxp, symp, passes=2)
    p = O.APSMParams(sigma2=0.64, eps=0.02, mu=1.0, window=4)
    f1 = O.train_from_pilots(rxp, symp, p)
    R, B = U.real_training(rxp, symp)
    f2 = O.Trainer(R, B, p, f0=f1)
    for _ in range(len(R)):
        f2.step()
    np.testing.assert_allclose(w2, f2.f.w, rtol=0, atol=1e-12)
    Rv, _ = U.real_validation(rxv, np.zeros((rxv.shape[0], 2, 2)))
    g = O.Filter(2, R.shape[1], 0.64)
    g.w, g.dict_vec, g.alpha, g.dict_idx = w2, R, a2, list(range(len(R)))
    np.testing.assert_allclose(O.evaluate_many(g, Rv), O.evaluate_many(f2.f, Rv), rtol=0, atol=1e-12)


def fd_grad(theta, inst, passes, h=1e-6):
    g = np.zeros(len(theta))
    for i in range(len(theta)):
        tp, tm = list(theta), list(theta)
        tp[i] += h
        tm[i] -= h
        g[i] = (U.loss_only(tp, inst, passes) - U.loss_only(tm, inst, passes)) / (2 * h)
    return g


@pytest.mark.parametrize("passes", [1, 3])
def test_gradient_equals_central_differences(passes):
    inst = small_instances()
    L, g = U.loss_and_grad(THETA, inst, passes)
    assert np.isfinite(L) and L > 0
    g_fd = fd_grad(THETA, inst, passes)
    scale = np.abs(g).max()
    np.testing.assert_allclose(g, g_fd, rtol=0, atol=1e-6 * scale)
    # every parameter matters here (none of the derivatives is trivially zero)
    assert np.all(np.abs(g) > 1e-6 * scale)


def test_loss_depends_on_omega_only_through_its_direction():
    """q_j is invariant to scaling omega, so L(c omega) = L(omega) and the
    omega-gradient is orthogonal to omega (Euler's relation for degree 0)."""
    inst = small_instances()
    L, g = U.loss_and_grad(THETA, inst, 2)
    th2 = THETA[:3] + [3.0 * x for x in THETA[3:]]
    assert abs(U.loss_only(th2, inst, 2) - L) <= 1e-13 * L
    om = np.array(THETA[3:])
    assert abs(om @ g[3:]) <= 1e-10 * np.linalg.norm(om) * np.linalg.norm(g[3:])


def test_linear_only_filter_does_not_depend_on_sigma():
    inst = small_instances()
    th = torch.tensor(THETA, dtype=torch.float64, requires_grad=True)
    R, B = U.real_training(inst[0][0], inst[0][1])
    Rv, Bv = U.real_validation(inst[0][2], inst[0][3])
    R, B, Rv, Bv = (torch.from_numpy(a) for a in (R, B, Rv, Bv))
    L = U.unrolled_sq_error(th, R, B, Rv, Bv, 2, w_lin=1.0, w_gauss=0.0)
    L.backward()
    assert th.grad[0].item() == 0.0
    assert th.grad[2].item() != 0.0


def test_mu_derivative_of_one_projection():
    """One sample pair (T = 2), W = 1, one pass, eps = 0: step 0 projects f_0 = 0
    onto the slab of r_0; step 1 projects onto the slab of r_1 = r2(0), which
    is orthogonal to r_0 (so only the Gaussian part links the two steps).
    Closed form of L(mu) on a validation vector, differentiated by hand."""
    rng = np.random.default_rng(3)
    x = rng.normal(size=4)                         # complex pilot, M = 2, planar
    b = np.array([[0.6, -0.4]])                    # K = 1
    v = rng.normal(size=4)                         # validation vector, planar
    bv = np.array([[0.3, 0.2]])
    sigma, mu, wl, wg = 0.9, 0.7, 0.5, 0.5
    inst = [(x[None, :], b[None, :, :], v[None, :], bv[None, :, :])]
    L, g = U.loss_and_grad([sigma, 0.0, mu, 1.0], inst, 1, w_lin=wl, w_gauss=wg)
    # by hand
    R, _ = U.real_training(x[None, :], b[None, :, :])
    r0, r1 = R
    kG = lambda u, w_: np.exp(-np.sum((u - w_) ** 2) / (2 * sigma ** 2))  # noqa: E731
    k = lambda u, w_: wl * u @ w_ + wg * kG(u, w_)                         # noqa: E731
    b0, b1 = b[0, 0], b[0, 1]
    c0 = mu * b0 / k(r0, r0)                      # beta_0 = (b_0 - 0) / kappa_00
    e1 = c0 * k(r0, r1)
    c1 = mu * (b1 - e1) / k(r1, r1)
    Rv, _ = U.real_validation(v[None, :], bv[None, :, :])
    f = [c0 * k(r0, u) + c1 * k(r1, u) for u in Rv]
    dc0 = b0 / k(r0, r0)
    de1 = dc0 * k(r0, r1)
    dc1 = (b1 - e1) / k(r1, r1) - mu * de1 / k(r1, r1)
    df = [dc0 * k(r0, u) + dc1 * k(r1, u) for u in Rv]
    L_hand = ((f[0] - bv[0, 0]) ** 2 + (f[1] - bv[0, 1]) ** 2) / 1
    dL_hand = 2 * (f[0] - bv[0, 0]) * df[0] + 2 * (f[1] - bv[0, 1]) * df[1]
    assert abs(L - L_hand) <= 1e-12 * L_hand
    assert abs(g[2] - dL_hand) <= 1e-10 * abs(dL_hand)
