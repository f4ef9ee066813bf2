"""Pins of the oracle's extensions of the iteration: initialisation by a
conventional linear filter (Sec. I; f_0 of eqn:apsm is arbitrary, Sec. II-D),
continuing a trained filter on further samples and decision-directed tracking
on detected data (Sec. II-E, remark on focusing on detection), and adaptive
set weights proportional to the slab violation (Sec. II-D, the weights q_j
may prioritise the sets adaptively).  As in test_oracle_pins.py, each check
is a consequence that a plausible mistake would break, not the formula
retyped."""
import math

import numpy as np
import pytest

import oracle as O


def _cplx(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def _qpsk(rng, *shape):
    return (rng.choice([-1.0, 1.0], shape) + 1j * rng.choice([-1.0, 1.0], shape)) / math.sqrt(2.0)


# ------------------------------------------------------- linear MMSE start --

def test_mmse_equals_the_push_through_form():
    """H (H^H H + n0 I)^-1 equals (H H^H + n0 I)^-1 H (a different formula of
    the same matrix), and minimises the mean squared error: perturbing U
    raises E|u^H r - x|^2 computed in closed form."""
    rng = np.random.default_rng(1)
    M, K, n0 = 6, 3, 0.2
    H = _cplx(rng, M, K)
    U = O.linear_mmse(H, n0)
    np.testing.assert_allclose(U, np.linalg.solve(H @ H.conj().T + n0 * np.eye(M), H), atol=1e-12)

    def mse(V):   # E|V^H r - x|^2 per user with E xx^H = I, E nn^H = n0 I
        A = V.conj().T @ H - np.eye(K)
        return np.real(np.sum(np.abs(A) ** 2, axis=1) + n0 * np.sum(np.abs(V) ** 2, axis=0))
    base = mse(U)
    for _ in range(5):
        assert np.all(mse(U + 1e-3 * _cplx(rng, M, K)) > base)


def test_zero_forcing_limit_inverts_the_channel():
    """n0 -> 0 with as many antennas as users: the filters invert H, so the
    linear filter of the real split detects noise-free symbols exactly."""
    rng = np.random.default_rng(2)
    M = K = 4
    H = _cplx(rng, M, K)
    f = O.filter_from_linear(O.linear_mmse(H, 0.0), sigma2=0.5)
    x = _qpsk(rng, 9, K)
    g = O.detect(f, x @ H.T)                     # r = H x for each row
    np.testing.assert_allclose(g, x, atol=1e-10)


def test_linear_filter_real_split_is_u_hermitian_r():
    rng = np.random.default_rng(3)
    U = _cplx(rng, 5, 2)
    f = O.filter_from_linear(U, sigma2=0.5)
    r = _cplx(rng, 7, 5)
    np.testing.assert_allclose(O.detect(f, r), r @ U.conj(), atol=1e-12)


def test_warm_started_linear_training_is_nlms_from_w0():
    """wG = 0, W = 1, eps = 0: training from f_0 = w0^T x is the NLMS
    recursion started at w0 (textbook, written here without kernels)."""
    rng = np.random.default_rng(4)
    T, M2, K = 40, 6, 2
    R = rng.standard_normal((T, M2)) / 2
    B = rng.choice([-1.0, 1.0], (T, K)) / math.sqrt(2)
    w0 = rng.standard_normal((K, M2)) * 0.3
    f0 = O.Filter(K, M2, 0.5)
    f0.w = w0.copy()
    p = O.APSMParams(sigma2=0.5, eps=0.0, mu=0.8, window=1, w_lin=0.5, w_gauss=0.0)
    tr = O.Trainer(R, B, p, f0=f0)
    for _ in range(T):
        tr.step()
    w = w0.copy()
    for n in range(T):
        w = w - 0.8 * np.outer(w @ R[n] - B[n], R[n]) / (R[n] @ R[n])
    np.testing.assert_allclose(tr.f.w, w, atol=1e-12)


def test_start_inside_every_slab_is_returned_unchanged():
    """If f_0 already lies in every hyperslab (|f_0(r_n) - b_n| <= eps), no
    projection moves it: the final filter is f_0."""
    rng = np.random.default_rng(5)
    T, M2, K, eps = 30, 4, 3, 0.05
    R = rng.standard_normal((T, M2))
    f0 = O.Filter(K, M2, 0.5)
    f0.w = rng.standard_normal((K, M2))
    B = R @ f0.w.T + rng.uniform(-0.9 * eps, 0.9 * eps, (T, K))
    tr = O.Trainer(R, B, O.APSMParams(eps=eps, window=5), f0=f0)
    for _ in range(T):
        tr.step()
    np.testing.assert_array_equal(tr.f.w, f0.w)
    assert np.all(tr.f.alpha == 0.0)
    # ... and one sample pushed outside its slab changes it (the check has teeth)
    B[7, 1] += 1.0
    tr = O.Trainer(R, B, O.APSMParams(eps=eps, window=5), f0=f0)
    for _ in range(T):
        tr.step()
    assert np.abs(tr.f.w - f0.w).max() > 1e-3


# ------------------------------------------------ continuing and tracking --

@pytest.mark.parametrize("cap", [None, 9, 1])
def test_continuing_with_window_one_equals_one_pass(cap):
    """With W = 1 the window restart at a block boundary changes nothing:
    training on the first part, then continuing on the rest (global
    dictionary indices), equals training on the whole sequence."""
    rng = np.random.default_rng(6)
    T, M2, K = 36, 4, 2
    R = rng.standard_normal((T, M2)) / 2
    B = rng.choice([-1.0, 1.0], (T, K)) / math.sqrt(2)
    p = O.APSMParams(sigma2=0.4, eps=0.05, mu=1.0, window=1, dict_cap=cap)
    whole = O.train(R, B, p)
    first = O.train(R[:20], B[:20], p)
    tr = O.Trainer(R[20:], B[20:], p, f0=first, n0=20)
    for _ in range(T - 20):
        tr.step()
    np.testing.assert_allclose(tr.f.w, whole.w, atol=1e-12)
    np.testing.assert_allclose(tr.f.alpha, whole.alpha, atol=1e-12)
    assert tr.f.dict_idx == whole.dict_idx


def test_continuing_restarts_the_window():
    """With W > 1 the continued training differs from one pass (the first
    steps of the block see a shorter window), and equals a one-pass training
    whose window is cut at the boundary: the term-list form over the whole
    sequence with the block's members only."""
    rng = np.random.default_rng(7)
    T, M2, K, W = 24, 4, 2, 4
    R = rng.standard_normal((T, M2)) / 2
    B = rng.choice([-1.0, 1.0], (T, K)) / math.sqrt(2)
    p = O.APSMParams(sigma2=0.4, eps=0.02, mu=1.0, window=W)
    whole = O.train(R, B, p)
    first = O.train(R[:10], B[:10], p)
    tr = O.Trainer(R[10:], B[10:], p, f0=first, n0=10)
    for _ in range(T - 10):
        tr.step()
    assert np.abs(tr.f.w - whole.w).max() > 1e-6
    # brute force: the same projections applied by hand with J_n cut at 10
    f = first.copy()
    for n in range(10, T):
        f.append(R[n], n)
        J = range(max(10, n - W + 1), n + 1)
        E = O.evaluate_many(f, R[list(J)])
        c = []
        for i, j in enumerate(J):
            kjj = 0.5 * (R[j] @ R[j]) + 0.5
            c.append((j, np.array([O.beta(E[i, k], B[j, k], p.eps, kjj) for k in range(K)]) / len(J)))
        for j, cj in c:
            f.w += np.outer(0.5 * cj, R[j])
            f.alpha[f.slot_of(j)] += 0.5 * cj
    np.testing.assert_allclose(tr.f.w, f.w, atol=1e-12)
    np.testing.assert_allclose(tr.f.alpha, f.alpha, atol=1e-12)


def test_decision_directed_with_correct_decisions_is_training_on_truth():
    """When every decision is right, decision-directed tracking is the same
    continuation as training on the transmitted symbols; the returned soft
    outputs are the frozen filter's."""
    rng = np.random.default_rng(8)
    M, K, P, S = 6, 2, 60, 25
    H = _cplx(rng, M, K)
    xp, xd = _qpsk(rng, P, K), _qpsk(rng, S, K)
    rp = xp @ H.T + 0.01 * _cplx(rng, P, M)
    rd = xd @ H.T + 0.01 * _cplx(rng, S, M)
    p = O.APSMParams(sigma2=2.0, eps=0.05, mu=1.0, window=4, dict_cap=80)
    Rp, Bp = O.training_sequence(rp, xp)
    f = O.train(Rp, Bp, p)
    planar = np.concatenate([rd.real, rd.imag], axis=1)
    soft = O.detect_planar(f, planar)
    assert np.array_equal(O.decided_symbols(soft, "qpsk"), xd)      # high SNR: all right
    g, soft2 = O.decision_directed(f, planar, "qpsk", p, n0=2 * P)
    np.testing.assert_array_equal(soft2, soft)
    Rd, Bd = O.training_sequence(rd, xd)
    tr = O.Trainer(Rd, Bd, p, f0=f, n0=2 * P)
    for _ in range(2 * S):
        tr.step()
    np.testing.assert_array_equal(g.w, tr.f.w)
    np.testing.assert_array_equal(g.alpha, tr.f.alpha)
    assert g.dict_idx == list(range(2 * P + 2 * S - 80, 2 * P + 2 * S))


def test_decided_symbols_are_nearest_levels():
    soft = np.array([[[0.3, -0.01]], [[-2.0, 0.0]]])
    d = O.decided_symbols(soft, "qpsk")
    a = 1 / math.sqrt(2)
    np.testing.assert_allclose(d, [[a - 1j * a], [-a + 1j * a]])
    lv = O.axis_levels("qam16")
    d = O.decided_symbols(np.array([[0.5, -0.1], [-5.0, 0.2]]), "qam16")
    np.testing.assert_allclose(d, [lv[2] + 1j * lv[1], lv[0] + 1j * lv[2]])   # thresholds 0, +-2/sqrt10


# ---------------------------------------------------- adaptive set weights --

def test_violation_weights_with_window_one_equal_uniform():
    rng = np.random.default_rng(9)
    R = rng.standard_normal((30, 4)) / 2
    B = rng.choice([-1.0, 1.0], (30, 3)) / math.sqrt(2)
    a = O.train(R, B, O.APSMParams(window=1, eps=0.05))
    b = O.train(R, B, O.APSMParams(window=1, eps=0.05, weight_mode="violation"))
    np.testing.assert_array_equal(a.w, b.w)
    np.testing.assert_array_equal(a.alpha, b.alpha)


def test_violation_weights_single_violated_member_lands_on_its_slab():
    """Only one member of the window outside its slab: it gets the whole
    weight, so with mu = 1 the step is that member's projection and
    f_{n+1}(r_j) lands on the slab boundary; uniform weights would land a
    quarter of the way."""
    rng = np.random.default_rng(10)
    M2, K, eps = 5, 1, 0.05
    R = rng.standard_normal((4, M2))
    f0 = O.Filter(K, M2, 0.5)
    f0.w = rng.standard_normal((K, M2))
    B = R @ f0.w.T                                   # every member inside
    B[2, 0] += 0.7                                   # ... but member 2
    p = O.APSMParams(eps=eps, mu=1.0, window=4, w_lin=0.5, w_gauss=0.5, weight_mode="violation")
    tr = O.Trainer(R, B, p, f0=f0)
    for _ in range(3):
        tr.step()                                    # steps 0..2: member 2 violated at step 2
    assert tr.f.evaluate(R[2])[0] == pytest.approx(B[2, 0] - eps, abs=1e-12)
    uni = O.Trainer(R, B, O.APSMParams(eps=eps, mu=1.0, window=4), f0=f0)
    for _ in range(3):
        uni.step()
    assert abs(uni.f.evaluate(R[2])[0] - (B[2, 0] - eps)) > 0.1


@pytest.mark.parametrize("mu,W", [(1.0, 4), (1.9, 6)])
def test_violation_weights_fejer_monotone(mu, W):
    """Any convex weights keep the iteration Fejer monotone toward a point
    of every slab (Sec. II-D, the weights only need q >= 0, sum 1)."""
    rng = np.random.default_rng(11)
    T, M2, K, eps, s2 = 40, 4, 2, 0.05, 0.4
    star = O.Filter(K, M2, s2)
    star.w = rng.standard_normal((K, M2)) * 0.5
    for m in range(4):
        star.append(rng.standard_normal(M2) * 0.6, -1 - m)
        star.alpha[-1] = rng.standard_normal(K) * 0.5
    R = rng.standard_normal((T, M2)) * 0.6
    B = np.array([star.evaluate(r) for r in R]) + rng.uniform(-0.9 * eps, 0.9 * eps, (T, K))
    tr = O.Trainer(R, B, O.APSMParams(sigma2=s2, eps=eps, mu=mu, window=W, weight_mode="violation"))
    prev = tr.f.h_norm2_diff(star, 0.5, 0.5)
    moved = 0
    for _ in range(T):
        tr.step()
        cur = tr.f.h_norm2_diff(star, 0.5, 0.5)
        assert np.all(cur <= prev * (1 + 1e-10) + 1e-12)
        moved += int(np.any(cur < prev * (1 - 1e-6)))
        prev = cur
    assert moved > 5


# ------------------------------------------ active-set weights, extrapolation

def test_active_weights_equal_uniform_while_every_member_is_violated():
    """Targets far from every prediction: all members violate their slabs, so
    uniform weights over the violated sets are the uniform weights."""
    rng = np.random.default_rng(31)
    R = rng.standard_normal((40, 4)) * 0.5
    B = 20.0 + rng.uniform(0, 1, (40, 2))
    base = dict(sigma2=0.5, eps=0.05, mu=0.2, window=6)
    a = O.Trainer(R, B, O.APSMParams(weight_mode="active", **base))
    b = O.Trainer(R, B, O.APSMParams(**base))
    held = 0
    for n in range(40):
        _, e, _ = b.step()
        if not all(np.all(np.abs(e[j] - B[j]) > base["eps"]) for j in e):
            break
        a.step()
        np.testing.assert_allclose(a.f.w, b.f.w, atol=1e-12)
        np.testing.assert_allclose(a.f.alpha, b.f.alpha, atol=1e-12)
        held += 1
    assert held >= 20


def test_active_weights_ignore_satisfied_members():
    """A member inside its slab gets weight 0: with two members of which only
    one is violated, the active step is that member's full projection."""
    rng = np.random.default_rng(32)
    R = rng.standard_normal((2, 4)) * 0.6
    p = O.APSMParams(sigma2=0.5, eps=0.1, mu=1.0, window=2, weight_mode="active")
    tr = O.Trainer(R, np.array([[0.0], [3.0]]), p)     # step 0: member 0 lands on its slab
    tr.step()
    f0 = tr.f.evaluate(R[0])[0]
    B = np.array([[f0], [3.0]])                          # member 0 now satisfied at step 1
    tr2 = O.Trainer(R, B, p)
    tr2.step()
    _, e, bet = tr2.step()
    assert abs(e[0][0] - B[0, 0]) <= p.eps and bet[0][0] == 0.0
    # q = (0, 1): f_{n+1}(r_1) lands on b_1 - eps
    np.testing.assert_allclose(tr2.f.evaluate(R[1])[0], B[1, 0] - p.eps, atol=1e-12)


def test_extrapolation_with_window_one_is_the_plain_step():
    rng = np.random.default_rng(33)
    R = rng.standard_normal((30, 4)) * 0.7
    B = rng.standard_normal((30, 3))
    a = O.train(R, B, O.APSMParams(window=1, extrapolate=True))
    b = O.train(R, B, O.APSMParams(window=1))
    np.testing.assert_allclose(a.w, b.w, atol=1e-13)
    np.testing.assert_allclose(a.alpha, b.alpha, atol=1e-13)


@pytest.mark.parametrize("mode", ["position", "active", "violation"])
def test_extrapolation_on_orthogonal_sets_is_every_projection_at_once(mode):
    """Gaussian part only, samples so far apart that their kernel sections are
    orthogonal: the extrapolated step moves every violated member onto its
    slab boundary (M_n undoes the averaging), which no averaged step does."""
    rng = np.random.default_rng(34)
    T, W = 24, 5
    R = rng.standard_normal((T, 4)) * 5.0
    B = rng.standard_normal((T, 2))
    p = O.APSMParams(sigma2=1e-3, eps=0.05, mu=1.0, window=W, w_lin=0.0, w_gauss=1.0,
                     extrapolate=True, weight_mode=mode)
    G = O.gram(R, p.sigma2, 0.0, 1.0)
    assert np.abs(G - np.eye(T)).max() < 1e-300          # orthogonal sections
    tr = O.Trainer(R, B, p)
    landed = 0
    for n in range(T):
        J, e, bet = tr.step()
        for j in J:
            for k in range(2):
                if abs(e[j][k] - B[j, k]) > p.eps:
                    target = B[j, k] + np.sign(e[j][k] - B[j, k]) * p.eps
                    np.testing.assert_allclose(tr.f.evaluate(R[j])[k], target, atol=1e-12)
                    landed += 1
    assert landed > T


@pytest.mark.parametrize("mu,mode", [(0.5, "position"), (1.0, "active"), (1.5, "violation"), (1.0, "position")])
def test_extrapolated_iteration_is_fejer_monotone(mu, mode):
    rng = np.random.default_rng(35)
    T, M2, K, eps, s2 = 45, 4, 2, 0.05, 0.4
    star = O.Filter(K, M2, s2)
    star.w = rng.standard_normal((K, M2)) * 0.5
    for m in range(5):
        star.append(rng.standard_normal(M2) * 0.6, -1 - m)
        star.alpha[-1] = rng.standard_normal(K) * 0.5
    R = rng.standard_normal((T, M2)) * 0.6
    B = np.array([star.evaluate(r) for r in R]) + rng.uniform(-0.9 * eps, 0.9 * eps, (T, K))
    p = O.APSMParams(sigma2=s2, eps=eps, mu=mu, window=6, extrapolate=True, weight_mode=mode)
    tr = O.Trainer(R, B, p)
    prev = tr.f.h_norm2_diff(star, 0.5, 0.5)
    moved = 0
    for _ in range(T):
        tr.step()
        cur = tr.f.h_norm2_diff(star, 0.5, 0.5)
        assert np.all(cur <= prev * (1 + 1e-10) + 1e-12)
        moved += int(np.any(cur < prev * (1 - 1e-6)))
        prev = cur
    assert moved > 5


def test_extrapolation_fejer_detects_an_overshoot():
    """Teeth: a step of 2.5 M_n (past the admissible relaxation) breaks Fejer."""
    rng = np.random.default_rng(36)
    T, M2, K, eps, s2 = 45, 4, 2, 0.05, 0.4
    star = O.Filter(K, M2, s2)
    star.w = rng.standard_normal((K, M2)) * 0.5
    R = rng.standard_normal((T, M2)) * 0.6
    B = np.array([star.evaluate(r) for r in R])
    p = O.APSMParams(sigma2=s2, eps=eps, mu=1.0, window=6, extrapolate=True)
    tr = O.Trainer(R, B, p)
    prev = tr.f.h_norm2_diff(star, 0.5, 0.5)
    broke = False
    for _ in range(T):
        w0 = tr.f.w.copy()
        tr.step()
        tr.f.w = w0 + 2.5 * (tr.f.w - w0)                 # planted mistake in the linear part
        cur = tr.f.h_norm2_diff(star, 0.5, 0.5)
        broke |= bool(np.any(cur > prev * (1 + 1e-6)))
        prev = cur
    assert broke
