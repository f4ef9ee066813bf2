"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each checks a consequence
(boundary landing of a projection, reduction to set-membership NLMS, exact
kernel interpolation, Fejer monotonicity, a brute-force unmerged form,
hand-derived closed forms) that a dropped term, a wrong sign, index or factor
in the oracle would break.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_seq(rng, T, M2, K, scale=1.0):
    R = rng.standard_normal((T, M2)) * scale / math.sqrt(M2)
    B = rng.choice([-1.0, 1.0], size=(T, K)) / math.sqrt(2.0)
    return R, B


# ---------------------------------------------------------------- eqn:beta --

@pytest.mark.parametrize("mu", [1.0, 0.5, 1.7])
@pytest.mark.parametrize("wl,wg", [(0.5, 0.5), (1.0, 0.0), (0.0, 1.0), (0.2, 0.9)])
def test_single_projection_lands_on_slab(mu, wl, wg):
    """W = 1: f_{n+1}(r_n) - b_n = (1 - mu)(e - b) + mu * sign(e - b) * eps when
    |e - b| > eps (mu = 1: exactly on the boundary), unchanged inside."""
    rng = np.random.default_rng(1)
    R, B = _rand_seq(rng, 40, 6, 3)
    p = O.APSMParams(sigma2=0.5, eps=0.05, mu=mu, window=1, w_lin=wl, w_gauss=wg)
    tr = O.Trainer(R, B, p)
    outside = inside = 0
    for n in range(len(R)):
        before = tr.f.evaluate(R[n]) if n > 0 else np.zeros(3)
        tr.step()
        after = tr.f.evaluate(R[n])
        x = before - B[n]
        for k in range(3):
            if abs(x[k]) > p.eps:
                want = (1 - mu) * x[k] + mu * math.copysign(p.eps, x[k])
                assert after[k] - B[n, k] == pytest.approx(want, abs=1e-12)
                outside += 1
            else:
                assert after[k] == pytest.approx(before[k], abs=1e-12)
                inside += 1
    assert outside > 10


def test_gaussian_only_interpolates():
    """wL = 0, eps = 0, W = 1, mu = 1: kernel NLMS interpolates the last sample."""
    rng = np.random.default_rng(2)
    R, B = _rand_seq(rng, 30, 4, 2)
    p = O.APSMParams(sigma2=0.3, eps=0.0, mu=1.0, window=1, w_lin=0.0, w_gauss=1.0)
    tr = O.Trainer(R, B, p)
    for n in range(len(R)):
        tr.step()
        np.testing.assert_allclose(tr.f.evaluate(R[n]), B[n], atol=1e-12)
    assert np.all(tr.f.w == 0.0)


# ------------------------------------------- linear part: NLMS reduction --

def _sm_nlms(R, B, W, mu, eps):
    """Set-membership NLMS with data reuse over a sliding window (textbook
    recursion, no kernels, no weights): every window member contributes the
    normalised correction -soft_eps(w^T r_j - b_j) r_j / ||r_j||^2, averaged."""
    T, M2 = R.shape
    K = B.shape[1]
    w = np.zeros((K, M2))
    for n in range(T):
        lo = max(0, n - W + 1)
        upd = np.zeros_like(w)
        for j in range(lo, n + 1):
            err = w @ R[j] - B[j]
            s = np.sign(err) * np.maximum(np.abs(err) - eps, 0.0)
            upd -= np.outer(s, R[j]) / (R[j] @ R[j])
        w = w + mu * upd / (n + 1 - lo)
    return w


@pytest.mark.parametrize("W,mu,eps,wl", [(1, 1.0, 0.0, 0.5), (4, 1.0, 0.05, 0.5),
                                          (8, 0.7, 0.1, 2.0), (3, 1.5, 0.02, 0.25)])
def test_linear_only_is_set_membership_nlms(W, mu, eps, wl):
    rng = np.random.default_rng(3)
    R, B = _rand_seq(rng, 60, 8, 3)
    f = O.train(R, B, O.APSMParams(sigma2=0.5, eps=eps, mu=mu, window=W, w_lin=wl, w_gauss=0.0))
    np.testing.assert_allclose(f.w, _sm_nlms(R, B, W, mu, eps), atol=1e-12)
    assert np.all(f.alpha == 0.0)


def test_linear_only_detector_is_complex_linear():
    """With wG = 0, g(r) = v^T r for a complex v, hence g(i r) = i g(r); the
    Gaussian part breaks this, which shows the check has teeth."""
    rng = np.random.default_rng(4)
    P, M, K = 20, 3, 2
    rx = rng.standard_normal((P, M)) + 1j * rng.standard_normal((P, M))
    sym = (rng.choice([-1, 1], (P, K)) + 1j * rng.choice([-1, 1], (P, K))) / math.sqrt(2)
    R, B = O.training_sequence(rx / 3, sym)
    test = (rng.standard_normal((7, M)) + 1j * rng.standard_normal((7, M))) / 3
    f = O.train(R, B, O.APSMParams(window=4, w_lin=0.5, w_gauss=0.0))
    np.testing.assert_allclose(O.detect(f, 1j * test), 1j * O.detect(f, test), atol=1e-12)
    f2 = O.train(R, B, O.APSMParams(window=4, w_lin=0.5, w_gauss=0.5))
    assert np.max(np.abs(O.detect(f2, 1j * test) - 1j * O.detect(f2, test))) > 1e-3


# ---------------------------------------------------------- kernels, Gram --

def test_gauss_kernel_values():
    # ||[1,0]-[0,1]||^2 = 2, sigma^2 = 0.5 -> exp(-2 / (2 * 0.5)) = e^-2
    assert O.kappa_gauss(np.array([1.0, 0.0]), np.array([0.0, 1.0]), 0.5) == pytest.approx(
        0.1353352832366127, abs=1e-16)
    assert O.kappa_gauss(np.array([0.3, -2.0]), np.array([0.3, -2.0]), 0.05) == 1.0
    assert O.kappa_lin(np.array([1.0, 2.0]), np.array([3.0, -4.0])) == -5.0


@pytest.mark.parametrize("wl,wg", [(0.5, 0.5), (0.0, 1.0), (1.0, 0.0)])
def test_gram_symmetric_psd(wl, wg):
    rng = np.random.default_rng(5)
    pts = rng.standard_normal((25, 6)) / 2
    G = O.gram(pts, 0.5, wl, wg)
    assert np.array_equal(G, G.T)
    ev = np.linalg.eigvalsh(G)
    assert ev.min() >= -1e-12 * np.trace(G)


# ------------------------------------------------------ Fejer monotonicity --

@pytest.mark.parametrize("mu,W", [(1.0, 4), (0.5, 1), (1.9, 6), (1.0, 1)])
def test_fejer_monotone_toward_planted_solution(mu, W):
    """Plant f* in H, make every hyperslab contain it (|f*(r_n) - b_n| <= eps);
    the iterates then never move away from f* in the H-norm of Fact 1."""
    rng = np.random.default_rng(6)
    T, M2, K, eps, s2 = 45, 4, 2, 0.05, 0.4
    star = O.Filter(K, M2, s2)
    star.w = rng.standard_normal((K, M2)) * 0.5
    for m in range(5):
        star.append(rng.standard_normal(M2) * 0.6, -1 - m)
        star.alpha[-1] = rng.standard_normal(K) * 0.5
    R = rng.standard_normal((T, M2)) * 0.6
    B = np.array([star.evaluate(r) for r in R]) + rng.uniform(-0.9 * eps, 0.9 * eps, (T, K))
    p = O.APSMParams(sigma2=s2, eps=eps, mu=mu, window=W, w_lin=0.5, w_gauss=0.5)
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


def test_fejer_detects_wrong_linear_weight():
    """Teeth: leaving out the wL factor of the linear update breaks Fejer."""
    rng = np.random.default_rng(6)
    T, M2, K, eps, s2 = 45, 4, 2, 0.05, 0.4
    star = O.Filter(K, M2, s2)
    star.w = rng.standard_normal((K, M2)) * 0.5
    R = rng.standard_normal((T, M2)) * 0.6
    B = np.array([star.evaluate(r) for r in R])
    p = O.APSMParams(sigma2=s2, eps=eps, mu=1.0, window=4, w_lin=0.25, w_gauss=0.5)
    tr = O.Trainer(R, B, p)
    prev = tr.f.h_norm2_diff(star, 0.25, 0.5)
    broke = False
    for n in range(T):
        w_before = tr.f.w.copy()
        tr.step()
        tr.f.w = w_before + (tr.f.w - w_before) / 0.25       # planted mistake
        cur = tr.f.h_norm2_diff(star, 0.25, 0.5)
        broke |= bool(np.any(cur > prev * (1 + 1e-6)))
        prev = cur
    assert broke


# ----------------------------------------- dictionary bookkeeping, caps --

@pytest.mark.parametrize("cap,W", [(None, 3), (5, 3), (3, 3), (4, 1), (7, 5)])
def test_termlist_equals_dictionary_form(cap, W):
    rng = np.random.default_rng(7)
    R, B = _rand_seq(rng, 24, 4, 2, scale=1.5)
    p = O.APSMParams(sigma2=0.5, eps=0.05, mu=1.0, window=W, w_lin=0.5, w_gauss=0.5, dict_cap=cap)
    a, b = O.Trainer(R, B, p), O.TermListTrainer(R, B, p)
    X = rng.standard_normal((6, 4))
    for _ in range(len(R)):
        a.step()
        b.step()
        for x in X:
            np.testing.assert_allclose(a.f.evaluate(x), b.evaluate(x), atol=1e-12)
        if cap is not None:
            assert len(a.f.dict_vec) <= cap


def test_termlist_with_position_weights():
    rng = np.random.default_rng(8)
    R, B = _rand_seq(rng, 20, 4, 2, scale=1.5)
    om = np.array([3.0, 1.0, 0.5, 2.0])
    p = O.APSMParams(sigma2=0.5, eps=0.02, mu=0.8, window=4, dict_cap=6, pos_weights=om)
    a, b = O.Trainer(R, B, p), O.TermListTrainer(R, B, p)
    X = rng.standard_normal((5, 4))
    for _ in range(len(R)):
        a.step()
        b.step()
    for x in X:
        np.testing.assert_allclose(a.f.evaluate(x), b.evaluate(x), atol=1e-12)


def test_position_weights_all_ones_equal_uniform():
    rng = np.random.default_rng(9)
    R, B = _rand_seq(rng, 30, 4, 2)
    f1 = O.train(R, B, O.APSMParams(window=5))
    f2 = O.train(R, B, O.APSMParams(window=5, pos_weights=np.full(5, 2.5)))
    np.testing.assert_allclose(f1.w, f2.w, atol=1e-13)
    np.testing.assert_allclose(f1.alpha, f2.alpha, atol=1e-13)


def test_cap_at_least_T_is_identical_to_uncapped():
    rng = np.random.default_rng(10)
    R, B = _rand_seq(rng, 40, 6, 3)
    f1 = O.train(R, B, O.APSMParams(window=6))
    f2 = O.train(R, B, O.APSMParams(window=6, dict_cap=40))
    f3 = O.train(R, B, O.APSMParams(window=6, dict_cap=39))
    assert np.array_equal(f1.w, f2.w) and np.array_equal(f1.alpha, f2.alpha)
    assert len(f3.dict_vec) == 39 and f3.dict_idx[0] == 1


def test_cap_below_window_rejected():
    with pytest.raises(ValueError):
        O.Trainer(np.zeros((4, 2)), np.zeros((4, 1)), O.APSMParams(window=4, dict_cap=3))


def test_window_sets():
    assert list(O.window(0, 4)) == [0]
    assert list(O.window(2, 4)) == [0, 1, 2]
    assert list(O.window(3, 4)) == [0, 1, 2, 3]
    assert list(O.window(9, 4)) == [6, 7, 8, 9]
    assert list(O.window(5, 1)) == [5]


# ------------------------------------------------ real split, detection --

def test_real_split_and_sequence_order():
    rx = np.array([[1 + 2j, 3 - 4j]])
    sym = np.array([[0.5 - 0.25j]])
    R, B = O.training_sequence(rx, sym)
    np.testing.assert_array_equal(R[0], [1, 3, 2, -4])      # r1 = [Re; Im]
    np.testing.assert_array_equal(R[1], [2, -4, -1, -3])    # r2 = [Im; -Re]
    np.testing.assert_array_equal(B[:, 0], [0.5, -0.25])


def test_golden_linear_two_steps():
    fx = json.load(open(os.path.join(GOLDEN, "linear_two_steps.json")))
    pr = fx["params"]
    p = O.APSMParams(sigma2=pr["sigma2"], eps=pr["eps"], mu=pr["mu"], window=pr["window"],
                     w_lin=pr["w_lin"], w_gauss=pr["w_gauss"])
    f = O.train_from_pilots(np.array(fx["rx_pilot"]), np.array(fx["sym_pilot"]), p)
    np.testing.assert_allclose(f.w, fx["expected_w"], atol=1e-14)
    soft = O.detect_planar(f, np.array(fx["rx_pilot"]))
    np.testing.assert_allclose(soft[:, 0, :], fx["expected_g_at_pilot"], atol=1e-14)


@pytest.mark.parametrize("case", ["uncapped", "cap1"])
def test_golden_gauss_two_steps(case):
    fx = json.load(open(os.path.join(GOLDEN, "gauss_two_steps.json")))
    pr = fx["params"]
    p = O.APSMParams(sigma2=pr["sigma2"], eps=pr["eps"], mu=pr["mu"], window=pr["window"],
                     w_lin=pr["w_lin"], w_gauss=pr["w_gauss"], dict_cap=fx[case]["dict_cap"])
    f = O.train_from_pilots(np.array(fx["rx_pilot"]), np.array(fx["sym_pilot"]), p)
    np.testing.assert_allclose(f.alpha, fx[case]["expected_alpha"], atol=1e-14)
    soft = O.detect_planar(f, np.array(fx["rx_pilot"]))
    np.testing.assert_allclose(soft[:, 0, :], fx[case]["expected_g_at_pilot"], atol=1e-14)


def test_golden_detect_two_entries():
    fx = json.load(open(os.path.join(GOLDEN, "detect_two_entries.json")))
    f = O.Filter(1, 2, fx["sigma2"])
    f.w = np.array(fx["w"])
    for d, a in zip(fx["dict"], fx["alpha"]):
        f.append(np.array(d), 0)
        f.alpha[-1] = a
    soft = O.detect_planar(f, np.array(fx["rx"]))
    np.testing.assert_allclose(soft, fx["expected_soft"], atol=1e-14)


def test_detect_matches_double_loop():
    rng = np.random.default_rng(11)
    M, K, D, S, s2 = 3, 2, 9, 13, 0.7
    f = O.Filter(K, 2 * M, s2)
    f.w = rng.standard_normal((K, 2 * M))
    for i in range(D):
        f.append(rng.standard_normal(2 * M), i)
        f.alpha[-1] = rng.standard_normal(K)
    rx = rng.standard_normal((S, M)) + 1j * rng.standard_normal((S, M))
    got = O.detect(f, rx, chunk=4)
    for s in range(S):
        for part in range(2):
            if part == 0:
                x = [v.real for v in rx[s]] + [v.imag for v in rx[s]]
            else:
                x = [v.imag for v in rx[s]] + [-v.real for v in rx[s]]
            for k in range(K):
                acc = sum(f.w[k, m] * x[m] for m in range(2 * M))
                for i in range(D):
                    d2 = sum((x[m] - f.dict_vec[i, m]) ** 2 for m in range(2 * M))
                    acc += f.alpha[i, k] * math.exp(-d2 / (2 * s2))
                val = got[s, k].real if part == 0 else got[s, k].imag
                assert val == pytest.approx(acc, abs=1e-12)


# ------------------------------------------------------ decisions, SER --

@pytest.mark.parametrize("mod,lv", [("qpsk", [-1, 1]), ("qam16", [-3, -1, 1, 3])])
def test_slicer_nearest_level(mod, lv):
    lv = np.array(lv, dtype=float) / math.sqrt(2 if mod == "qpsk" else 10)
    rng = np.random.default_rng(12)
    x = rng.uniform(-1.5, 1.5, 4000)
    brute = np.argmin(np.abs(x[:, None] - lv[None, :]), axis=1)
    np.testing.assert_array_equal(O.slice_axis(x, mod), brute)
    assert O.slice_axis(np.array([0.0]), mod)[0] == len(lv) // 2      # tie -> higher level
    assert O.slice_axis(np.array([-1e-12]), mod)[0] == len(lv) // 2 - 1


def test_labels_gray():
    s = 1 / math.sqrt(2)
    soft = np.array([[[-s, -s], [-s, s], [s, -s], [s, s]]])
    np.testing.assert_array_equal(O.decide(soft, "qpsk")[0], [0, 1, 2, 3])
    q = 1 / math.sqrt(10)
    levels = [-3 * q, -q, q, 3 * q]
    got = [int(O.decide(np.array([[[lv, -3 * q]]]), "qam16")[0, 0]) >> 2 for lv in levels]
    assert got == [0, 1, 3, 2]
    # adjacent levels differ in exactly one bit
    for a, b in zip(got[:-1], got[1:]):
        assert bin(a ^ b).count("1") == 1


def test_symbol_errors_and_boundary_distance():
    lab = np.array([[0, 1], [2, 1], [3, 0]], dtype=np.uint8)
    tru = np.array([[0, 1], [1, 1], [3, 3]], dtype=np.uint8)
    np.testing.assert_array_equal(O.symbol_errors(lab, tru), [1, 1])
    d = O.boundary_distance(np.array([[0.3, -0.01]]), "qpsk")
    assert d[0] == pytest.approx(0.01)


def test_position_weight_orientation():
    """omega[0] weights the newest set (j = n): W = 2 with omega = [1, ~0]
    is W = 1, while omega = [~0, 1] keeps mostly the older member."""
    rng = np.random.default_rng(13)
    R, B = _rand_seq(rng, 30, 4, 2)
    f1 = O.train(R, B, O.APSMParams(window=1))
    f2 = O.train(R, B, O.APSMParams(window=2, pos_weights=np.array([1.0, 1e-300])))
    np.testing.assert_allclose(f2.w, f1.w, atol=1e-12)
    np.testing.assert_allclose(f2.alpha, f1.alpha, atol=1e-12)
    f3 = O.train(R, B, O.APSMParams(window=2, pos_weights=np.array([1e-300, 1.0])))
    assert np.max(np.abs(f3.w - f1.w)) > 1e-3


@pytest.mark.parametrize("ratio,moves", [(1.005, True), (0.995, False), (-1.005, True), (-0.995, False)])
def test_slab_edge(ratio, moves):
    """Closed slab: |f(r_n) - b_n| slightly above eps projects onto the
    boundary, slightly below leaves f unchanged (eqn:beta, middle case)."""
    eps = 0.05
    r = np.array([0.6, 0.8])
    b = 0.3
    f0 = O.Filter(1, 2, 0.5)
    f0.w = np.array([[(b + ratio * eps) / 1.0 * r[0], (b + ratio * eps) / 1.0 * r[1]]])
    p = O.APSMParams(sigma2=0.5, eps=eps, mu=1.0, window=1, w_lin=1.0, w_gauss=0.0)
    tr = O.Trainer(r[None, :], np.array([[b]]), p, f0=f0)
    e0 = tr.f.evaluate(r)[0]
    assert e0 - b == pytest.approx(ratio * eps, abs=1e-14)
    tr.step()
    e1 = tr.f.evaluate(r)[0]
    if moves:
        assert e1 - b == pytest.approx(math.copysign(eps, ratio), abs=1e-14)
    else:
        assert e1 == e0
