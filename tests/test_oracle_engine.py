"""Pins of the oracle's generic projection engine (oracle/engine.py and the
set kinds of the trainer) against what the mathematics fixes:

* the norm of Fact 1 computed from the merged coefficients equals the
  quadratic form of the unmerged term list, sum_{s,t} c_s c_t kappa(r_s, r_t),
  the definition of the RKHS norm of a finite kernel expansion;
* the ball projection returns the closest point of the ball (no point of
  the ball is closer), scales the function, and fixes points inside;
* each interval projection with one member and mu = 1 lands f_{n+1}(r_n) on
  the nearest point of its interval (a hyperplane interpolates exactly);
* hyperslabs through the interval form equal eqn:beta's three cases;
* Fejer monotonicity of every projection step and every cycle of the POCS
  iteration for a point inside all the sets, with a planted-mistake check.
"""
import numpy as np
import pytest

import oracle as O
from oracle import engine as E


def planted(rng, T, M2, K, s2, eps, kinds, gain=0.5):
    """f* with a linear part and a Gaussian expansion, samples, and targets
    whose sets all contain f* (hyperplane samples get b = f*(r))."""
    star = O.Filter(K, M2, s2)
    star.w = rng.standard_normal((K, M2)) * gain
    for m in range(5):
        star.append(rng.standard_normal(M2) * 0.6, -1 - m)
        star.alpha[-1] = rng.standard_normal(K) * gain
    R = rng.standard_normal((T, M2)) * 0.6
    F = np.array([star.evaluate(r) for r in R])
    U = rng.uniform(-0.9 * eps, 0.9 * eps, (T, K))
    U[kinds == O.SET_PLANE] = 0.0
    return star, R, F + U


def term_norm2(tl: O.TermListTrainer, p: O.APSMParams) -> np.ndarray:
    idx = [j for j, _ in tl.terms]
    C = np.array([c for _, c in tl.terms])                     # [terms][K]
    G = O.gram(tl.R[idx], p.sigma2, p.w_lin, p.w_gauss)        # full kernel kappa = wL kL + wG kG
    return np.einsum("sk,st,tk->k", C, G, C)


@pytest.mark.parametrize("wl,wg", [(0.5, 0.5), (0.25, 1.0), (1.0, 0.0), (0.0, 1.0)])
def test_norm_equals_term_list_quadratic_form(wl, wg):
    rng = np.random.default_rng(11)
    R = rng.standard_normal((26, 4)) * 0.8
    B = rng.standard_normal((26, 2))
    p = O.APSMParams(sigma2=0.4, eps=0.05, mu=1.0, window=3, w_lin=wl, w_gauss=wg)
    a, b = O.Trainer(R, B, p), O.TermListTrainer(R, B, p)
    for n in range(len(R)):
        a.step()
        b.step()
        if n % 5 == 4:
            np.testing.assert_allclose(E.h_norm(a.f, wl, wg) ** 2, term_norm2(b, p), rtol=1e-10, atol=1e-13)


def test_ball_projection_is_the_closest_point_of_the_ball():
    rng = np.random.default_rng(12)
    R = rng.standard_normal((30, 4)) * 0.8
    B = rng.standard_normal((30, 3)) * 2.0
    p = O.APSMParams(sigma2=0.5, eps=0.05, mu=1.0, window=4)
    f = O.train(R, B, p)
    nrm = E.h_norm(f, 0.5, 0.5)
    rho = 0.6 * nrm.min()                                       # every user outside
    g = E.project_ball(f, rho, 0.5, 0.5)
    np.testing.assert_allclose(E.h_norm(g, 0.5, 0.5), rho, rtol=1e-12)
    x = rng.standard_normal((5, 4))
    np.testing.assert_allclose(O.evaluate_many(g, x), O.evaluate_many(f, x) * (rho / nrm)[None, :], rtol=1e-12)
    d_proj = f.h_norm2_diff(g, 0.5, 0.5)
    for _ in range(20):
        # random members of the ball: scaled random expansions on fresh points
        h = O.Filter(3, 4, 0.5)
        h.w = rng.standard_normal((3, 4))
        for m in range(4):
            h.append(rng.standard_normal(4), m)
            h.alpha[-1] = rng.standard_normal(3)
        h.w *= 1.0
        hn = E.h_norm(h, 0.5, 0.5)
        s = rho * rng.uniform(0.1, 1.0, 3) / hn
        h.w *= s[:, None]
        h.alpha *= s[None, :]
        assert np.all(f.h_norm2_diff(h, 0.5, 0.5) >= d_proj * (1 - 1e-12))
    # inside: unchanged; idempotent
    same = E.project_ball(f, 2.0 * nrm.max(), 0.5, 0.5)
    np.testing.assert_array_equal(same.w, f.w)
    np.testing.assert_array_equal(same.alpha, f.alpha)
    again = E.project_ball(g, rho, 0.5, 0.5)
    np.testing.assert_allclose(again.w, g.w, rtol=1e-12)


@pytest.mark.parametrize("kind", [O.SET_SLAB, O.SET_PLANE, O.SET_UPPER, O.SET_LOWER])
def test_interval_projection_lands_on_the_nearest_point(kind):
    rng = np.random.default_rng(13 + kind)
    T, K, eps = 40, 2, 0.1
    R = rng.standard_normal((T, 4)) * 0.7
    B = rng.standard_normal((T, K))
    types = np.full((T, K), kind)
    p = O.APSMParams(sigma2=0.5, eps=eps, mu=1.0, window=1)
    tr = O.Trainer(R, B, p, types=types)
    inside = 0
    for n in range(T):
        before = tr.f.evaluate(R[n]) if n else np.zeros(K)
        _, e, _ = tr.step()
        after = tr.f.evaluate(R[n])
        for k in range(K):
            lo, hi = O.set_interval(kind, B[n, k], eps)
            target = min(max(e[n][k], lo), hi)
            np.testing.assert_allclose(after[k], target, atol=1e-12)
            inside += int(lo <= e[n][k] <= hi)
    if kind != O.SET_PLANE:
        assert inside > 0                 # some samples already satisfied their set


def test_slab_kind_equals_eqn_beta():
    rng = np.random.default_rng(14)
    R = rng.standard_normal((50, 6)) * 0.7
    B = rng.standard_normal((50, 3))
    p = O.APSMParams(sigma2=0.5, eps=0.2, mu=1.0, window=5, dict_cap=20)
    a = O.train(R, B, p)
    tr = O.Trainer(R, B, p, types=np.zeros((50, 3), dtype=int))
    for _ in range(50):
        tr.step()
    np.testing.assert_allclose(tr.f.w, a.w, atol=1e-13)
    np.testing.assert_allclose(tr.f.alpha, a.alpha, atol=1e-13)


def test_halfspace_equals_slab_while_only_its_bound_binds():
    """While no prediction exceeds its upper bound b + eps, the lower
    halfspaces and the slabs take the same projections, step by step."""
    rng = np.random.default_rng(15)
    R = rng.standard_normal((30, 4)) * 0.5
    B = 5.0 + rng.uniform(0, 1, (30, 2))
    p = O.APSMParams(sigma2=0.5, eps=0.1, mu=1.0, window=1)
    a = O.Trainer(R, B, p, types=np.full((30, 2), O.SET_LOWER))
    b = O.Trainer(R, B, p)
    held = 0
    for n in range(30):
        _, e, _ = b.step()
        if not np.all(e[n] < B[n] + p.eps):            # an upper bound binds: the sets differ from here on
            break
        a.step()
        np.testing.assert_allclose(a.f.w, b.f.w, atol=1e-12)
        np.testing.assert_allclose(a.f.alpha, b.f.alpha, atol=1e-12)
        held += 1
    assert held >= 10


def _mixed_kinds(rng, T, K):
    return rng.integers(0, 4, (T, K))


@pytest.mark.parametrize("W", [1, 4])
def test_pocs_is_fejer_monotone(W):
    rng = np.random.default_rng(16)
    T, M2, K, eps, s2 = 24, 4, 2, 0.05, 0.4
    kinds = _mixed_kinds(rng, T, K)
    star, R, B = planted(rng, T, M2, K, s2, eps, kinds)
    rho = 1.2 * E.h_norm(star, 0.5, 0.5).max()                  # f* inside the ball
    p = O.APSMParams(sigma2=s2, eps=eps, mu=1.0, window=W, w_lin=0.5, w_gauss=0.5)
    f = O.Filter(K, M2, s2)
    prev = f.h_norm2_diff(star, 0.5, 0.5)
    moved = 0
    for cyc in range(3):
        tr = O.Trainer(R, B, p, f0=f, n0=cyc * T, types=kinds)
        for _ in range(T):
            tr.step()
            cur = tr.f.h_norm2_diff(star, 0.5, 0.5)
            assert np.all(cur <= prev * (1 + 1e-10) + 1e-12)
            moved += int(np.any(cur < prev * (1 - 1e-6)))
            prev = cur
        f = E.project_ball(tr.f, rho, 0.5, 0.5)
        cur = f.h_norm2_diff(star, 0.5, 0.5)
        assert np.all(cur <= prev * (1 + 1e-10) + 1e-12)
        prev = cur
    assert moved > 5


def test_pocs_fejer_detects_a_wrong_halfspace_side():
    """Teeth: projecting the upper halfspaces onto the wrong side breaks Fejer."""
    rng = np.random.default_rng(17)
    T, M2, K, eps, s2 = 24, 4, 2, 0.05, 0.4
    kinds = np.full((T, K), O.SET_UPPER)
    star, R, B = planted(rng, T, M2, K, s2, eps, kinds)
    wrong = B - 0.5                       # upper bounds that f* violates
    p = O.APSMParams(sigma2=s2, eps=eps, mu=1.0, window=4)
    tr = O.Trainer(R, wrong, p, types=kinds)
    prev = tr.f.h_norm2_diff(star, 0.5, 0.5)
    broke = False
    for _ in range(T):
        tr.step()
        cur = tr.f.h_norm2_diff(star, 0.5, 0.5)
        broke |= bool(np.any(cur > prev * (1 + 1e-6)))
        prev = cur
    assert broke


def test_pocs_driver_equals_the_cycles_written_out():
    rng = np.random.default_rng(18)
    P, M, K = 10, 3, 2
    rx = rng.standard_normal((P, 2 * M)).astype(np.float32) * 0.5
    sym = rng.choice([-0.7, 0.7], (P, K, 2)).astype(np.float32)
    st = rng.integers(0, 4, (P, K, 2)).astype(np.uint8)
    p = O.APSMParams(sigma2=0.5, eps=0.05, mu=1.0, window=3, dict_cap=25)
    f = E.pocs(rx, sym, p, 0.3, 3, set_types=st)
    g = None
    for c in range(3):
        g = O.train_from_pilots(rx, sym, p, f0=g, n0=2 * P * c, set_types=st)
        g = E.project_ball(g, 0.3, 0.5, 0.5)
    np.testing.assert_array_equal(f.w, g.w)
    np.testing.assert_array_equal(f.alpha, g.alpha)
    assert f.dict_idx == g.dict_idx == list(range(60 - 25, 60))
    assert np.all(E.h_norm(f, 0.5, 0.5) <= 0.3 * (1 + 1e-12))
