"""GPU parity of the generic projection engine against the FP64 oracle
(oracle/engine.py): training on per-sample set kinds (hyperslab,
hyperplane, upper and lower halfspace) on every single-detector training
path, with position and violation weights, and for a stack of detectors in
one launch; the ball projection (norms of Fact 1 evaluated through the
detection kernels, then scaling) on each detection kernel's shapes and with
one sum-space weight zero; cyclic projections (POCS) whose dictionary ring
wraps across cycles.  Tolerances: tests/parity_util.py."""
import numpy as np
import pytest

import oracle as O
import synth
import paper_2201_05024_amd as A
from oracle import engine as E
from parity_util import REL_TOL, compare_hard, compare_soft, oracle_model_to_ring, oracle_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def announce(msg):
    print(f"[case] {msg}", flush=True)


def opar(p, **kw):
    q = oracle_params(p)
    for k, v in kw.items():
        setattr(q, k, v)
    return q


def check_model(m, f, cap, what):
    w = m.w.cpu().numpy().astype(np.float64)
    assert np.abs(w - f.w).max() <= REL_TOL * max(np.abs(f.w).max(), 1e-3), what
    d_ref, a_ref = oracle_model_to_ring(f, cap)
    np.testing.assert_array_equal(m.dict.cpu().numpy().T, d_ref.astype(np.float32))
    assert np.abs(m.alpha.cpu().numpy() - a_ref).max() <= REL_TOL * max(np.abs(a_ref).max(), 1e-3), what


def check_detect(m, f, rx, mod, what):
    out = A.detect(m, cuda(rx), modulation=mod)
    torch.cuda.synchronize()
    ref = O.detect_planar(f, rx)
    worst, _ = compare_soft(out["soft"].cpu().numpy(), ref, mod)
    assert worst <= REL_TOL, (what, worst)
    outside, _ = compare_hard(out["hard"].cpu().numpy(), ref, mod)
    assert outside == 0, what


def kinds(rng, P, K):
    return rng.integers(0, 4, (P, K, 2)).astype(np.uint8)


PATHS = [
    # name, K, M, P, cap, W: register slots, coefficients in LDS, coefficients in the model buffers
    ("register_slots", 4, 8, 150, 256, 16),
    ("lds_coefficients", 6, 16, 600, 1100, 8),
    ("model_buffers", 16, 64, 300, 2200, 8),
]


@pytest.mark.parametrize("weights", ["position", "violation"])
@pytest.mark.parametrize("name,K,M,P,cap,W", PATHS)
def test_training_on_set_kinds(name, K, M, P, cap, W, weights):
    announce(f"set kinds {name} {weights}")
    inst = synth.make_instance(synth.InstanceSpec(K=K, M=M, P=P, S=300, snr_db=10.0, seed=7000 + K + W))
    st = kinds(np.random.default_rng(7000 + K), P, K)
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=W, dict_cap=cap, weights=weights, set_types=cuda(st))
    m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p)
    torch.cuda.synchronize()
    assert m.status()["flags"] == 0
    f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, opar(p, weight_mode=weights), set_types=st)
    check_model(m, f, cap, name)
    check_detect(m, f, inst.rx_data, "qpsk", name)
    # the kinds matter: hyperslabs everywhere give another filter
    g = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, opar(p, weight_mode=weights))
    assert np.abs(g.w - f.w).max() > 1e-3


def test_training_on_set_kinds_batched():
    """apsm_train_batched: three detectors of one shape with their own kinds."""
    announce("set kinds, three detectors in one launch")
    n, K, M, P, cap = 3, 6, 16, 200, 300
    insts = [synth.make_instance(synth.InstanceSpec(K=K, M=M, P=P, S=200, snr_db=12.0, seed=7100 + i))
             for i in range(n)]
    rng = np.random.default_rng(7100)
    st = np.stack([kinds(rng, P, K) for _ in range(n)])
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=16, dict_cap=cap, set_types=cuda(st))
    models = A.train_batched(cuda(np.stack([i.rx_pilot for i in insts])),
                             cuda(np.stack([i.sym_pilot for i in insts])), p)
    torch.cuda.synchronize()
    for i, (inst, m) in enumerate(zip(insts, models)):
        f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, opar(p), set_types=st[i])
        check_model(m, f, cap, f"detector {i}")


BALL = [
    # K, M, w_lin, w_gauss: the split-FP16 kernel's width (2M = 16), the
    # two-contraction kernel's (32, 128), one weight zero
    (4, 8, 0.5, 0.5), (6, 16, 0.5, 0.5), (16, 64, 0.5, 0.5), (6, 16, 1.0, 0.0), (6, 16, 0.0, 1.0),
]


@pytest.mark.parametrize("K,M,wl,wg", BALL)
def test_ball_projection(K, M, wl, wg):
    announce(f"ball K={K} 2M={2 * M} wL={wl} wG={wg}")
    P, cap = 250, 400
    inst = synth.make_instance(synth.InstanceSpec(K=K, M=M, P=P, S=300, snr_db=10.0, seed=7200 + K + M))
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=16, dict_cap=cap, w_lin=wl, w_gauss=wg)
    m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p)
    f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, opar(p))
    ref = E.h_norm(f, wl, wg)
    w0, a0 = m.w.clone(), m.alpha.clone()
    # a ball holding every user: the norms, the model unchanged
    nrm = A.project_ball(m, 10.0 * ref.max(), p).cpu().numpy()
    torch.cuda.synchronize()
    assert np.abs(nrm - ref).max() <= REL_TOL * ref.max(), (nrm, ref)
    assert torch.equal(m.w, w0) and torch.equal(m.alpha, a0)
    # a ball every user lies outside of
    rho = 0.5 * ref.min()
    A.project_ball(m, rho, p)
    torch.cuda.synchronize()
    g = E.project_ball(f, rho, wl, wg)
    check_model(m, g, cap, "projected")
    after = A.project_ball(m, 10.0 * rho, p).cpu().numpy()
    assert np.abs(after - rho).max() <= REL_TOL * rho
    check_detect(m, g, inst.rx_data, "qpsk", "projected")


@pytest.mark.parametrize("K,M,P,cap,W,weights", [(4, 8, 60, 150, 8, "position"), (6, 16, 100, 350, 16, "violation")])
def test_pocs_cycles(K, M, P, cap, W, weights):
    """Three cycles of projections onto the pilots' sets (mixed kinds) and
    onto a ball that binds; the ring wraps across cycles."""
    announce(f"POCS K={K} 2M={2 * M} P={P} cap={cap} {weights}")
    inst = synth.make_instance(synth.InstanceSpec(K=K, M=M, P=P, S=300, snr_db=12.0, seed=7300 + K))
    st = kinds(np.random.default_rng(7300 + K), P, K)
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=W, dict_cap=cap, weights=weights, set_types=cuda(st))
    q = opar(p, weight_mode=weights)
    free = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, q, set_types=st)
    rho = 0.6 * E.h_norm(free, 0.5, 0.5).min()
    m = A.pocs(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p, rho, 3)
    torch.cuda.synchronize()
    T = 3 * 2 * P
    assert m.status() == {"size": min(T, cap), "head": T % cap, "steps": T, "flags": 0}
    f = E.pocs(inst.rx_pilot, inst.sym_pilot, q, rho, 3, set_types=st)
    check_model(m, f, cap, "pocs")
    check_detect(m, f, inst.rx_data, "qpsk", "pocs")
    assert np.all(E.h_norm(f, 0.5, 0.5) <= rho * (1 + 1e-12))
