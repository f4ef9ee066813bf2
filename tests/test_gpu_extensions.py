"""GPU parity of the extensions of the iteration against the FP64 oracle:
the linear MMSE start (apsm_linear_mmse and APSM_INIT_LINEAR), continuing a
trained model (APSM_INIT_CONTINUE) on every training path, decision-directed
tracking (apsm_track) on a slowly changing channel, and set weights
proportional to the slab violation (APSM_WEIGHTS_VIOLATION).  Tolerances:
tests/parity_util.py."""
import numpy as np
import pytest

import oracle as O
import synth
import paper_2201_05024_amd as A
from parity_util import (REL_TOL, compare_hard, compare_soft, oracle_model_to_ring, oracle_params)

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
    return worst


# ------------------------------------------------------------ linear MMSE

@pytest.mark.parametrize("M,K,n0", [(8, 4, 0.1), (64, 16, 0.01), (3, 3, 0.0), (1, 1, 0.5)])
def test_linear_mmse(M, K, n0):
    announce(f"linear MMSE M={M} K={K} n0={n0}")
    rng = np.random.default_rng(M * 100 + K)
    n = 3
    H = (rng.standard_normal((n, M, K)) + 1j * rng.standard_normal((n, M, K))) / np.sqrt(2)
    h = np.concatenate([H.real, H.imag], axis=1).transpose(0, 2, 1).astype(np.float32)   # [n][K][2M]
    w = A.linear_mmse(cuda(h), n0).cpu().numpy()
    for i in range(n):
        Hq = h[i, :, :M].T.astype(np.float64) + 1j * h[i, :, M:].T.astype(np.float64)
        ref = O.filter_from_linear(O.linear_mmse(Hq, n0), 0.5).w
        assert np.abs(w[i] - ref).max() <= 1e-4 * np.abs(ref).max(), i


def _effective_channel(inst):
    """The channel of the stored (scaled) received vectors: scale x H x
    sqrt(p), noise variance scale^2 N0 (QPSK, no PA model)."""
    H = inst.extras["H"] * np.sqrt(inst.extras["p"])[None, :] * inst.scale
    n0 = 10.0 ** (-inst.spec.snr_db / 10.0) * inst.scale ** 2
    return H, n0


@pytest.mark.parametrize("path", ["single", "batch"])
def test_training_from_linear_start(path):
    """f_0 = the MMSE filter of the true channel, then APSM training (single
    path and batch path from kernel rows) against the oracle started from its
    own FP64 MMSE filter."""
    announce(f"linear start, {path}")
    inst = synth.make_instance(synth.InstanceSpec(K=4, M=8, P=150, S=600, snr_db=8.0, seed=5150))
    H, n0 = _effective_channel(inst)
    K, M2, cap = 4, 16, 200
    h = np.concatenate([H.real, H.imag], axis=0).T.astype(np.float32)      # [K][2M]
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=8, dict_cap=cap, init="linear")
    m = A.Model(M2, K, cap, DEV, 0.5)
    A.linear_mmse(cuda(h), n0, w=m.w)
    if path == "single":
        A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p, model=m)
    else:
        A.Batch(p, [A.BatchItem(model=m, rx_pilot=cuda(inst.rx_pilot), sym_pilot=cuda(inst.sym_pilot))]).train()
    torch.cuda.synchronize()
    f0 = O.filter_from_linear(O.linear_mmse(H, n0), 0.5)
    f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, opar(p), f0=f0)
    check_model(m, f, cap, path)
    check_detect(m, f, inst.rx_data, "qpsk", path)
    # the start matters: training from f_0 = 0 gives a different filter
    g = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, opar(p))
    assert np.abs(g.w - f.w).max() > 1e-2


# ---------------------------------------------------------- continuing

CONT = [
    # name, K, M, P1, P2, cap, W: register slots, coefficients in LDS, coefficients in the model buffers
    ("register_slots", 6, 16, 150, 130, 200, 8),
    ("lds_coefficients", 6, 16, 700, 500, 1100, 8),
    ("model_buffers", 16, 64, 400, 200, 2200, 8),
]


@pytest.mark.parametrize("name,K,M,P1,P2,cap,W", CONT)
def test_continue_training(name, K, M, P1, P2, cap, W):
    """A model trained on one pilot block continues on a second one (its ring
    wraps where 2 (P1 + P2) > cap): as the oracle continuing its own filter
    with global dictionary indices and a fresh window."""
    announce(f"continue {name}")
    inst = synth.make_instance(synth.InstanceSpec(K=K, M=M, P=P1 + P2, S=300, snr_db=10.0, seed=5200 + K))
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=W, dict_cap=cap)
    rx1, sy1 = inst.rx_pilot[:P1], inst.sym_pilot[:P1]
    rx2, sy2 = inst.rx_pilot[P1:], inst.sym_pilot[P1:]
    m = A.train(cuda(rx1), cuda(sy1), p)
    pc = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=W, dict_cap=cap, init="continue")
    A.train(cuda(rx2), cuda(sy2), pc, model=m)
    torch.cuda.synchronize()
    st = m.status()
    T = 2 * (P1 + P2)
    assert st == {"size": min(T, cap), "head": T % cap, "steps": T, "flags": 0}, st
    f1 = O.train_from_pilots(rx1, sy1, opar(p))
    f = O.train_from_pilots(rx2, sy2, opar(p), f0=f1, n0=2 * P1)
    check_model(m, f, cap, name)
    check_detect(m, f, inst.rx_data, "qpsk", name)


# ------------------------------------------------------------ tracking

def test_decision_directed_tracking_follows_a_drifting_channel():
    """Train on pilots, then track four data blocks whose channel rotates
    away from the pilots' (apsm_track per block), against the oracle's
    decision_directed on its own filter; tracking lowers the symbol error
    rate of the last block against the frozen trained filter."""
    announce("tracking on a drifting channel")
    spec = synth.InstanceSpec(K=4, M=8, P=200, S=256, snr_db=12.0, seed=5301)
    pil, blocks = synth.make_drifting_blocks(spec, 5, 0.3)     # the oracle: 193 errors frozen, 0 tracked
    cap = 600
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=8, dict_cap=cap)
    m = A.train(cuda(pil.rx_pilot), cuda(pil.sym_pilot), p)
    frozen = A.Model(16, 4, cap, DEV, 0.5)
    A.train(cuda(pil.rx_pilot), cuda(pil.sym_pilot), p, model=frozen)
    f = O.train_from_pilots(pil.rx_pilot, pil.sym_pilot, opar(p))
    n = 2 * spec.P
    for b, (rx, truth, _) in enumerate(blocks[:-1]):
        out = A.track(m, cuda(rx), p, modulation="qpsk", truth=cuda(truth))
        torch.cuda.synchronize()
        f, soft_ref = O.decision_directed(f, rx, "qpsk", opar(p), n0=n)
        n += 2 * rx.shape[0]
        # the decisions the block was tracked on are the oracle's (none near a threshold)
        assert O.boundary_distance(soft_ref, "qpsk").min() > 1e-3, b
        np.testing.assert_array_equal(out["decided"].cpu().numpy(),
                                      np.stack([O.decided_symbols(soft_ref, "qpsk").real,
                                                O.decided_symbols(soft_ref, "qpsk").imag], -1).astype(np.float32))
        st = m.status()
        assert st["steps"] == n and st["size"] == min(n, cap) and st["flags"] == 0, (b, st)
        check_model(m, f, cap, f"block {b}")
    rx, truth, _ = blocks[-1]
    check_detect(m, f, rx, "qpsk", "last block")
    e_track = A.detect(m, cuda(rx), truth=cuda(truth))["errors"].sum().item()
    e_frozen = A.detect(frozen, cuda(rx), truth=cuda(truth))["errors"].sum().item()
    torch.cuda.synchronize()
    print(f"[result] last block errors: tracked {e_track}, frozen {e_frozen}", flush=True)
    assert e_track < e_frozen


# ------------------------------------------------------ violation weights

VIOL = [
    # name, K, M, P, cap, W, batch
    ("register_slots", 4, 8, 150, 256, 16, False),
    ("lds_coefficients", 6, 16, 600, 1100, 8, False),
    ("model_buffers", 16, 64, 300, 2200, 8, False),
    ("rows_batch", 6, 16, 300, 400, 32, True),
]


@pytest.mark.parametrize("name,K,M,P,cap,W,batch", VIOL)
def test_violation_weights(name, K, M, P, cap, W, batch):
    announce(f"violation weights {name}")
    inst = synth.make_instance(synth.InstanceSpec(K=K, M=M, P=P, S=300, snr_db=10.0, seed=5400 + K + W))
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=W, dict_cap=cap, weights="violation")
    if batch:
        m = A.Model(2 * M, K, cap, DEV, 0.5)
        A.Batch(p, [A.BatchItem(model=m, rx_pilot=cuda(inst.rx_pilot), sym_pilot=cuda(inst.sym_pilot))]).train()
    else:
        m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p)
    torch.cuda.synchronize()
    f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, opar(p, weight_mode="violation"))
    check_model(m, f, cap, name)
    check_detect(m, f, inst.rx_data, "qpsk", name)
    # different from position weights
    g = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, opar(A.Params(sigma2=0.5, window=W, dict_cap=cap)))
    assert np.abs(g.w - f.w).max() > 1e-3


# ------------------------------------ active-set weights, extrapolated relaxation

RELAX = [
    # name, K, M, P, cap, W, batch, weights, extrapolate
    ("register_slots", 4, 8, 150, 256, 16, False, "active", False),
    ("register_slots", 4, 8, 150, 256, 16, False, "position", True),
    ("register_slots", 4, 8, 150, 256, 16, False, "active", True),
    ("lds_coefficients", 6, 16, 600, 1100, 8, False, "violation", True),
    ("lds_coefficients", 6, 16, 600, 1100, 8, False, "active", False),
    ("model_buffers", 16, 64, 300, 2200, 8, False, "position", True),
    ("rows_batch", 6, 16, 300, 400, 32, True, "active", True),
    ("rows_batch", 6, 16, 300, 400, 32, True, "position", True),
    ("rows_batch_wrap", 3, 8, 400, 300, 16, True, "violation", True),
]


@pytest.mark.parametrize("name,K,M,P,cap,W,batch,weights,extrapolate", RELAX)
def test_active_weights_and_extrapolation(name, K, M, P, cap, W, batch, weights, extrapolate):
    announce(f"{weights} weights, extrapolate={extrapolate}, {name}")
    inst = synth.make_instance(synth.InstanceSpec(K=K, M=M, P=P, S=300, snr_db=10.0, seed=5500 + K + W))
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=W, dict_cap=cap, weights=weights, extrapolate=extrapolate)
    if batch:
        m = A.Model(2 * M, K, cap, DEV, 0.5)
        A.Batch(p, [A.BatchItem(model=m, rx_pilot=cuda(inst.rx_pilot), sym_pilot=cuda(inst.sym_pilot))]).train()
    else:
        m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p)
    torch.cuda.synchronize()
    assert m.status()["flags"] == 0
    f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, opar(p, weight_mode=weights, extrapolate=extrapolate))
    check_model(m, f, cap, name)
    check_detect(m, f, inst.rx_data, "qpsk", name)
    g = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, opar(p))
    assert np.abs(g.w - f.w).max() > 1e-3
