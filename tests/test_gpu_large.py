"""GPU parity at the large-array width (2M = 128, 16 users, 16-QAM): training
with a dictionary capacity above 4096 whose ring fills and wraps, through the
batch path (kernel rows, the detector split into jobs of four users) and the
one-detector path (dictionary and coefficients in the model buffers),
against the FP64 oracle's results stored by tests/golden/make_large_wrap.py;
and batched detection of several large detectors against per-detector
detection.  Tolerances: tests/parity_util.py."""
import os

import numpy as np
import pytest

import oracle as O
import synth
import paper_2201_05024_amd as A
from parity_util import REL_TOL, compare_hard, compare_soft

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "large_wrap.npz")

# the case tests/golden/make_large_wrap.py wrote (same seeded inputs)
SPEC = dict(K=16, M=64, P=2100, S=128, snr_db=20.0, modulation="qam16", rapp=(2.0, 1.0), seed=4104)
PARAMS = dict(sigma2=0.5, eps=0.05, mu=1.0, window=8, w_lin=0.5, w_gauss=0.5, dict_cap=4104)


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def announce(msg):
    print(f"[case] {msg}", flush=True)


def check_against_golden(m, out, inst, g):
    cap = PARAMS["dict_cap"]
    T = 2 * SPEC["P"]
    st = m.status()
    assert st == {"size": cap, "head": T % cap, "steps": T, "flags": 0}, st
    # dictionary ring: slot n % cap holds r_n for the newest cap samples (bitwise)
    R, _ = O.training_sequence(synth.planar_to_complex(inst.rx_pilot), synth.pair_to_complex(inst.sym_pilot))
    d_ref = np.zeros((cap, R.shape[1]))
    for n in g["dict_idx"]:
        d_ref[n % cap] = R[n]
    np.testing.assert_array_equal(m.dict.cpu().numpy().T, d_ref.astype(np.float32))
    w_ref = g["w"]
    assert np.abs(m.w.cpu().numpy() - w_ref).max() <= REL_TOL * np.abs(w_ref).max()
    a_ref = g["alpha"]
    a_gpu = m.alpha.cpu().numpy()[g["slots"]]
    assert np.abs(a_gpu - a_ref).max() <= REL_TOL * np.abs(a_ref).max()
    soft_ref = g["soft"]
    worst, _ = compare_soft(out["soft"].cpu().numpy(), soft_ref, "qam16")
    assert worst <= REL_TOL, worst
    outside, inside = compare_hard(out["hard"].cpu().numpy(), soft_ref, "qam16")
    assert outside == 0, (outside, inside)
    return worst


def test_large_width_ring_wrap_batch_path():
    """Batch path: kernel rows, then four jobs of four users each with the
    coefficients of 16 slots per thread in registers."""
    announce("large width, cap 4104 > 4096, ring wraps: batch path")
    g = np.load(GOLDEN)
    inst = synth.make_instance(synth.InstanceSpec(**SPEC))
    p = A.Params(**PARAMS)
    m = A.Model(2 * SPEC["M"], SPEC["K"], PARAMS["dict_cap"], DEV, p.sigma2)
    rx = cuda(inst.rx_data)
    soft = torch.empty((SPEC["S"], SPEC["K"], 2), device=DEV)
    hard = torch.empty((SPEC["S"], SPEC["K"]), dtype=torch.uint8, device=DEV)
    b = A.Batch(p, [A.BatchItem(model=m, rx_pilot=cuda(inst.rx_pilot), sym_pilot=cuda(inst.sym_pilot), rx=rx,
                                modulation="qam16", soft=soft, hard=hard)])
    b.train().detect()
    torch.cuda.synchronize()
    worst = check_against_golden(m, {"soft": soft, "hard": hard}, inst, g)
    print(f"[result] batch path worst scaled error {worst:.2e}", flush=True)


def test_large_width_ring_wrap_single_path():
    """apsm_train: dictionary and coefficients in the model buffers."""
    announce("large width, cap 4104 > 4096, ring wraps: apsm_train")
    g = np.load(GOLDEN)
    inst = synth.make_instance(synth.InstanceSpec(**SPEC))
    p = A.Params(**PARAMS)
    m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p)
    out = A.detect(m, cuda(inst.rx_data), modulation="qam16")
    torch.cuda.synchronize()
    worst = check_against_golden(m, out, inst, g)
    print(f"[result] single path worst scaled error {worst:.2e}", flush=True)


def test_batched_large_detection_equals_per_detector():
    """Several detectors at the large-array width (full 8192-entry dictionary,
    ragged sample counts) in one persistent launch give bit-identical outputs
    to one apsm_detect launch each; also with the item list permuted (a
    different job order in the batch)."""
    announce("batched large detection vs per detector")
    K, M2, cap = 16, 128, 8192
    rng = np.random.default_rng(3)
    sizes = [40000, 33333, 1, 129]
    specs = [synth.spec_large(i, S=s, P=cap // 2 + 7 * i) for i, s in enumerate(sizes)]
    insts = [synth.make_instance_device(sp, DEV) for sp in specs]
    models = []
    for i, inst in enumerate(insts):
        m = A.Model(M2, K, cap, DEV, 0.5)
        R, _ = O.training_sequence(synth.planar_to_complex(inst.rx_pilot), synth.pair_to_complex(inst.sym_pilot))
        D = min(cap, len(R)) - 5 * i                   # partly filled dictionaries
        d = np.zeros((cap, M2), dtype=np.float32)
        d[:D] = R[:D]
        a = np.zeros((cap, K), dtype=np.float32)
        a[:D] = rng.standard_normal((D, K)) * 0.05
        m.dict.copy_(cuda(d.T))
        m.alpha.copy_(cuda(a))
        m.w.copy_(cuda(rng.standard_normal((K, M2)).astype(np.float32) * 0.05))
        m.state.copy_(cuda(np.array([D, D % cap, D, 0], dtype=np.int32)))
        m.pack()
        models.append(m)
    refs = [A.detect(m, inst.rx_data, modulation="qam16", truth=inst.truth) for m, inst in zip(models, insts)]
    for order in ([0, 1, 2, 3], [2, 0, 3, 1]):
        items = []
        for i in order:
            inst, m = insts[i], models[i]
            S = inst.spec.S
            items.append(A.BatchItem(model=m, rx_pilot=cuda(inst.rx_pilot), sym_pilot=cuda(inst.sym_pilot),
                                     rx=inst.rx_data, modulation="qam16", truth=inst.truth,
                                     soft=torch.empty((S, K, 2), device=DEV),
                                     hard=torch.empty((S, K), dtype=torch.uint8, device=DEV),
                                     errors=torch.zeros(K, dtype=torch.int64, device=DEV)))
        b = A.Batch(A.Params(window=8, dict_cap=cap), items)
        b.detect()
        torch.cuda.synchronize()
        for it, i in zip(items, order):
            r = refs[i]
            assert torch.equal(it.soft, r["soft"]), i
            assert torch.equal(it.hard, r["hard"]), i
            assert torch.equal(it.errors, r["errors"]), i
