"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded float32 inputs.  Rules and tolerances: tests/parity_util.py."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import synth
import paper_2201_05024_amd as A
from parity_util import (REL_TOL, compare_hard, compare_soft, oracle_model_to_ring,
                         oracle_params, ring_to_oracle_model, rounded)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def announce(msg):
    print(f"[case] {msg}", flush=True)


# ------------------------------------------------------------ detection only

def test_detect_golden_two_entries():
    fx = json.load(open(os.path.join(GOLDEN, "detect_two_entries.json")))
    m = A.Model(2, 1, 2, DEV, fx["sigma2"])
    m.dict.copy_(cuda(np.array(fx["dict"], dtype=np.float32).T))
    m.alpha.copy_(cuda(np.array(fx["alpha"], dtype=np.float32)))
    m.w.copy_(cuda(np.array(fx["w"], dtype=np.float32)))
    m.state.copy_(cuda(np.array([2, 0, 2, 0], dtype=np.int32)))
    m.pack()
    out = A.detect(m, cuda(np.array(fx["rx"], dtype=np.float32)), modulation=None)
    np.testing.assert_allclose(out["soft"].cpu().numpy(), fx["expected_soft"], atol=2e-6)


DETECT_CASES = [
    # K, M, P, S, cap, W, modulation
    (4, 8, 256, 2048, 256, 16, "qpsk"),
    (3, 3, 60, 1001, 70, 8, "qpsk"),        # M2 = 6 padded to 16; ragged D and S
    (1, 1, 20, 65, 33, 4, "qpsk"),
    (5, 12, 80, 333, 150, 10, "qam16"),     # M2 = 24 padded to 32
    (9, 16, 100, 77, 200, 16, "qpsk"),      # K > 8: one column tile per wave
    (16, 64, 64, 300, 100, 8, "qam16"),     # M2 = 128
    (6, 32, 40, 129, 80, 32, "qpsk"),       # M2 = 64
    # two-contraction kernel (2M > 64 or K > 8): every padded width, ragged
    # widths, users 1..16, several stages and a ragged last stage
    (12, 24, 200, 500, 300, 16, "qam16"),   # M2 = 48 -> 64, K = 12
    (10, 50, 150, 333, 260, 8, "qpsk"),     # M2 = 100 -> 128
    (16, 64, 300, 1000, 600, 32, "qam16"),  # M2 = 128, K = 16, 10 stages
    (1, 40, 60, 97, 100, 8, "qpsk"),        # M2 = 80, K = 1
    (9, 2, 50, 70, 64, 8, "qam16"),         # M2 = 4 -> 32, K = 9, D = 64 (one full stage)
]


@pytest.mark.parametrize("K,M,P,S,cap,W,mod", DETECT_CASES)
def test_detect_only_parity(K, M, P, S, cap, W, mod):
    """Oracle-trained model rounded to float32 -> GPU detect vs oracle detect."""
    announce(f"detect-only K={K} M={M} P={P} S={S} cap={cap} W={W} {mod}")
    inst = synth.make_instance(synth.InstanceSpec(K=K, M=M, P=P, S=S, snr_db=12, modulation=mod,
                                                  seed=1000 + K * 7 + M))
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=W, dict_cap=cap)
    f = rounded(O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, oracle_params(p)))
    d, al = oracle_model_to_ring(f, cap)
    m = A.Model(2 * M, K, cap, DEV, p.sigma2)
    m.dict.copy_(cuda(d.astype(np.float32).T))
    m.alpha.copy_(cuda(al.astype(np.float32)))
    m.w.copy_(cuda(f.w.astype(np.float32)))
    m.state.copy_(cuda(np.array([len(f.dict_vec), 0, 2 * P, 0], dtype=np.int32)))
    m.pack()
    out = A.detect(m, cuda(inst.rx_data), modulation=mod, truth=cuda(inst.truth))
    torch.cuda.synchronize()
    soft_ref = O.detect_planar(f, inst.rx_data)
    worst, _ = compare_soft(out["soft"].cpu().numpy(), soft_ref, mod)
    assert worst <= REL_TOL, worst
    hard = out["hard"].cpu().numpy()
    outside, inside = compare_hard(hard, soft_ref, mod)
    assert outside == 0, (outside, inside)
    np.testing.assert_array_equal(out["errors"].cpu().numpy(), O.symbol_errors(hard, inst.truth))


# ------------------------------------------------------------------ end to end

E2E_CASES = {
    # name: (spec kwargs, Params kwargs)
    "plain_small": (dict(K=4, M=8, P=256, S=2048, snr_db=10.0), dict(window=16, dict_cap=256)),
    "uncapped": (dict(K=4, M=8, P=128, S=500, snr_db=10.0), dict(window=16, dict_cap=256)),
    "window1": (dict(K=3, M=4, P=100, S=300, snr_db=15.0), dict(window=1, dict_cap=64)),
    "window64": (dict(K=4, M=8, P=150, S=300, snr_db=10.0), dict(window=64, dict_cap=64)),
    "mu_half": (dict(K=4, M=8, P=128, S=300, snr_db=10.0), dict(window=8, dict_cap=100, mu=0.5)),
    "mu_1p5": (dict(K=4, M=8, P=128, S=300, snr_db=10.0), dict(window=8, dict_cap=100, mu=1.5)),
    "linear_only": (dict(K=4, M=8, P=128, S=300, snr_db=10.0), dict(window=8, dict_cap=64, w_gauss=0.0, w_lin=1.0)),
    "gauss_only": (dict(K=4, M=8, P=128, S=300, snr_db=10.0), dict(window=8, dict_cap=64, w_lin=0.0, w_gauss=1.0)),
    "eps0": (dict(K=2, M=4, P=100, S=300, snr_db=10.0), dict(window=8, dict_cap=64, eps=0.0)),
    "pos_weights": (dict(K=4, M=8, P=128, S=300, snr_db=10.0),
                    dict(window=6, dict_cap=60, pos_weights=[3.0, 2.0, 1.0, 0.5, 0.25, 0.125])),
    "qam16": (dict(K=3, M=8, P=200, S=400, snr_db=25.0, modulation="qam16"), dict(window=16, dict_cap=256)),
    "k1_m1": (dict(K=1, M=1, P=64, S=100, snr_db=20.0), dict(window=4, dict_cap=32)),
    "odd_m": (dict(K=2, M=3, P=90, S=211, snr_db=12.0), dict(window=5, dict_cap=77)),
    "k16_m64": (dict(K=16, M=64, P=96, S=130, snr_db=20.0, modulation="qam16"), dict(window=16, dict_cap=128)),
    "model_buffer_path": (dict(K=6, M=32, P=300, S=200, snr_db=10.0), dict(window=32, dict_cap=520)),
    "m40_cap40": (dict(K=4, M=20, P=50, S=300, snr_db=12.0), dict(window=8, dict_cap=40)),
    "m48": (dict(K=3, M=24, P=60, S=200, snr_db=12.0, modulation="qam16"), dict(window=8, dict_cap=100)),
    "sigma_paper": (dict(K=6, M=16, P=160, S=300, snr_db=20.0), dict(window=20, dict_cap=320, sigma2=0.05)),
    "near_far_rapp": (dict(K=6, M=16, P=256, S=512, snr_db=10.0, near_far_db=(-6.0, 0.0), rapp=(2.0, 1.0)),
                      dict(window=32, dict_cap=256)),
}


def run_e2e(spec_kw, par_kw, seed):
    spec = synth.InstanceSpec(seed=seed, **spec_kw)
    inst = synth.make_instance(spec)
    p = A.Params(**{"sigma2": 0.5, "eps": 0.05, "mu": 1.0, **par_kw})
    m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p)
    out = A.detect(m, cuda(inst.rx_data), modulation=spec.modulation, truth=cuda(inst.truth))
    torch.cuda.synchronize()
    return inst, p, m, out


@pytest.mark.parametrize("name", list(E2E_CASES))
def test_end_to_end_parity(name):
    spec_kw, par_kw = E2E_CASES[name]
    announce(f"end-to-end {name} {spec_kw} {par_kw}")
    inst, p, m, out = run_e2e(spec_kw, par_kw, seed=2000 + len(name))
    mod = inst.spec.modulation
    f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, oracle_params(p))
    st = m.status()
    T = 2 * inst.spec.P
    assert st == {"size": min(T, p.dict_cap), "head": T % p.dict_cap, "steps": T, "flags": 0}
    # the trained model itself
    w_gpu = m.w.cpu().numpy().astype(np.float64)
    scale_w = max(np.abs(f.w).max(), 1e-3)
    assert np.abs(w_gpu - f.w).max() <= REL_TOL * scale_w
    d_ref, a_ref = oracle_model_to_ring(f, p.dict_cap)
    np.testing.assert_array_equal(m.dict.cpu().numpy().T, d_ref.astype(np.float32))
    if p.w_gauss > 0:
        scale_a = max(np.abs(a_ref).max(), 1e-3)
        assert np.abs(m.alpha.cpu().numpy() - a_ref).max() <= REL_TOL * scale_a
    # detection
    soft_ref = O.detect_planar(f, inst.rx_data)
    worst, _ = compare_soft(out["soft"].cpu().numpy(), soft_ref, mod)
    assert worst <= REL_TOL, worst
    hard = out["hard"].cpu().numpy()
    outside, inside = compare_hard(hard, soft_ref, mod)
    assert outside == 0, (outside, inside)
    errs = out["errors"].cpu().numpy()
    np.testing.assert_array_equal(errs, O.symbol_errors(hard, inst.truth))
    print(f"[result] {name}: worst scaled err {worst:.2e}, band mismatches {inside}, "
          f"SER gpu {errs.sum() / hard.size:.4g}", flush=True)


# ----------------------------------------------------------------- behaviour

def test_errors_accumulate_and_outputs_optional():
    inst = synth.make_instance(synth.InstanceSpec(K=3, M=4, P=64, S=500, snr_db=0.0, seed=5))
    p = A.Params(window=8, dict_cap=64)
    m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p)
    rx, truth = cuda(inst.rx_data), cuda(inst.truth)
    full = A.detect(m, rx, truth=truth)
    e1 = full["errors"].clone()
    assert int(e1.sum()) > 0                          # 0 dB: some errors to count
    A.detect(m, rx, truth=truth, errors=full["errors"], want_soft=False, want_hard=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(full["errors"].cpu().numpy(), 2 * e1.cpu().numpy())
    only_hard = A.detect(m, rx, want_soft=False)
    assert only_hard["soft"] is None
    assert torch.equal(only_hard["hard"], full["hard"])
    soft_only = A.detect(m, rx, modulation=None)
    assert soft_only["hard"] is None and torch.equal(soft_only["soft"], full["soft"])


@pytest.mark.parametrize("S", [0, 1, 15, 16, 17, 127, 128, 129])
def test_ragged_and_empty_inputs(S):
    inst = synth.make_instance(synth.InstanceSpec(K=2, M=4, P=40, S=max(S, 1), snr_db=10.0, seed=9))
    p = A.Params(window=4, dict_cap=40)
    m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p)
    rx = cuda(inst.rx_data[:S])
    soft = torch.full((S, 2, 2), 123.0, device=DEV)
    hard = torch.full((S, 2), 255, dtype=torch.uint8, device=DEV)
    A.detect(m, rx, soft=soft, hard=hard)
    torch.cuda.synchronize()
    if S == 0:
        return
    f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, oracle_params(p))
    ref = O.detect_planar(f, inst.rx_data[:S])
    worst, _ = compare_soft(soft.cpu().numpy(), ref, "qpsk")
    assert worst <= REL_TOL


def test_deterministic():
    inst = synth.make_instance(synth.InstanceSpec(K=6, M=16, P=300, S=5000, snr_db=8.0, seed=11))
    p = A.Params(window=32, dict_cap=256)
    outs = []
    for _ in range(2):
        m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p)
        o = A.detect(m, cuda(inst.rx_data), truth=cuda(inst.truth))
        torch.cuda.synchronize()
        outs.append((m.dict.clone(), m.alpha.clone(), m.w.clone(), o["soft"], o["hard"], o["errors"]))
    for x, y in zip(*outs):
        assert torch.equal(x, y)


def test_nonfinite_training_input_flagged():
    inst = synth.make_instance(synth.InstanceSpec(K=2, M=4, P=40, S=10, snr_db=10.0, seed=12))
    rx = inst.rx_pilot.copy()
    rx[7, 3] = np.nan
    m = A.train(cuda(rx), cuda(inst.sym_pilot), A.Params(window=4, dict_cap=40))
    assert m.status()["flags"] & 1
    m2 = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), A.Params(window=4, dict_cap=40), model=m)
    assert m2.status()["flags"] == 0


def test_batched_training_equals_single():
    """apsm_train_batched gives bit-identical models to per-instance training
    (and more instances than one launch holds are split correctly)."""
    specs = [synth.InstanceSpec(K=3, M=4, P=50, S=64, snr_db=8.0 + i, seed=300 + i) for i in range(35)]
    insts = [synth.make_instance(sp) for sp in specs]
    p = A.Params(window=6, dict_cap=64)
    rx = cuda(np.stack([i.rx_pilot for i in insts]))
    sym = cuda(np.stack([i.sym_pilot for i in insts]))
    models = A.train_batched(rx, sym, p)
    for idx in (0, 17, 31, 32, 34):
        single = A.train(cuda(insts[idx].rx_pilot), cuda(insts[idx].sym_pilot), p)
        torch.cuda.synchronize()
        for name in ("dict", "alpha", "w", "state", "packed"):
            assert torch.equal(getattr(models[idx], name), getattr(single, name)), (idx, name)


@pytest.mark.parametrize("M2,K,cap", [(2, 1, 7), (6, 3, 40), (16, 8, 64), (18, 2, 65), (32, 6, 100), (34, 4, 40),
                                      (40, 2, 40), (48, 5, 129), (62, 8, 64), (64, 7, 200), (66, 3, 50),
                                      (128, 16, 64)])
def test_training_and_packing_stay_inside_the_model(M2, K, cap):
    """Every byte the library writes lies inside the caller's buffers: each
    model array is carved from a larger buffer whose tail holds a guard
    pattern, which must be intact after training (and packing)."""
    P = 40
    rng = np.random.default_rng(M2 * 100 + K)
    rx = cuda(rng.normal(size=(P, M2)).astype(np.float32) * 0.3)
    sym = cuda(rng.choice([-0.7071, 0.7071], size=(P, K, 2)).astype(np.float32))
    m = A.Model(M2, K, cap, DEV, 0.5)
    guards = {}
    for name in ("dict", "alpha", "w", "state", "packed"):
        t = getattr(m, name)
        if t is None:
            continue
        nbytes = t.numel() * t.element_size()
        buf = torch.full((nbytes + 8192,), 0xA5, dtype=torch.uint8, device=DEV)
        buf[:nbytes].zero_()
        setattr(m, name, buf[:nbytes].view(t.dtype).view(t.shape))
        guards[name] = buf
    A.train(rx, sym, A.Params(window=4, dict_cap=cap), model=m)
    A.detect(m, rx, modulation="qpsk")
    torch.cuda.synchronize()
    for name, buf in guards.items():
        t = getattr(m, name)
        nbytes = t.numel() * t.element_size()
        assert bool((buf[nbytes:] == 0xA5).all()), (name, M2, K, cap)


# ------------------------------------------------------------ status flags

@pytest.mark.parametrize("K,M", [(4, 8), (9, 16)])     # split-FP16 path, FP32 path
def test_detect_flags_nonfinite_inputs(K, M):
    """Detection ORs FLAG_DETECT_NONFINITE into the model's flags word when a
    received vector holds a non-finite component, leaves it clear on finite
    inputs, and still writes every output; training resets the word."""
    announce(f"non-finite flag K={K} M={M}")
    inst = synth.make_instance(synth.InstanceSpec(K=K, M=M, P=64, S=300, snr_db=10.0, seed=901 + K))
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=8, dict_cap=128)
    m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p)
    out = A.detect(m, cuda(inst.rx_data), modulation="qpsk")
    assert m.status()["flags"] == 0
    rx = inst.rx_data.copy()
    rx[123, 2] = np.nan
    out2 = A.detect(m, cuda(rx), modulation="qpsk")
    st = m.status()
    assert st["flags"] == A.FLAG_DETECT_NONFINITE, st
    assert st["size"] == 128 and st["steps"] == 128           # the rest of the state is untouched
    s1, s2 = out["soft"].cpu().numpy(), out2["soft"].cpu().numpy()
    assert not np.isfinite(s2[123]).all()
    keep = np.arange(len(rx)) != 123
    # other vectors unaffected (a wave's power-of-two input scale may change)
    np.testing.assert_allclose(s1[keep], s2[keep], rtol=1e-6, atol=1e-6)
    rx[123, 2] = np.inf
    A.detect(m, cuda(rx), modulation="qpsk")
    assert m.status()["flags"] == A.FLAG_DETECT_NONFINITE
    m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p, model=m)
    assert m.status()["flags"] == 0


def test_batch_detect_flags_nonfinite_inputs():
    announce("non-finite flag, batched")
    insts = [synth.make_instance(synth.InstanceSpec(K=3, M=8, P=64, S=200, snr_db=10.0, seed=950 + i))
             for i in range(3)]
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=8, dict_cap=128)
    items = []
    for i, inst in enumerate(insts):
        rx = inst.rx_data.copy()
        if i == 1:
            rx[7, 0] = np.nan
        items.append(A.BatchItem(model=A.Model(16, 3, 128, DEV, 0.5), rx_pilot=cuda(inst.rx_pilot),
                                 sym_pilot=cuda(inst.sym_pilot), rx=cuda(rx), modulation="qpsk",
                                 soft=torch.empty((200, 3, 2), device=DEV)))
    b = A.Batch(p, items)
    b.train().detect()
    torch.cuda.synchronize()
    assert [it.model.status()["flags"] for it in items] == [0, A.FLAG_DETECT_NONFINITE, 0]



# ------------------------------------------------------------ large array

def test_detect_large_array_full_size_sampled():
    """The large-array shape at full size: 16 users (16-QAM), 2M = 128, a full
    dictionary of 8192 entries, 4,194,304 received vectors in one launch.  The
    dictionary is the last 8192 real training vectors of the pilots (what a
    capacity-8192 training leaves), the coefficients and linear weights are
    seeded draws (training at this size is covered elsewhere).  Outputs of a
    spread sample (the first and last 32 vectors and every 16384th) are
    checked against the FP64 oracle; on all vectors the decisions must be the
    slicer of the soft outputs, the error counts must equal the mismatches
    with the truth, and no non-finite flag may be raised."""
    announce("large array: K=16 2M=128 D=8192 S=4194304")
    spec = synth.spec_large(0)
    inst = synth.make_instance_device(spec, DEV)
    K, M2, cap = spec.K, 2 * spec.M, 8192
    rx_c = synth.planar_to_complex(inst.rx_pilot)
    sym_c = synth.pair_to_complex(inst.sym_pilot)
    R, _ = O.training_sequence(rx_c, sym_c)
    d = R[-cap:].astype(np.float32)                      # slot n % cap of sample n = 8192 + s
    rng = np.random.default_rng(55)
    alpha = (rng.standard_normal((cap, K)) * 0.05).astype(np.float32)
    w = (rng.standard_normal((K, M2)) * 0.05).astype(np.float32)
    m = A.Model(M2, K, cap, DEV, 0.5)
    m.dict.copy_(cuda(d.T))
    m.alpha.copy_(cuda(alpha))
    m.w.copy_(cuda(w))
    m.state.copy_(cuda(np.array([cap, 0, 2 * spec.P, 0], dtype=np.int32)))
    m.pack()
    out = A.detect(m, inst.rx_data, modulation="qam16", truth=inst.truth)
    torch.cuda.synchronize()
    S = spec.S
    idx = np.unique(np.r_[0:32, np.arange(0, S, 16384), S - 32:S])
    rx_sub = inst.rx_data[torch.from_numpy(idx).to(DEV)].cpu().numpy()
    f = ring_to_oracle_model(d.astype(np.float64), alpha.astype(np.float64), w.astype(np.float64), 0.5, cap)
    soft_ref = O.detect_planar(f, rx_sub, chunk=8)
    soft = out["soft"].cpu().numpy()
    worst, _ = compare_soft(soft[idx], soft_ref, "qam16")
    assert worst <= REL_TOL, worst
    hard = out["hard"].cpu().numpy()
    outside, inside = compare_hard(hard[idx], soft_ref, "qam16")
    assert outside == 0, (outside, inside)
    # decisions are the slicer of the soft outputs (values within 1e-6 of a
    # threshold excepted: the kernel compares against FP32 thresholds)
    s64 = soft.astype(np.float64)
    mism = (hard != O.decide(s64, "qam16")) & (O.boundary_distance(s64, "qam16") >= 1e-6)
    assert not mism.any(), int(mism.sum())
    truth = inst.truth.cpu().numpy()
    np.testing.assert_array_equal(out["errors"].cpu().numpy(), O.symbol_errors(hard, truth))
    assert m.status()["flags"] == 0
