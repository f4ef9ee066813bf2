"""GPU parity of batched training and detection (apsm_batch_* through the C
ABI): detectors of different shapes in one training launch and one detection
launch, against the FP64 oracle and against the one-detector-per-launch path
(apsm_train / apsm_detect) on the same inputs.  Rules and tolerances:
tests/parity_util.py."""
import os

import numpy as np
import pytest

import oracle as O
import synth
import paper_2201_05024_amd as A
from parity_util import REL_TOL, compare_hard, compare_soft, oracle_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def announce(msg):
    print(f"[case] {msg}", flush=True)


# K, M, P, S, cap, sigma2, modulation: every detection specialisation class
# (2M padded to 16 / 32 / 64, K 1..8), the FP32 path (K > 8 or 2M > 64),
# register-resident and model-buffer training, S = 0 and ragged tails.
MIXED = [
    (1, 1, 20, 65, 33, 0.5, "qpsk"),
    (2, 4, 60, 130, 64, 0.5, "qpsk"),
    (3, 3, 70, 1001, 70, 0.3, "qpsk"),
    (4, 8, 256, 2048, 256, 0.5, "qpsk"),
    (5, 12, 80, 333, 150, 0.5, "qam16"),
    (6, 16, 300, 200, 520, 0.5, "qpsk"),
    (7, 16, 90, 77, 100, 0.8, "qam16"),
    (8, 32, 100, 129, 200, 0.5, "qpsk"),
    (8, 8, 300, 0, 300, 0.5, "qpsk"),       # trained, nothing to detect
    (6, 32, 40, 64, 80, 0.5, "qam16"),
    (9, 16, 100, 77, 200, 0.5, "qpsk"),     # K > 8: FP32 detection path
    (16, 64, 64, 300, 100, 0.5, "qam16"),   # 2M = 128
    (2, 20, 50, 1, 40, 0.5, "qpsk"),
    (3, 4, 40, 70, 5000, 0.5, "qpsk"),     # dict_cap > 4096: trained without kernel rows
]
W = 8


def make_mixed(seed0=4000):
    insts, caps, sig = [], [], []
    for i, (K, M, P, S, cap, s2, mod) in enumerate(MIXED):
        spec = synth.InstanceSpec(K=K, M=M, P=P, S=max(S, 1), snr_db=12.0, modulation=mod, seed=seed0 + i)
        inst = synth.make_instance(spec)
        if S == 0:
            inst.rx_data = inst.rx_data[:0]
            inst.truth = inst.truth[:0]
        insts.append(inst)
        caps.append(cap)
        sig.append(s2)
    return insts, caps, sig


def build_batch(insts, caps, sig, params):
    items = []
    for inst, cap, s2 in zip(insts, caps, sig):
        K, M2, S = inst.spec.K, 2 * inst.spec.M, inst.rx_data.shape[0]
        m = A.Model(M2, K, cap, DEV, s2)
        items.append(A.BatchItem(
            model=m, rx_pilot=cuda(inst.rx_pilot), sym_pilot=cuda(inst.sym_pilot), rx=cuda(inst.rx_data),
            modulation=inst.spec.modulation, soft=torch.full((S, K, 2), 7.0, device=DEV),
            hard=torch.full((S, K), 255, dtype=torch.uint8, device=DEV), truth=cuda(inst.truth),
            errors=torch.zeros(K, dtype=torch.int64, device=DEV), sigma2=s2))
    return A.Batch(params, items), items


def test_batch_mixed_shapes_parity():
    announce(f"mixed batch of {len(MIXED)} shapes")
    insts, caps, sig = make_mixed()
    params = A.Params(eps=0.05, mu=1.0, window=W)
    batch, items = build_batch(insts, caps, sig, params)
    print("[step] batch planned and bound", flush=True)
    batch.train()
    torch.cuda.synchronize()
    print("[step] batch trained", flush=True)
    batch.detect()
    torch.cuda.synchronize()
    print("[step] batch detected", flush=True)
    for i, (inst, cap, s2, it) in enumerate(zip(insts, caps, sig, items)):
        print(f"[step] item {i}: {MIXED[i]}", flush=True)
        mod = inst.spec.modulation
        p = A.Params(sigma2=s2, eps=0.05, mu=1.0, window=W, dict_cap=cap)
        f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, oracle_params(p))
        T = 2 * inst.spec.P
        assert it.model.status() == {"size": min(T, cap), "head": T % cap, "steps": T, "flags": 0}, i
        assert np.abs(it.model.w.cpu().numpy() - f.w).max() <= REL_TOL * max(np.abs(f.w).max(), 1e-3), i
        S = inst.rx_data.shape[0]
        if S == 0:
            continue
        soft_ref = O.detect_planar(f, inst.rx_data)
        worst, _ = compare_soft(it.soft.cpu().numpy(), soft_ref, mod)
        assert worst <= REL_TOL, (i, worst)
        hard = it.hard.cpu().numpy()
        outside, inside = compare_hard(hard, soft_ref, mod)
        assert outside == 0, (i, outside, inside)
        np.testing.assert_array_equal(it.errors.cpu().numpy(), O.symbol_errors(hard, inst.truth))

        # the one-detector-per-launch path on the batch-trained model: same tiles, same code
        single = A.detect(it.model, it.rx, modulation=mod, truth=it.truth)
        torch.cuda.synchronize()
        assert torch.equal(single["soft"], it.soft), i
        assert torch.equal(single["hard"], it.hard), i
        assert torch.equal(single["errors"], it.errors), i

        # and training alone per detector agrees within the tolerance
        alone = A.train(it.rx_pilot, it.sym_pilot, p)
        torch.cuda.synchronize()
        assert torch.equal(alone.dict, it.model.dict), i
        scale = max(float(alone.w.abs().max()), 1e-3)
        assert float((alone.w - it.model.w).abs().max()) <= 1e-5 * scale, i
    print(f"[result] mixed batch ok", flush=True)


def test_batch_repeated_detect_and_tuned_form():
    """Repeated detection (the persistent form's claim counter returns to zero
    after every launch), then tuning, then detection in the tuned form: every
    run gives the same outputs and error counts accumulate exactly."""
    insts, caps, sig = make_mixed(seed0=4100)
    params = A.Params(window=W)
    batch, items = build_batch(insts, caps, sig, params)
    batch.train().detect()
    torch.cuda.synchronize()
    first = [(it.soft.clone(), it.hard.clone(), it.errors.clone()) for it in items]
    for rep in range(2, 4):
        batch.detect()
        torch.cuda.synchronize()
        for it, (s0, h0, e0) in zip(items, first):
            assert torch.equal(it.soft, s0) and torch.equal(it.hard, h0)
            assert torch.equal(it.errors, rep * e0)
    batch.tune()
    for it in items:
        it.errors.zero_()
    batch.detect()
    torch.cuda.synchronize()
    # tuning may move a shape class to the other detection kernel: the tuned
    # batch equals the one-detector path (which uses the same tuned choice)
    # bit for bit, and the untuned outputs within the tolerance
    for it, (s0, h0, e0) in zip(items, first):
        if it.rx.shape[0] == 0:
            continue
        single = A.detect(it.model, it.rx, modulation=it.modulation, truth=it.truth)
        torch.cuda.synchronize()
        assert torch.equal(single["soft"], it.soft) and torch.equal(single["hard"], it.hard)
        assert torch.equal(single["errors"], it.errors)
        ref = s0.cpu().numpy().astype(np.float64)
        worst, _ = compare_soft(it.soft.cpu().numpy(), ref, it.modulation)
        assert worst <= 2e-5, worst
    # both launch forms give the same outputs
    tuned = [(it.soft.clone(), it.hard.clone()) for it in items]
    for form, cus in ((False, 0), (True, 0), (True, 7), (False, 0), (True, 100000)):
        batch.set_form(form, cus).detect()
        torch.cuda.synchronize()
        for it, (s1, h1) in zip(items, tuned):
            assert torch.equal(it.soft, s1) and torch.equal(it.hard, h1), (form, cus)


def test_batch_graph_capture_replay():
    """The whole train -> pack -> detect -> error-count sequence captured once
    in a HIP graph (error counters cleared by a fill kernel inside it) and
    replayed three times, with eager work between replays; every replay
    equals the eager run."""
    insts, caps, sig = make_mixed(seed0=4200)
    params = A.Params(window=W)
    batch, items = build_batch(insts, caps, sig, params)
    batch.train().detect()
    torch.cuda.synchronize()
    ref = [(it.model.w.clone(), it.model.alpha.clone(), it.soft.clone(), it.hard.clone(), it.errors.clone())
           for it in items]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        for it in items:
            it.errors.zero_()
        batch.train().detect()
    torch.cuda.synchronize()
    for rep in range(3):
        for it in items:                       # eager work between replays
            it.soft.fill_(-1.0)
            it.hard.fill_(0)
            it.model.w.mul_(3.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, (it, (w0, a0, s0, h0, e0)) in enumerate(zip(items, ref)):
            assert torch.equal(it.model.w, w0), (rep, i)
            assert torch.equal(it.model.alpha, a0), (rep, i)
            assert torch.equal(it.soft, s0) and torch.equal(it.hard, h0), (rep, i)
            assert torch.equal(it.errors, e0), (rep, i)


def test_batch_split_training_on_two_streams():
    """Kernel rows on one stream and training on another, ordered by an event,
    give the same models as train() on one stream."""
    insts, caps, sig = make_mixed(seed0=4300)
    params = A.Params(window=W)
    b1, items1 = build_batch(insts, caps, sig, params)
    b1.train()
    torch.cuda.synchronize()
    ref = [(it.model.w.clone(), it.model.alpha.clone(), it.model.dict.clone(), it.model.status()) for it in items1]
    b2, items2 = build_batch(insts, caps, sig, params)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ev = torch.cuda.Event()
    b2.kernel_rows(s1)
    ev.record(s1)
    s2.wait_event(ev)
    b2.train_prepared(s2)
    torch.cuda.synchronize()
    for i, ((w, a, d, st), it) in enumerate(zip(ref, items2)):
        assert torch.equal(it.model.w, w) and torch.equal(it.model.alpha, a), i
        assert torch.equal(it.model.dict, d) and it.model.status() == st, i


def test_batch_full_mixed_workload_sampled():
    """The batched mixed workload at full size (256 detectors, K 2..8, 8/16/32
    antennas, dictionaries of 64..2048 entries with as many pilots, 65,536
    vectors each, QPSK/16-QAM, W = 32) in the launch configuration the
    benchmark times.  Every detector is checked against the
    one-detector-per-launch path on the GPU; the three with the smallest
    dictionaries are trained by the oracle and a sample of their outputs is
    evaluated by it."""
    n = synth.BATCH_INSTANCES
    announce(f"full mixed batch, {n} detectors")
    specs = [synth.spec_batch_mixed(i) for i in range(n)]
    params = A.Params(eps=0.05, mu=1.0, window=32)
    items, insts = [], []
    for spec, D in specs:
        inst = synth.make_instance(spec)
        insts.append(inst)
        K, M2, S = spec.K, 2 * spec.M, spec.S
        items.append(A.BatchItem(
            model=A.Model(M2, K, D, DEV, 0.5), rx_pilot=cuda(inst.rx_pilot), sym_pilot=cuda(inst.sym_pilot),
            rx=cuda(inst.rx_data), modulation=spec.modulation,
            soft=torch.empty((S, K, 2), device=DEV), hard=torch.empty((S, K), dtype=torch.uint8, device=DEV),
            truth=cuda(inst.truth), errors=torch.zeros(K, dtype=torch.int64, device=DEV), sigma2=0.5))
    print("[step] inputs resident", flush=True)
    batch = A.Batch(params, items)
    batch.train().detect()
    torch.cuda.synchronize()
    print("[step] batch done", flush=True)
    for i, (it, (spec, D)) in enumerate(zip(items, specs)):
        st = it.model.status()
        assert st["size"] == D and st["steps"] == 2 * D and st["flags"] == 0, i
        single = A.detect(it.model, it.rx, modulation=spec.modulation, truth=it.truth)
        torch.cuda.synchronize()
        assert torch.equal(single["soft"], it.soft), i
        assert torch.equal(single["errors"], it.errors), i
    print("[step] per-detector path agrees", flush=True)
    rng = np.random.default_rng(17)
    for i in sorted(range(n), key=lambda i: specs[i][1])[:3]:
        spec, D = specs[i]
        inst, it = insts[i], items[i]
        p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=32, dict_cap=D)
        f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, oracle_params(p))
        assert np.abs(it.model.w.cpu().numpy() - f.w).max() <= REL_TOL * max(np.abs(f.w).max(), 1e-3)
        idx = np.unique(np.concatenate([np.arange(64), np.arange(spec.S - 64, spec.S),
                                        rng.integers(0, spec.S, 512)]))
        soft_ref = O.detect_planar(f, inst.rx_data[idx])
        worst, _ = compare_soft(it.soft.cpu().numpy()[idx], soft_ref, spec.modulation)
        assert worst <= REL_TOL, (i, worst)
        outside, inside = compare_hard(it.hard.cpu().numpy()[idx], soft_ref, spec.modulation)
        assert outside == 0, (i, outside, inside)
        print(f"[result] detector {i} (K={spec.K}, M={spec.M}, D={D}): worst {worst:.2e}", flush=True)
    # the hardest detectors (largest dictionary; largest among 8 users, 16-QAM,
    # 2M = 64) against the oracle results stored by
    # tests/golden/make_oracle_samples.py
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "mixed_large.npz"))
    for i in [int(v) for v in g["which"]]:
        spec, D = specs[i]
        inst, it = insts[i], items[i]
        w_ref, a_ref = g[f"w_{i}"], g[f"alpha_{i}"]
        assert np.abs(it.model.w.cpu().numpy() - w_ref).max() <= REL_TOL * np.abs(w_ref).max(), i
        assert np.abs(it.model.alpha.cpu().numpy() - a_ref).max() <= REL_TOL * np.abs(a_ref).max(), i
        idx, soft_ref = g[f"idx_{i}"], g[f"soft_{i}"]
        worst, _ = compare_soft(it.soft.cpu().numpy()[idx], soft_ref, spec.modulation)
        assert worst <= REL_TOL, (i, worst)
        outside, inside = compare_hard(it.hard.cpu().numpy()[idx], soft_ref, spec.modulation)
        assert outside == 0, (i, outside, inside)
        print(f"[result] stored detector {i} (K={spec.K}, M={spec.M}, D={D}, {spec.modulation}): "
              f"worst {worst:.2e}, band mismatches {inside}", flush=True)


def test_both_detection_kernels_on_dual_shapes(tmp_path):
    """Shapes both detection kernels hold (2M <= 64, K <= 8): each kernel,
    selected through the tuning cache, matches the oracle; the cache choice
    is honoured by apsm_detect and by batches planned after it."""
    import json
    insts = [synth.make_instance(synth.InstanceSpec(K=K, M=M, P=120, S=700, snr_db=12.0, seed=4400 + K))
             for K, M in ((3, 8), (6, 16), (8, 32))]
    p = A.Params(window=W, dict_cap=200)
    models = [A.train(cuda(i.rx_pilot), cuda(i.sym_pilot), p) for i in insts]
    # learn the cache's device prefix from a tuned batch
    b = A.Batch(p, [A.BatchItem(model=models[0], rx_pilot=cuda(insts[0].rx_pilot),
                                sym_pilot=cuda(insts[0].sym_pilot), rx=cuda(insts[0].rx_data), modulation="qpsk",
                                soft=torch.empty((700, 3, 2), device=DEV))])
    b.tune()
    path = tmp_path / "cache.json"
    A.tune_save(str(path))
    keys = [k for k in json.loads(path.read_text()) if "|detect|" in k]
    assert keys, "tuning recorded no kernel choice"
    prefix = keys[0].split("|detect|")[0]
    for choice in ("f16", "wide"):
        entries = {f"{prefix}|detect|m2p{m2p}|k{K}": choice for m2p, K in ((16, 3), (32, 6), (64, 8))}
        path.write_text(json.dumps(entries))
        A.tune_load(str(path))
        for inst, m in zip(insts, models):
            f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, oracle_params(
                A.Params(window=W, dict_cap=200, sigma2=0.5, eps=0.05, mu=1.0)))
            out = A.detect(m, cuda(inst.rx_data), modulation="qpsk")
            torch.cuda.synchronize()
            soft_ref = O.detect_planar(f, inst.rx_data)
            worst, _ = compare_soft(out["soft"].cpu().numpy(), soft_ref, "qpsk")
            assert worst <= REL_TOL, (choice, inst.spec.K, worst)
            outside, _ = compare_hard(out["hard"].cpu().numpy(), soft_ref, "qpsk")
            assert outside == 0
            # a batch planned now uses the same kernel: bit-identical outputs
            soft = torch.empty_like(out["soft"])
            A.Batch(p, [A.BatchItem(model=m, rx_pilot=cuda(inst.rx_pilot), sym_pilot=cuda(inst.sym_pilot),
                                    rx=cuda(inst.rx_data), modulation="qpsk", soft=soft)]).detect()
            torch.cuda.synchronize()
            assert torch.equal(soft, out["soft"]), choice
    A.shutdown()
