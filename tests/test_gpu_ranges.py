"""GPU parity at the edges of the detection kernels' number formats, and
output bounds.

Both detection kernels form x.d from FP16 hi/lo splits of operands scaled by
powers of two: one exponent per tile of 16 received vectors and one per
dictionary.  Cases that strain those choices, each with the split-FP16
kernel and the two-contraction kernel on shapes both hold (2M = 32 and 64,
K <= 8) and with the two-contraction kernel alone at 2M = 128, K = 16:

  * every aligned tile of 16 received vectors spans magnitudes 2^0 .. 2^-20
    and holds one zero vector (its position moves from tile to tile);
  * one dictionary entry 2^10 times larger than the others;
  * detection on the training vectors themselves (r = d for dictionary
    entries: distance exactly zero in the oracle).

Output bounds: ragged S with guard tails after soft, hard and the error
counters, for each kernel, single and batched.  Tolerances:
tests/parity_util.py."""
import json

import numpy as np
import pytest

import oracle as O
import synth
import paper_2201_05024_amd as A
from parity_util import REL_TOL, compare_hard, compare_soft, oracle_model_to_ring, oracle_params, rounded

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def announce(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(autouse=True)
def clear_tuning_cache():
    """Each test starts and ends with an empty tuning cache (default kernels)."""
    A.shutdown()
    yield
    A.shutdown()


_PREFIX = []


def device_prefix(tmp_path):
    """The tuning cache's key prefix of this device (learnt once from a tuned batch)."""
    if _PREFIX:
        return _PREFIX[0]
    inst = synth.make_instance(synth.InstanceSpec(K=2, M=8, P=64, S=256, snr_db=10.0, seed=6000))
    p = A.Params(window=8, dict_cap=64)
    m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p)
    A.Batch(p, [A.BatchItem(model=m, rx_pilot=cuda(inst.rx_pilot), sym_pilot=cuda(inst.sym_pilot),
                            rx=cuda(inst.rx_data), modulation="qpsk",
                            soft=torch.empty((256, 2, 2), device=DEV))]).tune()
    path = tmp_path / "prefix.json"
    A.tune_save(str(path))
    keys = [k for k in json.loads(path.read_text()) if "|detect|" in k]
    assert keys, "tuning recorded no kernel choice"
    _PREFIX.append(keys[0].split("|detect|")[0])
    return _PREFIX[0]


def use_kernel(kernel, M2, K, tmp_path):
    """Select the detection kernel of the shape class of (M2, K) through the
    tuning cache ("f16" or "wide"; shapes only one kernel holds ignore it)."""
    A.shutdown()
    m2p = 16 if M2 <= 16 else 32 if M2 <= 32 else 64
    path = tmp_path / "kernel.json"
    path.write_text(json.dumps({f"{device_prefix(tmp_path)}|detect|m2p{m2p}|k{K}": kernel}))
    A.tune_load(str(path))


def model_from(f, cap, steps):
    m = A.Model(f.M2, f.K, cap, DEV, f.sigma2)
    d, al = oracle_model_to_ring(f, cap)
    m.dict.copy_(cuda(d.astype(np.float32).T))
    m.alpha.copy_(cuda(al.astype(np.float32)))
    m.w.copy_(cuda(f.w.astype(np.float32)))
    m.state.copy_(cuda(np.array([len(f.dict_vec), steps % cap, steps, 0], dtype=np.int32)))
    return m.pack()


def trained(K, M, mod, seed, P=200, cap=256, W=16):
    inst = synth.make_instance(synth.InstanceSpec(K=K, M=M, P=P, S=512, snr_db=15.0, modulation=mod, seed=seed))
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=W, dict_cap=cap)
    f = rounded(O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, oracle_params(p)))
    return inst, f


def check(m, f, rx, mod, what):
    out = A.detect(m, cuda(rx), modulation=mod)
    torch.cuda.synchronize()
    ref = O.detect_planar(f, rx)
    worst, _ = compare_soft(out["soft"].cpu().numpy(), ref, mod)
    outside, inside = compare_hard(out["hard"].cpu().numpy(), ref, mod)
    print(f"[result] {what}: worst scaled err {worst:.2e}, band mismatches {inside}", flush=True)
    assert worst <= REL_TOL, (what, worst)
    assert outside == 0, (what, outside)
    assert m.status()["flags"] == 0, what


RANGE_CASES = [
    # K, M, modulation, kernel
    (6, 16, "qpsk", "f16"), (6, 16, "qpsk", "wide"),
    (8, 32, "qam16", "f16"), (8, 32, "qam16", "wide"),
    (16, 64, "qam16", "wide"),
]


@pytest.mark.parametrize("K,M,mod,kernel", RANGE_CASES)
def test_tiles_spanning_twenty_octaves(K, M, mod, kernel, tmp_path):
    announce(f"tile magnitudes 2^0..2^-20 with a zero vector, K={K} 2M={2 * M} {kernel}")
    inst, f = trained(K, M, mod, 6100 + K)
    use_kernel(kernel, 2 * M, K, tmp_path)
    m = model_from(f, 256, 400)
    rx = inst.rx_data.astype(np.float64)
    S = rx.shape[0]
    expo = np.array([0, 1, 3, 4, 6, 7, 9, 10, 12, 13, 15, 16, 18, 19, 20], dtype=np.float64)
    scale = np.empty(S)
    for t in range(S // 16):
        e = np.append(2.0 ** -expo, 0.0)                  # 15 magnitudes and one zero vector
        scale[16 * t:16 * t + 16] = np.roll(e, t)
    rx = (rx * scale[:, None]).astype(np.float32)
    check(m, f, rx, mod, f"octaves {kernel}")


@pytest.mark.parametrize("K,M,mod,kernel", RANGE_CASES)
def test_dictionary_with_an_outlier(K, M, mod, kernel, tmp_path):
    announce(f"dictionary outlier x1024, K={K} 2M={2 * M} {kernel}")
    inst, f = trained(K, M, mod, 6200 + K)
    f.dict_vec = f.dict_vec.copy()
    f.dict_vec[len(f.dict_vec) // 3] *= 1024.0              # exact in float32
    use_kernel(kernel, 2 * M, K, tmp_path)
    m = model_from(f, 256, 400)
    check(m, f, inst.rx_data, mod, f"outlier {kernel}")


@pytest.mark.parametrize("K,M,mod,kernel", RANGE_CASES)
def test_detect_on_the_dictionary_vectors(K, M, mod, kernel, tmp_path):
    """The received vectors are the pilots: r1 and r2 of the later ones are
    dictionary entries, so the Gaussian distance cancels to zero."""
    announce(f"r = d, K={K} 2M={2 * M} {kernel}")
    inst, f = trained(K, M, mod, 6300 + K)
    use_kernel(kernel, 2 * M, K, tmp_path)
    m = model_from(f, 256, 400)
    check(m, f, inst.rx_pilot, mod, f"r=d {kernel}")


# ------------------------------------------------------------ output bounds

GUARD = 96


def guarded(S, K):
    soft = torch.full((S + GUARD, K, 2), 123.0, device=DEV)
    hard = torch.full((S + GUARD, K), 201, dtype=torch.uint8, device=DEV)
    errs = torch.full((K + GUARD,), 777, dtype=torch.int64, device=DEV)
    errs[:K] = 0
    return soft, hard, errs


def assert_guards(soft, hard, errs, S, K, what):
    assert bool((soft[S:] == 123.0).all()), (what, "soft")
    assert bool((hard[S:] == 201).all()), (what, "hard")
    assert bool((errs[K:] == 777).all()), (what, "errors")


GUARD_SHAPES = [
    # K, M, kernel: split-FP16 (2M = 16), both kernels at 2M = 64, two-contraction only (K > 8)
    (3, 8, "f16"), (8, 32, "f16"), (8, 32, "wide"), (12, 24, "wide"),
]


@pytest.mark.parametrize("S", [1, 15, 17, 129, 1000])
@pytest.mark.parametrize("K,M,kernel", GUARD_SHAPES)
def test_ragged_detection_stays_inside_its_outputs(K, M, kernel, S, tmp_path):
    announce(f"guards K={K} 2M={2 * M} {kernel} S={S}")
    inst = synth.make_instance(synth.InstanceSpec(K=K, M=M, P=120, S=S, snr_db=10.0, modulation="qam16",
                                                  seed=6400 + S))
    p = A.Params(window=8, dict_cap=150)
    use_kernel(kernel, 2 * M, K, tmp_path)
    m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p)
    soft, hard, errs = guarded(S, K)
    A.detect(m, cuda(inst.rx_data), modulation="qam16", truth=cuda(inst.truth),
             soft=soft[:S], hard=hard[:S], errors=errs[:K])
    torch.cuda.synchronize()
    assert_guards(soft, hard, errs, S, K, "single")
    f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, oracle_params(
        A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=8, dict_cap=150)))
    ref = O.detect_planar(f, inst.rx_data)
    worst, _ = compare_soft(soft[:S].cpu().numpy(), ref, "qam16")
    assert worst <= REL_TOL, worst
    h = hard[:S].cpu().numpy()
    np.testing.assert_array_equal(errs[:K].cpu().numpy(), O.symbol_errors(h, inst.truth))


@pytest.mark.parametrize("persistent", [True, False])
def test_ragged_batch_stays_inside_its_outputs(persistent, tmp_path):
    """One batch holding both kernels' shapes with ragged S, in both launch
    forms; every output has a guard tail."""
    announce(f"batch guards persistent={persistent}")
    shapes = [(3, 8, 1), (8, 32, 17), (12, 24, 129), (16, 64, 1000), (2, 4, 77)]
    p = A.Params(window=8, dict_cap=150)
    items, guards, insts = [], [], []
    for i, (K, M, S) in enumerate(shapes):
        inst = synth.make_instance(synth.InstanceSpec(K=K, M=M, P=120, S=S, snr_db=10.0, modulation="qam16",
                                                      seed=6500 + i))
        soft, hard, errs = guarded(S, K)
        items.append(A.BatchItem(model=A.Model(2 * M, K, 150, DEV, 0.5), rx_pilot=cuda(inst.rx_pilot),
                                 sym_pilot=cuda(inst.sym_pilot), rx=cuda(inst.rx_data), modulation="qam16",
                                 soft=soft[:S], hard=hard[:S], truth=cuda(inst.truth), errors=errs[:K]))
        guards.append((soft, hard, errs, S, K))
        insts.append(inst)
    A.Batch(p, items).set_form(persistent).train().detect()
    torch.cuda.synchronize()
    for i, ((soft, hard, errs, S, K), inst, it) in enumerate(zip(guards, insts, items)):
        assert_guards(soft, hard, errs, S, K, f"item {i}")
        single = A.detect(it.model, it.rx, modulation="qam16", truth=it.truth)
        torch.cuda.synchronize()
        assert torch.equal(single["soft"], soft[:S]), i
        assert torch.equal(single["hard"], hard[:S]), i
        assert torch.equal(single["errors"], errs[:K]), i
