"""GPU parity at full size against oracle results stored by
tests/golden/make_oracle_samples.py (the oracle's training at these sizes
takes minutes):

  * the realistic slot (6 users, 16 antennas, near-far powers, Rapp PA,
    1024 pilots, 1,048,576 data symbols, W = 32, capacity 1024) at every SNR
    point 5, 10, 15, 20 dB, trained and detected one detector per call and
    as the four-detector batch of the benchmark (kernel rows, persistent
    detection on all CUs but four);
  * symbol error counts on the stored sample equal to the oracle's, with
    decisions inside the rounding band resolved by the oracle's decision
    (and counted).

Inputs are regenerated from the seeded recipe.  Tolerances:
tests/parity_util.py."""
import os

import numpy as np
import pytest

import oracle as O
import synth
import paper_2201_05024_amd as A
from parity_util import BAND, REL_TOL, compare_hard, compare_soft

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PARAMS = dict(sigma2=0.5, eps=0.05, mu=1.0, window=32, w_lin=0.5, w_gauss=0.5, dict_cap=1024)


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def announce(msg):
    print(f"[case] {msg}", flush=True)


def resolved_errors(hard_sample, soft_ref, truth_sample, modulation):
    """Symbol errors of the sampled GPU decisions, with those whose oracle
    soft value lies inside the rounding band replaced by the oracle's
    decision; and how many were replaced."""
    ref_lab = O.decide(soft_ref, modulation)
    near = O.boundary_distance(soft_ref, modulation) < BAND
    lab = np.where(near, ref_lab, hard_sample)
    return O.symbol_errors(lab, truth_sample), int(np.sum(near & (hard_sample != ref_lab)))


def check_against_stored(m, soft, hard, errs, inst, g, key, modulation, what):
    cap = m.dict_cap
    T = 2 * inst.spec.P
    st = m.status()
    assert st == {"size": min(T, cap), "head": T % cap, "steps": T, "flags": 0}, (what, st)
    R, _ = O.training_sequence(synth.planar_to_complex(inst.rx_pilot), synth.pair_to_complex(inst.sym_pilot))
    d_ref = np.zeros((cap, R.shape[1]))
    for n in range(max(0, T - cap), T):
        d_ref[n % cap] = R[n]
    np.testing.assert_array_equal(m.dict.cpu().numpy().T, d_ref.astype(np.float32), err_msg=what)
    w_ref, a_ref = g[f"w_{key}"], g[f"alpha_{key}"]
    assert np.abs(m.w.cpu().numpy() - w_ref).max() <= REL_TOL * np.abs(w_ref).max(), what
    assert np.abs(m.alpha.cpu().numpy() - a_ref).max() <= REL_TOL * np.abs(a_ref).max(), what
    idx, soft_ref = g[f"idx_{key}"], g[f"soft_{key}"]
    worst, _ = compare_soft(soft.cpu().numpy()[idx], soft_ref, modulation)
    assert worst <= REL_TOL, (what, worst)
    h = hard.cpu().numpy()
    outside, inside = compare_hard(h[idx], soft_ref, modulation)
    assert outside == 0, (what, outside, inside)
    np.testing.assert_array_equal(errs.cpu().numpy(), O.symbol_errors(h, inst.truth), err_msg=what)
    e_gpu, replaced = resolved_errors(h[idx], soft_ref, inst.truth[idx], modulation)
    e_ref = O.symbol_errors(O.decide(soft_ref, modulation), inst.truth[idx])
    np.testing.assert_array_equal(e_gpu, e_ref, err_msg=what)
    ser = errs.sum().item() / h.size
    print(f"[result] {what}: worst {worst:.2e}, sample SER {e_ref.sum() / h[idx].size:.4g} "
          f"(band decisions resolved: {replaced}), full SER {ser:.4g}", flush=True)


def test_slot_every_snr_against_stored_oracle():
    g = np.load(os.path.join(GOLDEN, "slot_snr.npz"))
    snrs = [float(s) for s in g["snrs"]]
    assert snrs == list(synth.SLOT_SNRS_DB)
    p = A.Params(**PARAMS)
    insts = []
    for snr in snrs:
        announce(f"slot {snr} dB, one detector per call")
        inst = synth.make_instance(synth.spec_slot(snr))
        insts.append(inst)
        m = A.train(cuda(inst.rx_pilot), cuda(inst.sym_pilot), p)
        out = A.detect(m, cuda(inst.rx_data), modulation="qpsk", truth=cuda(inst.truth))
        torch.cuda.synchronize()
        check_against_stored(m, out["soft"], out["hard"], out["errors"], inst, g, int(snr), "qpsk",
                             f"single {snr} dB")
    announce("slot, the four SNR points as one batch")
    K, M2, S = 6, 32, insts[0].spec.S
    items = [A.BatchItem(model=A.Model(M2, K, PARAMS["dict_cap"], DEV, 0.5), rx_pilot=cuda(i.rx_pilot),
                         sym_pilot=cuda(i.sym_pilot), rx=cuda(i.rx_data), modulation="qpsk",
                         soft=torch.empty((S, K, 2), device=DEV),
                         hard=torch.empty((S, K), dtype=torch.uint8, device=DEV), truth=cuda(i.truth),
                         errors=torch.zeros(K, dtype=torch.int64, device=DEV)) for i in insts]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    b = A.Batch(p, items).set_form(True, cus - len(items))
    b.kernel_rows()
    b.train_prepared()
    b.detect()
    torch.cuda.synchronize()
    for snr, inst, it in zip(snrs, insts, items):
        check_against_stored(it.model, it.soft, it.hard, it.errors, inst, g, int(snr), "qpsk",
                             f"batch {snr} dB")
