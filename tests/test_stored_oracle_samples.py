"""The stored oracle results of tests/golden/make_oracle_samples.py (used by
the full-size GPU parity tests) are consistent with the seeded inputs the
tests regenerate: the stored model (linear weights, ring coefficients, and
the dictionary the ring holds after training) reproduces the stored soft
outputs through the oracle's detection, and the coefficients sit exactly in
the ring slots a capacity-bound training fills."""
import os

import numpy as np
import pytest

import oracle as O
import synth
from parity_util import ring_to_oracle_model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ring_dictionary(inst, cap):
    R, _ = O.training_sequence(synth.planar_to_complex(inst.rx_pilot), synth.pair_to_complex(inst.sym_pilot))
    T = R.shape[0]
    d = np.zeros((cap, R.shape[1]))
    for n in range(max(0, T - cap), T):
        d[n % cap] = R[n]
    return d


def check(inst, g, key, cap):
    w, alpha, idx, soft = g[f"w_{key}"], g[f"alpha_{key}"], g[f"idx_{key}"], g[f"soft_{key}"]
    assert w.shape == (inst.spec.K, 2 * inst.spec.M) and alpha.shape == (cap, inst.spec.K)
    assert np.all(np.diff(idx) > 0) and idx[0] == 0 and idx[-1] == inst.spec.S - 1
    assert soft.shape == (len(idx), inst.spec.K, 2)
    f = ring_to_oracle_model(ring_dictionary(inst, cap), alpha, w, 0.5, cap)
    pick = np.r_[0:4, len(idx) - 4:len(idx)]
    np.testing.assert_allclose(O.detect_planar(f, inst.rx_data[idx[pick]]), soft[pick], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("snr", list(synth.SLOT_SNRS_DB))
def test_slot_samples_consistent(snr):
    g = np.load(os.path.join(GOLDEN, "slot_snr.npz"))
    check(synth.make_instance(synth.spec_slot(snr)), g, int(snr), 1024)


def test_mixed_samples_consistent():
    g = np.load(os.path.join(GOLDEN, "mixed_large.npz"))
    which = [int(v) for v in g["which"]]
    specs = [synth.spec_batch_mixed(i) for i in which]
    assert max(D for _, D in (synth.spec_batch_mixed(i) for i in range(synth.BATCH_INSTANCES))) == specs[0][1]
    assert specs[1][0].K == 8 and specs[1][0].M == 32 and specs[1][0].modulation == "qam16"
    for i, (spec, D) in zip(which, specs):
        check(synth.make_instance(spec), g, i, D)
