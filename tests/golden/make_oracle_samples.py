"""Writes the FP64 oracle's results for the full-size workloads whose oracle
training takes too long to repeat inside a test:

  slot_snr.npz     the realistic slot (6 users, 16 antennas, near-far powers,
                   Rapp PA, 1024 pilots, 1,048,576 data symbols, W = 32,
                   capacity 1024) at each SNR point 5, 10, 15, 20 dB: the
                   trained linear weights and ring coefficients, and the soft
                   outputs of a spread sample of 1024 data symbols.
  mixed_large.npz  the two hardest detectors of the 256-detector mixed batch
                   (W = 32, capacity = pilots): the one with the largest
                   dictionary, and the largest dictionary among those with
                   8 users, 16-QAM and 2M = 64; same contents, 512 symbols.

Inputs are regenerated from the seeded recipe (synth) by the tests.  Calls
only oracle/ and synth/ (no HIP library).  About six minutes of CPU.
Run: python tests/golden/make_oracle_samples.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import synth  # noqa: E402

PARAMS = dict(sigma2=0.5, eps=0.05, mu=1.0, window=32, w_lin=0.5, w_gauss=0.5)


def sample_indices(S, edge, spread, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.r_[0:edge, S - edge:S, rng.integers(0, S, spread)])


def ring_alpha(f, cap):
    alpha = np.zeros((cap, f.K))
    for n, a in zip(f.dict_idx, f.alpha):
        alpha[n % cap] = a
    return alpha


def hardest_mixed():
    """Index of the largest dictionary, and of the largest among the 8-user
    16-QAM detectors with 32 antennas."""
    specs = [synth.spec_batch_mixed(i) for i in range(synth.BATCH_INSTANCES)]
    big = max(range(len(specs)), key=lambda i: specs[i][1])
    cand = [i for i in range(len(specs))
            if specs[i][0].K == 8 and specs[i][0].M == 32 and specs[i][0].modulation == "qam16"]
    return [big, max(cand, key=lambda i: specs[i][1])]


def run(spec, cap, edge, spread, seed):
    inst = synth.make_instance(spec)
    f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, O.APSMParams(dict_cap=cap, **PARAMS))
    idx = sample_indices(spec.S, edge, spread, seed)
    soft = O.detect_planar(f, inst.rx_data[idx])
    return dict(w=f.w, alpha=ring_alpha(f, cap), idx=idx, soft=soft)


def main():
    out = {}
    for snr in synth.SLOT_SNRS_DB:
        r = run(synth.spec_slot(snr), 1024, 128, 768, int(snr))
        for k, v in r.items():
            out[f"{k}_{int(snr)}"] = v
        print("slot", snr, "dB done", flush=True)
    np.savez_compressed(os.path.join(HERE, "slot_snr.npz"), snrs=np.asarray(synth.SLOT_SNRS_DB), **out)
    out = {}
    which = hardest_mixed()
    for i in which:
        spec, D = synth.spec_batch_mixed(i)
        r = run(spec, D, 64, 384, 100 + i)
        for k, v in r.items():
            out[f"{k}_{i}"] = v
        print("mixed detector", i, spec.K, spec.M, D, spec.modulation, "done", flush=True)
    np.savez_compressed(os.path.join(HERE, "mixed_large.npz"), which=np.asarray(which), **out)


if __name__ == "__main__":
    main()
