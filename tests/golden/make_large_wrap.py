"""Writes large_wrap.npz: the FP64 oracle's training of one detector at the
large-array width (16 users with 16-QAM, 2M = 128, Rapp PA, 20 dB) with a
dictionary capacity above 4096 (4104 entries), over 2P = 4200 steps so that
the ring fills and then wraps 96 times; and the oracle's detection of 128
data vectors with the trained filter.  Stored: the linear weights, the
Gaussian coefficients of a spread set of ring slots, and the soft outputs.
Inputs are regenerated from the seeded recipe (synth) by the test.

Calls only oracle/ and synth/ (no HIP library).  About two minutes of CPU.
Run: python tests/golden/make_large_wrap.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import synth  # noqa: E402

SPEC = dict(K=16, M=64, P=2100, S=128, snr_db=20.0, modulation="qam16", rapp=(2.0, 1.0), seed=4104)
PARAMS = dict(sigma2=0.5, eps=0.05, mu=1.0, window=8, w_lin=0.5, w_gauss=0.5, dict_cap=4104)


def slots(cap):
    """Ring slots whose coefficients are stored: the first and last 64 and
    every 37th."""
    return np.unique(np.r_[0:64, cap - 64:cap, np.arange(0, cap, 37)])


def main():
    inst = synth.make_instance(synth.InstanceSpec(**SPEC))
    p = O.APSMParams(**PARAMS)
    f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, p)
    cap = PARAMS["dict_cap"]
    alpha = np.zeros((cap, SPEC["K"]))
    for n, a in zip(f.dict_idx, f.alpha):
        alpha[n % cap] = a
    sl = slots(cap)
    soft = O.detect_planar(f, inst.rx_data)
    np.savez_compressed(os.path.join(HERE, "large_wrap.npz"), w=f.w, slots=sl, alpha=alpha[sl], soft=soft,
                        dict_idx=np.asarray(f.dict_idx))
    print("wrote large_wrap.npz", f.w.shape, alpha[sl].shape, soft.shape)


if __name__ == "__main__":
    main()
