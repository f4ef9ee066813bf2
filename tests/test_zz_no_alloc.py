"""apsm_train_noalloc (training that allocates no device memory, its kernel
rows in the library's static scratch array) against apsm_batch_train on a
one-item batch, which runs the same kernels from a caller workspace: the
model arrays must be bit-identical, and so must detection with them.  Two
calls in a row, the second with a smaller input, so that the second reuses
scratch the first left behind."""
import numpy as np
import pytest

import synth
import paper_2201_05024_amd as A

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def model_arrays(m):
    out = [m.dict, m.alpha, m.w, m.state]
    if m.packed is not None:
        out.append(m.packed)
    return [t.cpu().numpy().copy() for t in out]


CASES = [
    # K, M, P, cap, W, S: the second is smaller in every size
    (6, 16, 600, 1024, 32, 700),
    (3, 4, 70, 96, 8, 130),
]


def test_noalloc_training_matches_batched_training():
    for K, M, P, cap, W, S in CASES:
        print(f"[case] noalloc K={K} M={M} P={P} cap={cap} W={W}", flush=True)
        inst = synth.make_instance(synth.InstanceSpec(K=K, M=M, P=P, S=S, snr_db=10.0, seed=7000 + K))
        p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=W, dict_cap=cap)
        rx_p, sym_p, rx = cuda(inst.rx_pilot), cuda(inst.sym_pilot), cuda(inst.rx_data)
        m_ref = A.Model(2 * M, K, cap, DEV, p.sigma2)
        b = A.Batch(p, [A.BatchItem(model=m_ref, rx_pilot=rx_p, sym_pilot=sym_p)])
        b.train()
        m = A.Model(2 * M, K, cap, DEV, p.sigma2)
        # garbage in the model: the no-alloc call must overwrite all of it
        for t in (m.dict, m.alpha, m.w):
            t.fill_(3.0)
        A.train_noalloc(rx_p, sym_p, p, m)
        torch.cuda.synchronize()
        for a, r in zip(model_arrays(m), model_arrays(m_ref)):
            np.testing.assert_array_equal(a, r)
        o = A.detect(m, rx, modulation="qpsk", truth=cuda(inst.truth))
        o_ref = A.detect(m_ref, rx, modulation="qpsk", truth=cuda(inst.truth))
        np.testing.assert_array_equal(o["soft"].cpu().numpy(), o_ref["soft"].cpu().numpy())
        np.testing.assert_array_equal(o["hard"].cpu().numpy(), o_ref["hard"].cpu().numpy())
        np.testing.assert_array_equal(o["errors"].cpu().numpy(), o_ref["errors"].cpu().numpy())


def test_noalloc_rejects_what_does_not_fit():
    inst = synth.make_instance(synth.InstanceSpec(K=2, M=4, P=40, S=10, snr_db=10.0, seed=1))
    m = A.Model(8, 2, 8192, DEV, 0.5)
    with pytest.raises(A.APSMError) as e:       # dict_cap above the kernel-rows form
        A.train_noalloc(cuda(inst.rx_pilot), cuda(inst.sym_pilot),
                        A.Params(window=8, dict_cap=8192), m)
    assert e.value.code == 3
    big = synth.make_instance(synth.InstanceSpec(K=2, M=4, P=5000, S=10, snr_db=10.0, seed=2))
    m = A.Model(8, 2, 4096, DEV, 0.5)
    with pytest.raises(A.APSMError) as e:       # 2P (cap + W) floats beyond the scratch array
        A.train_noalloc(cuda(big.rx_pilot), cuda(big.sym_pilot), A.Params(window=8, dict_cap=4096), m)
    assert e.value.code == A.ERR_WORKSPACE
