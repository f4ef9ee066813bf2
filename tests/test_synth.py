"""The seeded generator: determinism, shapes, scaling and constellation."""
import math

import numpy as np

import synth


def test_deterministic_bytes():
    a = synth.make_instance(synth.spec_plain_small(S=64))
    b = synth.make_instance(synth.spec_plain_small(S=64))
    for name in ("rx_pilot", "sym_pilot", "rx_data", "sym_data", "truth"):
        assert getattr(a, name).tobytes() == getattr(b, name).tobytes()
    c = synth.make_instance(synth.spec_plain_small(seed=5, S=64))
    assert a.rx_pilot.tobytes() != c.rx_pilot.tobytes()


def test_shapes_dtypes_and_scale():
    inst = synth.make_instance(synth.spec_slot(10.0, S=300, P=128))
    K, M2 = 6, 32
    assert inst.rx_pilot.shape == (128, M2) and inst.rx_pilot.dtype == np.float32
    assert inst.sym_pilot.shape == (128, K, 2) and inst.sym_pilot.dtype == np.float32
    assert inst.rx_data.shape == (300, M2) and inst.truth.shape == (300, K)
    assert inst.truth.dtype == np.uint8
    p2 = np.mean(np.sum(inst.rx_pilot.astype(np.float64) ** 2, axis=1))
    assert abs(p2 - 1.0) < 1e-5
    pw = inst.extras["p"]
    assert np.all((pw <= 1.0) & (pw >= 10 ** (-0.6)))


def test_constellation_and_labels():
    inst = synth.make_instance(synth.InstanceSpec(K=3, M=2, P=4, S=4000, snr_db=10,
                                                   modulation="qam16", seed=3))
    re = inst.sym_data[..., 0].astype(np.float64)
    assert np.allclose(np.sort(np.unique(np.round(re * math.sqrt(10)))), [-3, -1, 1, 3])
    assert abs(np.mean(re ** 2 + inst.sym_data[..., 1].astype(np.float64) ** 2) - 1.0) < 0.05
    lv = synth.levels("qam16")
    idx_re = np.argmin(np.abs(re[..., None] - lv), axis=-1)
    assert np.array_equal(inst.truth >> 2, synth.gray(idx_re))


def test_rapp_qpsk_gain():
    b = np.array([1 + 0j, (1 + 1j) / math.sqrt(2)])
    x = synth._rapp(b, 2.0, 1.0)
    assert np.allclose(np.abs(x), 2 ** -0.25)


def test_device_generator_follows_the_host_recipe():
    """make_instance_device: pilots and channel equal make_instance's; the data
    block (drawn by torch) has the recipe's statistics and label alphabet and
    is reproducible from the seed."""
    torch = __import__("pytest").importorskip("torch")
    spec = synth.spec_large(3, S=4000, P=300)
    host = synth.make_instance(spec)
    dev = synth.make_instance_device(spec, "cpu")
    np.testing.assert_array_equal(dev.rx_pilot, host.rx_pilot)
    np.testing.assert_array_equal(dev.sym_pilot, host.sym_pilot)
    assert dev.scale == host.scale
    assert dev.rx_data.shape == (4000, 128) and dev.rx_data.dtype == torch.float32
    assert dev.truth.shape == (4000, 16) and int(dev.truth.max()) <= 15
    # unit mean squared norm over the pilots; the data block shares the scale
    m = float((dev.rx_data.double() ** 2).sum(1).mean())
    assert abs(m - 1.0) < 0.03, m
    again = synth.make_instance_device(spec, "cpu")
    assert torch.equal(again.rx_data, dev.rx_data) and torch.equal(again.truth, dev.truth)
    # every one of the 16 labels occurs, about equally often
    counts = np.bincount(dev.truth.numpy().ravel(), minlength=16)
    assert counts.min() > 0.8 * counts.mean()
