"""Seeded synthetic uplink NOMA data for the APSM detector.

This module draws the workload the detector is run on: channels, constellation
symbols, transmitter nonlinearity, noise.  It holds none of the detector's own
arithmetic (no real split, no kernels, no projections, no decisions); the same
float32 arrays it returns are fed unchanged to the FP64 oracle and to the HIP
library.

Signal model: the non-dispersive uplink of Sec. II-C, eqn:uplink_signal,
r(t) = sum_k sqrt(p_k) x_k(t) h_k + n(t), with x_k the (optionally Rapp
PA-distorted) constellation symbol b_k(t) of user k.

Storage convention for complex arrays handed to the library (an interface both
sides must agree on):

* a complex vector r in C^M is stored as M2 = 2M float32 values
  [Re r_0 .. Re r_{M-1}, Im r_0 .. Im r_{M-1}];
* a complex symbol b is stored as two float32 values (Re b, Im b);
* a decided/true symbol is stored as one uint8 label
  (gray(i_re) << bits_per_axis) | gray(i_im), with i_re / i_im the per-axis
  level index in increasing amplitude order and gray the binary-reflected
  Gray code of that index.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Per-axis amplitude levels of the unit-average-energy square constellations
# (QPSK: +-1/sqrt2; 16-QAM: {+-1, +-3}/sqrt10), increasing order.
_LEVELS = {
    "qpsk": np.array([-1.0, 1.0]) / np.sqrt(2.0),
    "qam16": np.array([-3.0, -1.0, 1.0, 3.0]) / np.sqrt(10.0),
}
BITS_PER_AXIS = {"qpsk": 1, "qam16": 2}


def gray(i: np.ndarray) -> np.ndarray:
    """Binary-reflected Gray code of a non-negative integer array."""
    i = np.asarray(i)
    return i ^ (i >> 1)


def levels(modulation: str) -> np.ndarray:
    return _LEVELS[modulation].copy()


def label_of(idx_re: np.ndarray, idx_im: np.ndarray, modulation: str) -> np.ndarray:
    b = BITS_PER_AXIS[modulation]
    return ((gray(idx_re) << b) | gray(idx_im)).astype(np.uint8)


@dataclass
class InstanceSpec:
    """Shape and channel recipe of one detector instance."""

    K: int                      # users
    M: int                      # receive antennas (complex); M2 = 2M reals
    P: int                      # pilot (training) symbols per user
    S: int                      # data symbols per user
    snr_db: float               # per-antenna SNR relative to a unit-power user
    modulation: str = "qpsk"    # "qpsk" | "qam16"
    near_far_db: Optional[tuple] = None   # (lo, hi): p_k = 10^(U[lo,hi]/10)
    rapp: Optional[tuple] = None          # (p, A_sat) Rapp AM/AM at each transmitter
    seed: int = 0


@dataclass
class Instance:
    spec: InstanceSpec
    rx_pilot: np.ndarray        # [P][2M] float32
    sym_pilot: np.ndarray       # [P][K][2] float32 (Re, Im) of the transmitted symbol b
    rx_data: np.ndarray         # [S][2M] float32
    sym_data: np.ndarray        # [S][K][2] float32
    truth: np.ndarray           # [S][K] uint8 labels of the data symbols
    scale: float                # real scalar applied to every received vector
    extras: dict = field(default_factory=dict)


def _draw_symbols(rng: np.random.Generator, n: int, K: int, modulation: str):
    L = len(_LEVELS[modulation])
    idx = rng.integers(0, L, size=(n, K, 2))
    lv = _LEVELS[modulation]
    b = lv[idx[..., 0]] + 1j * lv[idx[..., 1]]
    return b, idx


def _rapp(b: np.ndarray, p: float, a_sat: float) -> np.ndarray:
    """Rapp solid-state PA AM/AM characteristic (no AM/PM)."""
    a = np.abs(b)
    return b * (1.0 + (a / a_sat) ** (2.0 * p)) ** (-1.0 / (2.0 * p))


def _to_planar(r: np.ndarray) -> np.ndarray:
    return np.concatenate([r.real, r.imag], axis=-1).astype(np.float32)


def make_instance(spec: InstanceSpec) -> Instance:
    """Draw one instance.  Every random number comes from PCG64(spec.seed) in a
    fixed order, so the same spec gives byte-identical arrays."""
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    K, M = spec.K, spec.M
    # Block-fading i.i.d. Rayleigh channel, H[m, k] ~ CN(0, 1).
    H = (rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))) / np.sqrt(2.0)
    if spec.near_far_db is not None:
        lo, hi = spec.near_far_db
        p = 10.0 ** (rng.uniform(lo, hi, size=K) / 10.0)
    else:
        p = np.ones(K)
    n0 = 10.0 ** (-spec.snr_db / 10.0)

    def block(n):
        b, idx = _draw_symbols(rng, n, K, spec.modulation)
        x = _rapp(b, *spec.rapp) if spec.rapp is not None else b
        noise = (rng.standard_normal((n, M)) + 1j * rng.standard_normal((n, M))) * np.sqrt(n0 / 2.0)
        r = (x * np.sqrt(p)[None, :]) @ H.T + noise
        return r, b, idx

    r_p, b_p, _ = block(spec.P)
    r_d, b_d, idx_d = block(spec.S)
    # One real scale per instance so that the pilot block has unit mean
    # squared norm; the same scale applies to the data block.
    scale = 1.0 / np.sqrt(np.mean(np.sum(np.abs(r_p) ** 2, axis=1)))
    r_p = r_p * scale
    r_d = r_d * scale

    sym_p = np.stack([b_p.real, b_p.imag], axis=-1).astype(np.float32)
    sym_d = np.stack([b_d.real, b_d.imag], axis=-1).astype(np.float32)
    truth = label_of(idx_d[..., 0], idx_d[..., 1], spec.modulation)
    return Instance(spec=spec, rx_pilot=_to_planar(r_p), sym_pilot=sym_p,
                    rx_data=_to_planar(r_d), sym_data=sym_d, truth=truth,
                    scale=float(scale), extras={"H": H, "p": p})


def planar_to_complex(x: np.ndarray) -> np.ndarray:
    """Inverse of the storage convention: [..., 2M] float -> [..., M] complex128."""
    x = np.asarray(x, dtype=np.float64)
    M = x.shape[-1] // 2
    return x[..., :M] + 1j * x[..., M:]


def pair_to_complex(x: np.ndarray) -> np.ndarray:
    """[..., 2] (Re, Im) float -> [...] complex128."""
    x = np.asarray(x, dtype=np.float64)
    return x[..., 0] + 1j * x[..., 1]


# Named workloads.  Sizes follow the five benchmark configurations of the
# detector (tiny plain case, realistic slot, batched mixed shapes, differentiable
# unrolled training, large array) plus the paper's own shape (Sec. V: 6 users,
# 16 antennas, 685 training and 3840 data symbols, W = 20, sigma^2 = 0.05).
BASE_SEED = 220105024


def spec_plain_small(seed: int = BASE_SEED + 1, S: int = 2048) -> InstanceSpec:
    return InstanceSpec(K=4, M=8, P=256, S=S, snr_db=10.0, modulation="qpsk", seed=seed)


SLOT_SNRS_DB = (5.0, 10.0, 15.0, 20.0)


def spec_slot(snr_db: float, seed: int = BASE_SEED + 2, S: int = 1 << 20,
              P: int = 1024) -> InstanceSpec:
    return InstanceSpec(K=6, M=16, P=P, S=S, snr_db=snr_db, modulation="qpsk",
                        near_far_db=(-6.0, 0.0), rapp=(2.0, 1.0),
                        seed=seed + int(round(snr_db * 10)))


def spec_paper_shape(seed: int = BASE_SEED + 6) -> InstanceSpec:
    return InstanceSpec(K=6, M=16, P=685, S=3840, snr_db=20.0, modulation="qpsk", seed=seed)


BATCH_INSTANCES = 256


def spec_batch_mixed(i: int, seed: int = BASE_SEED + 3, S: int = 1 << 16):
    """Instance i of the batched mixed-shape workload: K uniform in {2..8}
    users, M in {8, 16, 32} antennas, dictionary size D uniform in [64, 2048]
    with P = D pilots (so the capacity binds after half the training steps),
    QPSK or 16-QAM by a fair coin, SNR uniform in [5, 20] dB, unit user powers.
    Returns (spec, D)."""
    rng = np.random.default_rng([seed, i])
    K = int(rng.integers(2, 9))
    M = int(rng.choice([8, 16, 32]))
    D = int(rng.integers(64, 2049))
    mod = "qam16" if rng.random() < 0.5 else "qpsk"
    snr = float(rng.uniform(5.0, 20.0))
    spec = InstanceSpec(K=K, M=M, P=D, S=S, snr_db=snr, modulation=mod, seed=seed * 1000 + i)
    return spec, D


LARGE_INSTANCES = 16


def spec_large(i: int = 0, seed: int = BASE_SEED + 5, S: int = 1 << 22, P: int = 8192) -> InstanceSpec:
    """Instance i of the large-array workload: 16 users with 16-QAM, 64
    receive antennas (2M = 128), Rapp PA at every transmitter, 20 dB, 8192
    pilots (2P = 16384 real training vectors, twice the dictionary capacity
    8192) and 4,194,304 data symbols."""
    return InstanceSpec(K=16, M=64, P=P, S=S, snr_db=20.0, modulation="qam16", rapp=(2.0, 1.0),
                        seed=seed * 1000 + i)


@dataclass
class DeviceInstance:
    """An instance whose data block lives in device memory (torch tensors);
    pilots and channel are host arrays as in Instance."""
    spec: InstanceSpec
    rx_pilot: np.ndarray        # [P][2M] float32 (host)
    sym_pilot: np.ndarray       # [P][K][2] float32 (host)
    rx_data: object             # [S][2M] float32 torch tensor on the device
    truth: object               # [S][K] uint8 torch tensor on the device
    scale: float
    extras: dict = field(default_factory=dict)


def make_instance_device(spec: InstanceSpec, device) -> DeviceInstance:
    """The recipe of make_instance for data blocks too large to draw on the
    host.  The channel, the user powers and the pilot block come from
    PCG64(spec.seed) in make_instance's order (so they equal make_instance's);
    the data block is drawn on `device` by torch's Philox generator seeded
    with spec.seed: symbol indices uniform over the constellation levels,
    the same Rapp PA, powers, channel and noise level, and the pilots' scale.
    The same spec and device type give the same arrays."""
    import torch

    rng = np.random.Generator(np.random.PCG64(spec.seed))
    K, M = spec.K, spec.M
    H = (rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))) / np.sqrt(2.0)
    if spec.near_far_db is not None:
        lo, hi = spec.near_far_db
        p = 10.0 ** (rng.uniform(lo, hi, size=K) / 10.0)
    else:
        p = np.ones(K)
    n0 = 10.0 ** (-spec.snr_db / 10.0)
    b_p, _ = _draw_symbols(rng, spec.P, K, spec.modulation)
    x_p = _rapp(b_p, *spec.rapp) if spec.rapp is not None else b_p
    noise = (rng.standard_normal((spec.P, M)) + 1j * rng.standard_normal((spec.P, M))) * np.sqrt(n0 / 2.0)
    r_p = (x_p * np.sqrt(p)[None, :]) @ H.T + noise
    scale = 1.0 / np.sqrt(np.mean(np.sum(np.abs(r_p) ** 2, axis=1)))
    r_p = r_p * scale

    g = torch.Generator(device=device)
    g.manual_seed(int(spec.seed))
    S = spec.S
    lv = torch.tensor(_LEVELS[spec.modulation], dtype=torch.float32, device=device)
    idx = torch.randint(0, len(_LEVELS[spec.modulation]), (S, K, 2), generator=g, device=device)
    b = torch.complex(lv[idx[..., 0]], lv[idx[..., 1]])
    if spec.rapp is not None:
        pr, a_sat = spec.rapp
        b = b * (1.0 + (b.abs() / a_sat) ** (2.0 * pr)) ** (-1.0 / (2.0 * pr))
    amp = torch.tensor(np.sqrt(p), dtype=torch.float32, device=device)
    Ht = torch.tensor(H.T.copy(), dtype=torch.complex64, device=device).contiguous()   # [K][M]
    r = (b * amp[None, :]) @ Ht
    del b
    nz = torch.randn((S, M, 2), generator=g, device=device) * float(np.sqrt(n0 / 2.0))
    r = (r + torch.complex(nz[..., 0], nz[..., 1])) * float(scale)
    del nz
    rx = torch.cat([r.real, r.imag], dim=-1).contiguous()
    del r
    bits = BITS_PER_AXIS[spec.modulation]
    gray_t = idx ^ (idx >> 1)
    truth = ((gray_t[..., 0] << bits) | gray_t[..., 1]).to(torch.uint8)
    sym_p = np.stack([b_p.real, b_p.imag], axis=-1).astype(np.float32)
    return DeviceInstance(spec=spec, rx_pilot=_to_planar(r_p), sym_pilot=sym_p, rx_data=rx, truth=truth,
                          scale=float(scale), extras={"H": H, "p": p})


def make_drifting_blocks(spec: InstanceSpec, blocks: int, step_rad: float):
    """Pilots on channel H and then `blocks` data blocks of spec.S symbols
    each on a slowly changing channel H_b = cos(b a) H + sin(b a) H2 (a =
    step_rad; H2 an independent draw, so every H_b has the statistics of H).
    Unit powers, no PA model; the pilot block's scale applies throughout.
    Returns (pilot Instance with the block-0 data, list of (rx [S][2M]
    float32, truth [S][K] uint8, sym [S][K][2] float32) per block)."""
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    K, M = spec.K, spec.M
    H = (rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))) / np.sqrt(2.0)
    H2 = (rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))) / np.sqrt(2.0)
    n0 = 10.0 ** (-spec.snr_db / 10.0)

    def block(n, Hb):
        b, idx = _draw_symbols(rng, n, K, spec.modulation)
        noise = (rng.standard_normal((n, M)) + 1j * rng.standard_normal((n, M))) * np.sqrt(n0 / 2.0)
        return b @ Hb.T + noise, b, idx

    r_p, b_p, _ = block(spec.P, H)
    scale = 1.0 / np.sqrt(np.mean(np.sum(np.abs(r_p) ** 2, axis=1)))
    out = []
    for bi in range(blocks):
        Hb = np.cos(bi * step_rad) * H + np.sin(bi * step_rad) * H2
        r, b, idx = block(spec.S, Hb)
        out.append((_to_planar(r * scale), label_of(idx[..., 0], idx[..., 1], spec.modulation),
                    np.stack([b.real, b.imag], axis=-1).astype(np.float32)))
    pil = Instance(spec=spec, rx_pilot=_to_planar(r_p * scale),
                   sym_pilot=np.stack([b_p.real, b_p.imag], axis=-1).astype(np.float32),
                   rx_data=out[0][0], sym_data=out[0][2], truth=out[0][1], scale=float(scale),
                   extras={"H": H, "H2": H2, "n0": n0})
    return pil, out
