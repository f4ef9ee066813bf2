"""GPU parity of the differentiable unrolled training (apsm_unrolled_* through
the C ABI and the autograd binding): the loss against the FP64 reference
forward, the hand-written adjoint against the FP64 reference gradient
(automatic differentiation, itself pinned to finite differences) and against
central finite differences of the FP64 forward, to 1e-3 relative per
component (components below 1e-3 of the largest judged on that floor); checkpoint
interval invariance and repeatability."""
import numpy as np
import pytest

import synth
import paper_2201_05024_amd as A
from oracle import unrolled as U

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"
GRAD_TOL = 1e-3
GRAD_FLOOR = 1e-3


def announce(msg):
    print(f"[case] {msg}", flush=True)


def make(n, K, M, P, S, snr=8.0, seed=500):
    insts = [synth.make_instance(synth.InstanceSpec(K=K, M=M, P=P, S=S, snr_db=snr, seed=seed + i))
             for i in range(n)]
    host = [(i.rx_pilot, i.sym_pilot, i.rx_data, i.sym_data) for i in insts]
    dev = [torch.from_numpy(np.stack([h[q] for h in host])).to(DEV) for q in range(4)]
    return host, dev


def gpu_loss_grad(theta, dev, passes, ckpt, wl=0.5, wg=0.5):
    th = torch.tensor(theta, dtype=torch.float32, device=DEV, requires_grad=True)
    L = A.unrolled_loss(th, *dev, passes=passes, ckpt_every=ckpt, w_lin=wl, w_gauss=wg)
    L.backward()
    torch.cuda.synchronize()
    return float(L.detach()), th.grad.detach().cpu().numpy().astype(np.float64)


def assert_grad_close(g, ref, tol=GRAD_TOL, floor=GRAD_FLOOR):
    """Every component to `tol` relative: |g_i - ref_i| <= tol * max(|ref_i|,
    floor * max_j |ref_j|).  The floor covers components that nearly cancel
    (far below the largest), whose FP32 rounding is set by the size of the
    terms summed into them rather than by their own value."""
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.abs(ref), floor * np.abs(ref).max())
    rel = np.abs(np.asarray(g, dtype=np.float64) - ref) / scale
    print(f"[result] gradient: worst per-component error {rel.max():.2e} at component {int(rel.argmax())} "
          f"(|ref| {abs(ref[rel.argmax()]):.3e}, largest {np.abs(ref).max():.3e})", flush=True)
    assert rel.max() <= tol, (g, ref, rel)


CASES = {
    # name: (n, K, M, P, S, W, passes, ckpt, theta[:3], omega)
    "tiny": (2, 2, 2, 6, 5, 4, 3, 1, [0.7, 0.05, 0.9], [1.0, 0.8, 0.6, 0.5]),
    "k6_m8": (3, 6, 8, 40, 64, 8, 4, 2, [0.8, 0.05, 1.0], list(np.linspace(1.0, 0.3, 8))),
    "k9_wide": (2, 9, 4, 24, 30, 6, 2, 1, [0.6, 0.02, 1.1], [1.0, 1.0, 0.5, 0.5, 0.25, 0.25]),
    "m64": (1, 3, 32, 20, 16, 5, 2, 1, [1.5, 0.05, 0.8], [1.0, 0.9, 0.8, 0.7, 0.6]),
}


@pytest.mark.parametrize("name", list(CASES))
def test_unrolled_gradient_parity(name):
    n, K, M, P, S, W, passes, ckpt, th3, om = CASES[name]
    announce(f"unrolled {name}: n={n} K={K} M={M} P={P} S={S} W={W} passes={passes}")
    host, dev = make(n, K, M, P, S)
    theta = th3 + list(om)
    L, g = gpu_loss_grad(theta, dev, passes, ckpt)
    L_ref, g_ref = U.loss_and_grad(theta, host, passes)
    assert abs(L - L_ref) <= 1e-4 * L_ref, (L, L_ref)
    assert_grad_close(g, g_ref)
    if name == "tiny":
        # central finite differences of the FP64 forward
        h = 1e-6
        g_fd = np.zeros(len(theta))
        for i in range(len(theta)):
            tp, tm = list(theta), list(theta)
            tp[i] += h
            tm[i] -= h
            g_fd[i] = (U.loss_only(tp, host, passes) - U.loss_only(tm, host, passes)) / (2 * h)
        assert_grad_close(g, g_fd)
    print(f"[result] {name}: L {L:.6g} (ref {L_ref:.6g}), max grad err "
          f"{np.abs(g - g_ref).max() / np.abs(g_ref).max():.2e}", flush=True)


def test_unrolled_checkpoint_interval_does_not_change_results():
    host, dev = make(2, 4, 8, 30, 40, seed=600)
    theta = [0.8, 0.05, 1.0] + list(np.linspace(1.0, 0.5, 6))
    outs = [gpu_loss_grad(theta, dev, passes=5, ckpt=c) for c in (1, 2, 5)]
    for L, g in outs[1:]:
        assert L == outs[0][0]
        np.testing.assert_array_equal(g, outs[0][1])


def test_unrolled_backward_repeatable_and_scaled_by_upstream():
    host, dev = make(2, 3, 4, 20, 20, seed=700)
    th = torch.tensor([0.7, 0.05, 1.0, 1.0, 0.5, 0.25], dtype=torch.float32, device=DEV, requires_grad=True)
    L = A.unrolled_loss(th, *dev, passes=3, ckpt_every=2)
    (g1,) = torch.autograd.grad(L, th, retain_graph=True)
    (g2,) = torch.autograd.grad(L, th, retain_graph=True)
    (g3,) = torch.autograd.grad(3.0 * L, th)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    torch.testing.assert_close(g3, 3.0 * g1, rtol=1e-6, atol=0)


def test_unrolled_full_size_one_instance():
    """Per-instance size of the differentiable workload (K = 6, 16 antennas,
    512 pilots, 4096 validation symbols, W = 32, 20 passes, checkpoint every
    5): loss and gradient of one instance against the FP64 reference."""
    announce("unrolled full size, one instance")
    host, dev = make(1, 6, 16, 512, 4096, snr=10.0, seed=800)
    theta = [0.7, 0.05, 1.0] + [1.0] * 32
    L, g = gpu_loss_grad(theta, dev, passes=20, ckpt=5)
    print("[step] gpu done", flush=True)
    L_ref, g_ref = U.loss_and_grad(theta, host, 20)
    assert abs(L - L_ref) <= 1e-4 * L_ref, (L, L_ref)
    assert_grad_close(g, g_ref)
    print(f"[result] full size: L {L:.6g}, max grad err {np.abs(g - g_ref).max() / np.abs(g_ref).max():.2e}",
          flush=True)


def test_unrolled_full_batch_checkpoint_invariance():
    """64 instances at full size: the gradient with checkpoints every 5 passes
    equals the one with a single segment, bit for bit, and is finite."""
    announce("unrolled full batch, 64 instances")
    host, dev = make(64, 6, 16, 512, 4096, snr=10.0, seed=900)
    theta = [0.7, 0.05, 1.0] + [1.0] * 32
    L5, g5 = gpu_loss_grad(theta, dev, passes=20, ckpt=5)
    L20, g20 = gpu_loss_grad(theta, dev, passes=20, ckpt=20)
    assert np.all(np.isfinite(g5)) and np.isfinite(L5)
    assert L5 == L20
    np.testing.assert_array_equal(g5, g20)
