"""Benchmark of the APSM detector hot path on one MI355X.

Headline workload (the largest single-GPU configuration): the large array,
batched.  16 detector instances, each with 16 users (16-QAM, Rapp PA p = 2,
A_sat = 1, 20 dB) received on 64 antennas (2M = 128), 8192 pilot symbols
(16,384 real training steps, window 32, dictionary capacity 8192) and
4,194,304 data symbols.  One step trains the 16 detectors (kernel rows in one
launch, training in one launch, packing) and detects all 16 x 4,194,304
received vectors with decisions and symbol-error counts (one launch, a
workgroup per 128 received vectors).  Steps are pipelined over two model sets on two streams (the
training of step k runs beside the detection of step k - 1); every step still
trains 16 detectors and detects 16 frames.  Inputs are synthetic (seeded),
generated on the device, and resident in HBM before the timed region.

Further workloads in the same JSON line: the realistic slot (4 SNR points of
one 6-user, 16-antenna slot with 1,048,576 symbols), the batched mixed-shape
workload (256 detectors; serialized, graph replay and pipelined as the
headline), the differentiable unrolled training (64
instances, forward + backward), the small plain case (per-call latency) and
the paper's own shape (detection latency, context for its Table).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = ("detected symbols/s and kernel evals/s vs roofline at oracle SER; "
          "batched vs plain")
# Dense FP16 matrix-core peak of the MI355X: 256 CUs x 4096 flops/clock x 2.4 GHz.
PEAK_FP16_MFMA_TFLOPS = 256 * 4096 * 2.4e9 / 1e12               # 2516.6
# FP32 vector peak: 256 CUs x 4 SIMDs x 32 lanes x 2 flops (FMA) x 2.4 GHz.
PEAK_FP32_VALU_TFLOPS = 256 * 4 * 32 * 2 * 2.4e9 / 1e12         # 157.3


def detection_roofline(kernel, det_s, vectors, D, M2, K, M2P):
    """Roofline of one two-contraction detection launch over `vectors` real
    vectors against D dictionary entries each.  `achieved` counts the
    method's algorithmic flops, D (2 2M + 3 + 2K) + 2 2M (K + 1) per real
    vector (distance block, norm combine, coefficients, linear part), over
    the FP16 matrix-core peak, the type the contractions execute in.  The
    split-FP16 formulation executes three FP16 products per FP32 product, on
    operands padded to 2M -> M2P and K -> 16: those executed flops, their
    fraction of the same peak, the algorithmic rate as a multiple of the FP32
    peak (the bound of any FP32 formulation) and the VALU flop-equivalents
    per evaluation (exponent FMA 2, exp2 8, hi/lo split 6) are reported
    beside it."""
    evals = vectors * D
    alg = vectors * (D * (2 * M2 + 3 + 2 * K) + 2 * M2 * (K + 1))
    executed = evals * 6 * (M2P + 16) + vectors * 6 * M2P * 16
    achieved = alg / det_s / 1e12
    return {
        "kernel": kernel, "bound": "mfma", "achieved": achieved, "peak": PEAK_FP16_MFMA_TFLOPS,
        "unit": "TFLOP/s", "frac": achieved / PEAK_FP16_MFMA_TFLOPS,
        "per_launch": {
            "real_vectors": vectors, "kernel_evals": evals, "algorithmic_flops": alg,
            "algorithmic_flops_per_real_vector": alg / vectors, "avg_ms": det_s * 1e3,
            "executed_fp16_mfma_flops": executed,
            "executed_fp16_mfma_frac": executed / det_s / 1e12 / PEAK_FP16_MFMA_TFLOPS,
            "algorithmic_rate_over_fp32_peak": achieved / PEAK_FP32_VALU_TFLOPS,
            "valu_frac_of_fp32_peak": evals * 16 / det_s / 1e12 / PEAK_FP32_VALU_TFLOPS,
        },
    }

# HBM bytes per launch of the batched two-contraction detection kernel on the
# headline workload, from rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by a
# plain device copy (profiles/).  Valid only for the sources they were taken
# with; reported as null otherwise.
MEASURED_TRAFFIC = {
    # FETCH_SIZE + WRITE_SIZE of detect_wide_batch_kernel<128> per dispatch,
    # both x1.000 by the 256 MiB copy of the same runs
    # (profiles/detect_wide_large_array_counters.md)
    "bytes": int((57266160.2 * 1.0 + 14680064.2 * 1.0) * 1024),
    "sources": {"paper_2201_05024_amd/csrc/detect_wide.h": "c4466cec43db01aaded2f9d1e5d12b7c8ce86ff1",
                "paper_2201_05024_amd/csrc/detect_wide.hip": "8ed459dc5ba8dc9f93072750609e6a1b67afc71f"},
}


def measured_traffic():
    import hashlib
    if MEASURED_TRAFFIC["bytes"] is None:
        return None
    root = os.path.dirname(os.path.abspath(__file__))
    for rel, digest in MEASURED_TRAFFIC["sources"].items():
        try:
            with open(os.path.join(root, rel), "rb") as fh:
                if hashlib.sha1(fh.read()).hexdigest() != digest:
                    return None
        except OSError:
            return None
    return MEASURED_TRAFFIC["bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle timings")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the large-array workload (profiling runs); same as --extra ''")
    ap.add_argument("--extra", default="slot,mixed,unrolled,small",
                    help="comma list of the further workloads after the headline: "
                         "slot, mixed, unrolled, small (default: all)")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-detector forms")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (HBM counter calibration)")
    return ap.parse_args()


def cuda_events(n=2):
    import torch
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    except Exception:  # pragma: no cover
        return 1


def best_of(fn, reps=3):
    best = None
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return best


# ------------------------------------------------------------------ headline

def oracle_built_model(inst, cap, K, seed):
    """A full-capacity filter for the large-array shape built without
    training (training it in FP64 takes about an hour): the dictionary is the
    newest `cap` real training vectors of the pilots (what a capacity-`cap`
    training leaves), coefficients and linear weights are seeded draws."""
    import oracle as O
    import synth
    R, _ = O.training_sequence(synth.planar_to_complex(inst.rx_pilot), synth.pair_to_complex(inst.sym_pilot))
    rng = np.random.default_rng(seed)
    d = R[-cap:].astype(np.float32)
    alpha = (rng.standard_normal((cap, K)) * 0.05).astype(np.float32)
    w = (rng.standard_normal((K, R.shape[1])) * 0.05).astype(np.float32)
    return d, alpha, w


def run_large(args, dev, s_train, s_det):
    import torch
    import oracle as O
    import synth
    import paper_2201_05024_amd as A

    n = synth.LARGE_INSTANCES
    specs = [synth.spec_large(i) for i in range(n)]
    sp0 = specs[0]
    K, M2, P, S, cap, W = sp0.K, 2 * sp0.M, sp0.P, sp0.S, 8192, 32
    params = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=W, w_lin=0.5, w_gauss=0.5, dict_cap=cap)
    log(f"[bench] large array: generating {n} instances on the device")
    insts = [synth.make_instance_device(sp, dev) for sp in specs]
    rx_p = [torch.from_numpy(i.rx_pilot).to(dev) for i in insts]
    sym_p = [torch.from_numpy(i.sym_pilot).to(dev) for i in insts]
    soft = [torch.empty((S, K, 2), dtype=torch.float32, device=dev) for _ in insts]
    hard = [torch.empty((S, K), dtype=torch.uint8, device=dev) for _ in insts]
    errs = [torch.zeros(K, dtype=torch.int64, device=dev) for _ in insts]
    # two model sets, one batch each; both detect into the same outputs
    # (their detections are ordered on one stream)
    models = [[A.Model(M2, K, cap, dev, params.sigma2) for _ in insts] for _ in range(2)]
    batches = [A.Batch(params, [A.BatchItem(model=ms[i], rx_pilot=rx_p[i], sym_pilot=sym_p[i], rx=insts[i].rx_data,
                                            modulation="qam16", soft=soft[i], hard=hard[i], truth=insts[i].truth,
                                            errors=errs[i]) for i in range(n)]) for ms in models]
    # one workgroup per work item: the trainings on the other stream get CUs
    # as detection workgroups retire
    for b in batches:
        b.set_form(False)
    trained = [torch.cuda.Event(), torch.cuda.Event()]
    detected = [torch.cuda.Event(), torch.cuda.Event()]
    rows_ready = [torch.cuda.Event(), torch.cuda.Event()]
    det_events = []

    def detect_set(k, record):
        for e in errs:
            e.zero_()
        if record:
            e0, e1 = cuda_events()
            e0.record(s_det)
        batches[k].detect(s_det)
        if record:
            e1.record(s_det)
            det_events.append((e0, e1))

    def step(k, record):
        cur, prev = k % 2, (k + 1) % 2
        with torch.cuda.stream(s_det):
            batches[cur].kernel_rows(s_det)
            rows_ready[cur].record(s_det)
        with torch.cuda.stream(s_train):
            s_train.wait_event(detected[cur])
            s_train.wait_event(rows_ready[cur])
            batches[cur].train_prepared(s_train)
            trained[cur].record(s_train)
        with torch.cuda.stream(s_det):
            s_det.wait_event(trained[prev])
            detect_set(prev, record)
            detected[prev].record(s_det)

    torch.cuda.synchronize()
    log(f"[bench] large array: warmup {args.warmup}")
    with torch.cuda.stream(s_train):
        batches[1].train(s_train)
        trained[1].record(s_train)
    for k in range(args.warmup):
        step(k, False)
    torch.cuda.synchronize()
    # parts alone, for the report
    ev = cuda_events(4)
    ev[0].record(s_det)
    batches[0].kernel_rows(s_det)
    ev[1].record(s_det)
    batches[0].train_prepared(s_det)
    ev[2].record(s_det)
    detect_set(0, False)
    ev[3].record(s_det)
    torch.cuda.synchronize()
    rows_ms, train_ms, det1_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])
    serial_ms = ev[0].elapsed_time(ev[3])
    # re-arm the pipeline: set 1 trained, set 0 free
    with torch.cuda.stream(s_train):
        batches[1].train(s_train)
        trained[1].record(s_train)
    with torch.cuda.stream(s_det):
        detected[0].record(s_det)
    torch.cuda.synchronize()

    log(f"[bench] large array: timing {args.steps} steps")
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k, True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log("[bench] large array: timed region done")
    ser_gpu = float(sum(e.sum().item() for e in errs)) / (n * S * K)

    det_ms = [a.elapsed_time(b) for a, b in det_events]
    det_s = float(np.mean(det_ms)) / 1e3
    evals = n * 2 * S * cap                                     # (real vector, entry) pairs per launch
    roof = detection_roofline("detect_wide_batch_kernel<128>", det_s, n * 2 * S, cap, M2, K, 128)
    roof["traffic"] = measured_traffic()
    roof["per_launch"]["launches_timed"] = len(det_ms)

    out = {
        "value": n * S * K / (elapsed / args.steps),
        "ms_per_step": elapsed / args.steps * 1e3,
        "config": {
            "workload": ("large array, batched: 16 instances x (K=16 users 16-QAM, 64 Rx antennas (2M=128), "
                         "Rapp PA p=2 A_sat=1, 20 dB, 8192 pilots, 4194304 data symbols, W=32, sigma2=0.5, "
                         "eps=0.05, mu=1, dictionary cap 8192); one step trains and detects all 16"),
            "instances_per_step": n, "data_symbols": S, "pilots": P, "users": K, "antennas": M2 // 2,
        },
        "roofline": roof,
        "detect_only": {"user_symbols_per_s": n * S * K / det_s, "kernel_evals_per_s": evals / det_s,
                        "ms_one_launch_16_instances": det_s * 1e3},
        "train_ms_16_instances": {"kernel_rows": rows_ms, "training_and_packing": train_ms},
        "ms_per_step_serialized": serial_ms,
        "detect_ms_serialized_run": det1_ms,
        "schedule": ("pipelined: the kernel rows of step k (one launch) precede the detection launch on the "
                     "detection stream; the training of step k (one launch, 64 four-user jobs) runs beside the "
                     "detection of step k-1 (one launch over all 16 instances, one workgroup per 128 received "
                     "vectors) on a second stream"),
        "ser_gpu": ser_gpu,
    }

    # detection-only parity on the headline's data and launch form: a
    # full-capacity filter built from the pilots (no training) detects
    # instance 0's 4,194,304 vectors; the oracle evaluates a spread sample
    log("[bench] large array: detection parity sample")
    d, alpha, w = oracle_built_model(insts[0], cap, K, seed=55)
    pm = A.Model(M2, K, cap, dev, 0.5)
    pm.dict.copy_(torch.from_numpy(np.ascontiguousarray(d.T)).to(dev))
    pm.alpha.copy_(torch.from_numpy(alpha).to(dev))
    pm.w.copy_(torch.from_numpy(w).to(dev))
    pm.state.copy_(torch.tensor([cap, 0, 2 * P, 0], dtype=torch.int32, device=dev))
    pm.pack()
    po = A.detect(pm, insts[0].rx_data, modulation="qam16", truth=insts[0].truth)
    torch.cuda.synchronize()
    idx = np.unique(np.r_[0:32, np.arange(0, S, 16384), S - 32:S])
    f = O.Filter(K, M2, 0.5)
    f.w, f.dict_vec, f.alpha = w.astype(np.float64), d.astype(np.float64), alpha.astype(np.float64)
    f.dict_idx = list(range(cap))
    rx_sub = insts[0].rx_data[torch.from_numpy(idx).to(dev)].cpu().numpy()
    soft_ref = O.detect_planar(f, rx_sub, chunk=8)
    soft_gpu = po["soft"].cpu().numpy()[idx].astype(np.float64)
    a_min = 1 / np.sqrt(10)
    scaled = np.abs(soft_gpu - soft_ref) / np.maximum(np.abs(soft_ref), a_min)
    lab_ref = O.decide(soft_ref, "qam16")
    near = O.boundary_distance(soft_ref, "qam16") < 1e-5
    hard_gpu = po["hard"].cpu().numpy()[idx]
    truth_sub = insts[0].truth.cpu().numpy()[idx]
    diff = hard_gpu != lab_ref
    out["parity_sample"] = {
        "what": ("detection only, instance 0 of the headline data (4194304 vectors, one launch) with a "
                 "full-capacity filter built from its pilots; oracle on the first and last 32 and every "
                 f"16384th symbol ({len(idx)} symbols x 16 users)"),
        "max_scaled_error": float(scaled.max()),
        "decision_mismatch_outside_band": int(np.sum(diff & ~near)),
        "decision_mismatch_inside_band": int(np.sum(diff & near)),
        "ser_gpu_sample": float(np.mean(hard_gpu != truth_sub)),
        "ser_oracle_sample": float(np.mean(lab_ref != truth_sub)),
    }

    if not args.no_plain:
        log("[bench] large array: plain form (one launch per detector)")
        pmodels = models[0]

        def plain_detect():
            for i in range(n):
                A.detect(pmodels[i], insts[i].rx_data, modulation="qam16", truth=insts[i].truth,
                         soft=soft[i], hard=hard[i], errors=errs[i], stream=s_det)

        with torch.cuda.stream(s_det):
            plain_detect()
            torch.cuda.synchronize()
            e = cuda_events()
            e[0].record(s_det)
            plain_detect()
            e[1].record(s_det)
            torch.cuda.synchronize()
            plain_det_ms = e[0].elapsed_time(e[1])
            e = cuda_events()
            e[0].record(s_det)
            for i in range(n):
                A.train(rx_p[i], sym_p[i], params, model=pmodels[i], stream=s_det)
            e[1].record(s_det)
            torch.cuda.synchronize()
            plain_train_ms = e[0].elapsed_time(e[1])
        plain_step_ms = plain_det_ms + plain_train_ms
        out["plain"] = {
            "what": "16 apsm_train launches then 16 apsm_detect launches, one detector each, on one stream",
            "ms_per_step": plain_step_ms, "train_ms": plain_train_ms, "detect_ms": plain_det_ms,
            "user_symbols_per_s": n * S * K / (plain_step_ms / 1e3),
            "speedup_batched_vs_plain": plain_step_ms / out["ms_per_step"],
            "detect_speedup_batched_vs_plain": plain_det_ms / (det_s * 1e3),
        }

    if not args.no_cpu_baseline:
        log("[bench] large array: timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline_large(insts[0], d, alpha, w, params, n, S, P, cap, W)
    return out


def cpu_baseline_large(inst, d, alpha, w, params, n, S, P, cap, W):
    """The FP64 oracle (best of 3) on a bounded sample of the headline
    workload: detection of 64 symbols and 6 training steps with a full
    8192-entry dictionary, scaled to one step (16 trainings of 16384 steps,
    16 x 4194304 detected symbols)."""
    import oracle as O
    K, M2 = alpha.shape[1], d.shape[1]
    steps = 6
    f = O.Filter(K, M2, params.sigma2)
    f.w, f.dict_vec, f.alpha = w.astype(np.float64), d.astype(np.float64), alpha.astype(np.float64)
    # the entries of the steps before the timed ones
    f.dict_idx = list(range(2 * P - steps - cap, 2 * P - steps))
    rx = inst.rx_data[:64].cpu().numpy()
    t_det = best_of(lambda: O.symbol_errors(O.decide(O.detect_planar(f, rx, chunk=8), "qam16"),
                                            inst.truth[:64].cpu().numpy()))
    rng = np.random.default_rng(1)
    Rt = rng.standard_normal((2 * P, M2)) * 0.09
    Bt = rng.standard_normal((2 * P, K)) * 0.5
    p = O.APSMParams(sigma2=params.sigma2, eps=params.eps, mu=params.mu, window=W, w_lin=params.w_lin,
                     w_gauss=params.w_gauss, dict_cap=cap)

    def train_steps():
        tr = O.Trainer(Rt, Bt, p, f0=f)
        tr.n = 2 * P - steps                  # the last steps: full dictionary and window
        for _ in range(steps):
            tr.step()

    t_steps = best_of(train_steps)
    # cost of a step is proportional to |J_n| D_n; the timed steps had W and cap
    units = sum(min(k + 1, W) * min(k + 1, cap) for k in range(2 * P)) / (W * cap)
    t_train = t_steps / steps * units
    t_inst = t_train + t_det / 64 * S
    return {
        "value": S * 16 / t_inst,
        "unit": "user-symbols/s",
        "cores": blas_threads(),
        "kind": "oracle",
        "sample": (f"FP64 oracle (numpy, {blas_threads()} BLAS threads of {os.cpu_count()} host cores), best of 3: "
                   f"detection of 64 of 4194304 symbols with a full 8192-entry dictionary ({t_det:.2f} s) and "
                   f"{steps} training steps with full dictionary and window ({t_steps:.2f} s), scaled to one "
                   f"instance (2P = {2 * P} steps weighted by |J_n| D_n: {t_train:.0f} s training, "
                   f"{t_det / 64 * S:.0f} s detection); value = one instance's symbols over its time "
                   f"(the {n} instances of a step take {n} times as long)"),
    }


# ------------------------------------------------------- realistic slot (C2)

def run_slot(args, dev, s_train, s_det):
    import torch
    import oracle as O
    import synth
    import paper_2201_05024_amd as A

    snrs = synth.SLOT_SNRS_DB
    params = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=32, w_lin=0.5, w_gauss=0.5, dict_cap=1024)
    log(f"[bench] slot: generating {len(snrs)} instances")
    insts = [synth.make_instance(synth.spec_slot(s)) for s in snrs]
    K, M2, P, S = insts[0].spec.K, 2 * insts[0].spec.M, insts[0].spec.P, insts[0].spec.S
    cu = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    rx_p = [cu(i.rx_pilot) for i in insts]
    sym_p = [cu(i.sym_pilot) for i in insts]
    rx_d = [cu(i.rx_data) for i in insts]
    truth = [cu(i.truth) for i in insts]
    soft = [torch.empty((S, K, 2), dtype=torch.float32, device=dev) for _ in insts]
    hard = [torch.empty((S, K), dtype=torch.uint8, device=dev) for _ in insts]
    errs = [torch.zeros(K, dtype=torch.int64, device=dev) for _ in insts]
    models = [[A.Model(M2, K, params.dict_cap, dev, params.sigma2) for _ in insts] for _ in range(2)]
    batches = [A.Batch(params, [A.BatchItem(model=ms[i], rx_pilot=rx_p[i], sym_pilot=sym_p[i], rx=rx_d[i],
                                            modulation="qpsk", soft=soft[i], hard=hard[i], truth=truth[i],
                                            errors=errs[i]) for i in range(len(insts))]) for ms in models]
    # persistent detection on all CUs but the four the trainings of the next
    # step occupy (one workgroup per detector)
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    for b in batches:
        b.set_form(True, cus - len(insts))
    trained = [torch.cuda.Event(), torch.cuda.Event()]
    detected = [torch.cuda.Event(), torch.cuda.Event()]
    rows_ready = [torch.cuda.Event(), torch.cuda.Event()]
    det_events = []

    def detect_set(k, record):
        for e in errs:
            e.zero_()
        if record:
            e0, e1 = cuda_events()
            e0.record(s_det)
        batches[k].detect(s_det)
        if record:
            e1.record(s_det)
            det_events.append((e0, e1))

    def step(k, record):
        cur, prev = k % 2, (k + 1) % 2
        with torch.cuda.stream(s_det):
            batches[cur].kernel_rows(s_det)
            rows_ready[cur].record(s_det)
        with torch.cuda.stream(s_train):
            s_train.wait_event(detected[cur])
            s_train.wait_event(rows_ready[cur])
            batches[cur].train_prepared(s_train)
            trained[cur].record(s_train)
        with torch.cuda.stream(s_det):
            s_det.wait_event(trained[prev])
            detect_set(prev, record)
            detected[prev].record(s_det)

    torch.cuda.synchronize()
    with torch.cuda.stream(s_train):
        batches[1].train(s_train)
        trained[1].record(s_train)
    for k in range(3):
        step(k, False)
    torch.cuda.synchronize()
    ev = cuda_events(3)
    ev[0].record(s_det)
    batches[0].train(s_det)
    ev[1].record(s_det)
    detect_set(0, False)
    ev[2].record(s_det)
    torch.cuda.synchronize()
    train_ms, serial_ms = ev[0].elapsed_time(ev[1]), ev[0].elapsed_time(ev[2])
    with torch.cuda.stream(s_train):
        batches[1].train(s_train)
        trained[1].record(s_train)
    with torch.cuda.stream(s_det):
        detected[0].record(s_det)
    torch.cuda.synchronize()
    steps = 20
    t0 = time.perf_counter()
    for k in range(steps):
        step(k, True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    det_s = float(np.mean([a.elapsed_time(b) for a, b in det_events])) / 1e3
    n = len(insts)
    evals = n * 2 * S * params.dict_cap
    ser = {f"{s:g}dB": float(e.sum().item()) / (S * K) for s, e in zip(snrs, errs)}
    out = {
        "workload": ("realistic slot: K=6 users QPSK, 16 Rx antennas (2M=32), near-far [-6,0] dB, Rapp PA p=2 "
                     "A_sat=1, SNR 5/10/15/20 dB (4 instances), 1024 pilots, 1048576 data symbols, W=32, "
                     "sigma2=0.5, eps=0.05, mu=1, dictionary cap 1024; pipelined as the headline"),
        "user_symbols_per_s": n * S * K / (elapsed / steps),
        "ms_per_step": elapsed / steps * 1e3,
        "ms_per_step_serialized": serial_ms,
        "train_ms_4_instances": train_ms,
        "detect_ms_one_launch_4_instances": det_s * 1e3,
        "kernel_evals_per_s": evals / det_s,
        "roofline": detection_roofline("detect_wide_batch_kernel<32>", det_s, n * 2 * S, params.dict_cap,
                                       M2, K, 32),
        "ser_gpu": ser,
    }
    if not args.no_cpu_baseline:
        # the oracle trains the 10 dB instance itself and detects a sample:
        # its SER and decision mismatches against the GPU's on those symbols,
        # and its time (best of 3 for detection) scaled to the step
        log("[bench] slot: oracle training and sampled detection")
        i10 = snrs.index(10.0)
        inst = insts[i10]
        p = O.APSMParams(sigma2=0.5, eps=0.05, mu=1.0, window=32, dict_cap=1024)
        t0 = time.perf_counter()
        f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, p)
        t_train = time.perf_counter() - t0
        rng = np.random.default_rng(7)
        idx = np.unique(np.r_[0:256, S - 256:S, rng.integers(0, S, 1536)])
        soft_ref = [None]

        def det():
            soft_ref[0] = O.detect_planar(f, inst.rx_data[idx])
        t_det = best_of(det)
        sr = soft_ref[0]
        lab_ref = O.decide(sr, "qpsk")
        near = O.boundary_distance(sr, "qpsk") < 1e-5
        # the detection of the timed region's last step used the last trained set
        hard_gpu = hard[i10].cpu().numpy()[idx]
        soft_gpu = soft[i10].cpu().numpy()[idx].astype(np.float64)
        diff = hard_gpu != lab_ref
        t_step = n * (t_train + t_det / len(idx) * S)
        out["oracle_sample"] = {
            "what": f"the oracle's own training of the 10 dB instance and detection of {len(idx)} symbols",
            "max_scaled_error": float(np.max(np.abs(soft_gpu - sr) / np.maximum(np.abs(sr), 1 / np.sqrt(2)))),
            "decision_mismatch_outside_band": int(np.sum(diff & ~near)),
            "decision_mismatch_inside_band": int(np.sum(diff & near)),
            "ser_gpu_sample": float(np.mean(hard_gpu != inst.truth[idx])),
            "ser_oracle_sample": float(np.mean(lab_ref != inst.truth[idx])),
        }
        out["cpu_baseline"] = {
            "value": n * S * K / t_step, "unit": "user-symbols/s", "cores": blas_threads(), "kind": "oracle",
            "sample": (f"FP64 oracle ({blas_threads()} BLAS threads of {os.cpu_count()} host cores): full training "
                       f"of the 10 dB instance ({t_train:.2f} s) and detection of {len(idx)} of {S} symbols "
                       f"(best of 3, {t_det:.2f} s), extrapolated linearly to {n} instances x {S} symbols"),
        }
    return out


# ---------------------------------------------------- batched mixed shapes (C3)

def run_batched_mixed(args, dev, s_train, s_det):
    import torch
    import synth
    import paper_2201_05024_amd as A

    n = synth.BATCH_INSTANCES
    log(f"[bench] mixed batch: generating {n} detectors")
    params = A.Params(eps=0.05, mu=1.0, window=32)
    items, evals, syms = [], 0, 0
    cu = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    # every detector's error counts are a view of one tensor, cleared at once
    shapes = [synth.spec_batch_mixed(i) for i in range(n)]
    errs_all = torch.zeros(sum(sp.K for sp, _ in shapes), dtype=torch.int64, device=dev)
    off = 0
    for i in range(n):
        spec, D = shapes[i]
        inst = synth.make_instance(spec)
        K, M2, S = spec.K, 2 * spec.M, spec.S
        items.append(A.BatchItem(
            model=A.Model(M2, K, D, dev, 0.5), rx_pilot=cu(inst.rx_pilot), sym_pilot=cu(inst.sym_pilot),
            rx=cu(inst.rx_data), modulation=spec.modulation,
            soft=torch.empty((S, K, 2), dtype=torch.float32, device=dev),
            hard=torch.empty((S, K), dtype=torch.uint8, device=dev), truth=cu(inst.truth),
            errors=errs_all[off:off + K], sigma2=0.5))
        off += K
        evals += 2 * S * D
        syms += S * K
    batch = A.Batch(params, items)
    stream = torch.cuda.current_stream()
    batch.train(stream).detect(stream)
    batch.tune(stream)
    torch.cuda.synchronize()

    def batched_step():
        errs_all.zero_()
        batch.train(stream).detect(stream)

    def timed(fn, steps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    t_batched = timed(batched_step, 5)
    # the same step captured once in a HIP graph and replayed
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        errs_all.zero_()
        batch.train(side).detect(side)
    torch.cuda.synchronize()
    t_graph = timed(g.replay, 5)
    ev = []
    for _ in range(5):
        e = cuda_events()
        e[0].record(stream)
        batch.detect(stream)
        e[1].record(stream)
        ev.append(e)
    e = cuda_events()
    e[0].record(stream)
    batch.train(stream)
    e[1].record(stream)
    torch.cuda.synchronize()
    det_s = float(np.mean([a.elapsed_time(b) for a, b in ev])) / 1e3

    # Pipelined as the headline: a second model set detecting into the same
    # outputs; the kernel rows of step k and the detection of step k - 1 on
    # one stream, the training of step k on the other.  Plain-form detection,
    # so the trainings get CUs as detection workgroups retire.
    items2 = [A.BatchItem(model=A.Model(it.model.M2, it.model.K, it.model.dict_cap, dev, 0.5),
                          rx_pilot=it.rx_pilot, sym_pilot=it.sym_pilot, rx=it.rx, modulation=it.modulation,
                          soft=it.soft, hard=it.hard, truth=it.truth, errors=it.errors, sigma2=0.5)
              for it in items]
    sets = [batch, A.Batch(params, items2)]
    for b in sets:
        b.set_form(False)
    trained = [torch.cuda.Event(), torch.cuda.Event()]
    detected = [torch.cuda.Event(), torch.cuda.Event()]
    rows_ready = [torch.cuda.Event(), torch.cuda.Event()]

    def pipelined_step(k):
        cur, prev = k % 2, (k + 1) % 2
        with torch.cuda.stream(s_det):
            sets[cur].kernel_rows(s_det)
            rows_ready[cur].record(s_det)
        with torch.cuda.stream(s_train):
            s_train.wait_event(detected[cur])
            s_train.wait_event(rows_ready[cur])
            sets[cur].train_prepared(s_train)
            trained[cur].record(s_train)
        with torch.cuda.stream(s_det):
            s_det.wait_event(trained[prev])
            errs_all.zero_()
            sets[prev].detect(s_det)
            detected[prev].record(s_det)

    torch.cuda.synchronize()
    with torch.cuda.stream(s_train):
        sets[1].train(s_train)
        trained[1].record(s_train)
    with torch.cuda.stream(s_det):
        detected[0].record(s_det)
    for k in range(2):
        pipelined_step(k)
    torch.cuda.synchronize()
    steps = max(args.steps, 5)
    t0 = time.perf_counter()
    for k in range(steps):
        pipelined_step(k)
    torch.cuda.synchronize()
    t_pipe = (time.perf_counter() - t0) / steps
    for b in sets[1:]:
        b.close()

    out = {
        "workload": (f"{n} detectors, K 2..8, 8/16/32 antennas, dictionaries 64..2048 (= pilots), "
                     "65536 vectors each, QPSK/16-QAM mixed, SNR 5..20 dB, W=32, sigma2=0.5"),
        "batched_user_symbols_per_s": syms / t_batched,
        "ms_per_step_batched": t_batched * 1e3,
        "pipelined_user_symbols_per_s": syms / t_pipe,
        "ms_per_step_pipelined": t_pipe * 1e3,
        "schedule_pipelined": ("training of step k (kernel rows, then one training launch) beside the "
                               "plain-form detection of step k - 1 on a second stream, two model sets"),
        "graph_replay_ms": t_graph * 1e3,
        "train_ms_one_batch": e[0].elapsed_time(e[1]),
        "detect_ms_one_batch": det_s * 1e3,
        "kernel_evals_per_s": evals / det_s,
    }
    if not args.no_plain:
        def plain_detect():
            for it in items:
                A.detect(it.model, it.rx, modulation=it.modulation, truth=it.truth, soft=it.soft, hard=it.hard,
                         errors=it.errors, stream=stream)

        def plain_step():
            errs_all.zero_()
            for it in items:
                p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=32, dict_cap=it.model.dict_cap)
                A.train(it.rx_pilot, it.sym_pilot, p, model=it.model, stream=stream)
            plain_detect()
        t_plain = timed(plain_step, 1)
        t_plain_det = timed(plain_detect, 2)
        out.update({
            "plain_user_symbols_per_s": syms / t_plain,
            "ms_per_step_plain": t_plain * 1e3,
            "speedup_vs_plain": t_plain / t_batched,
            "pipelined_speedup_vs_plain": t_plain / t_pipe,
            "detect_ms_plain": t_plain_det * 1e3,
            "detect_speedup_vs_plain": t_plain_det / det_s,
        })
    return out


# ------------------------------------------------ differentiable training (C4)

def run_unrolled(dev):
    import torch
    import synth
    import paper_2201_05024_amd as A

    n, K, M, P, S, W = 64, 6, 16, 512, 4096, 32
    log(f"[bench] unrolled: {n} instances")
    insts = [synth.make_instance(synth.InstanceSpec(K=K, M=M, P=P, S=S, snr_db=10.0, seed=900 + i))
             for i in range(n)]
    data = [torch.from_numpy(np.stack([getattr(i, a) for i in insts])).to(dev)
            for a in ("rx_pilot", "sym_pilot", "rx_data", "sym_data")]
    theta = torch.tensor([0.7, 0.05, 1.0] + [1.0] * W, dtype=torch.float32, device=dev, requires_grad=True)

    def fwd_bwd():
        theta.grad = None
        L = A.unrolled_loss(theta, *data, passes=20, ckpt_every=5)
        L.backward()
        return L

    fwd_bwd()
    torch.cuda.synchronize()
    e = cuda_events(3)
    e[0].record()
    L = A.unrolled_loss(theta, *data, passes=20, ckpt_every=5)
    e[1].record()
    L.backward()
    e[2].record()
    torch.cuda.synchronize()
    return {"workload": ("differentiable unrolled training: 64 instances x (K=6, 16 antennas, 512 pilots, 4096 "
                         "validation symbols), W=32, 20 passes, checkpoint every 5; gradient w.r.t. sigma, eps, "
                         "mu and 32 position weights"),
            "forward_ms": e[0].elapsed_time(e[1]), "backward_ms": e[1].elapsed_time(e[2]),
            "forward_backward_ms": e[0].elapsed_time(e[2]), "loss": float(L.detach())}


# ---------------------------------------- small plain case (C1), paper shape (P0)

def run_small(dev):
    import torch
    import synth
    import paper_2201_05024_amd as A

    cu = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    out = {}
    inst = synth.make_instance(synth.spec_plain_small())
    p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=16, dict_cap=256)
    rxp, symp, rx, truth = cu(inst.rx_pilot), cu(inst.sym_pilot), cu(inst.rx_data), cu(inst.truth)
    m = A.train(rxp, symp, p)
    o = A.detect(m, rx, truth=truth)
    b = A.Batch(p, [A.BatchItem(model=A.Model(16, 4, 256, dev, 0.5), rx_pilot=rxp, sym_pilot=symp, rx=rx,
                                soft=torch.empty_like(o["soft"]), hard=torch.empty_like(o["hard"]), truth=truth,
                                errors=torch.zeros(4, dtype=torch.int64, device=dev))])
    b.train().detect()
    torch.cuda.synchronize()

    def lat(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        e = cuda_events()
        e[0].record()
        for _ in range(reps):
            fn()
        e[1].record()
        torch.cuda.synchronize()
        return e[0].elapsed_time(e[1]) / reps * 1e3

    out["small_plain"] = {
        "workload": "K=4 QPSK, 8 antennas, 256 pilots, 2048 data symbols, W=16, cap 256, 10 dB",
        "train_us": lat(lambda: A.train(rxp, symp, p, model=m)),
        "detect_us": lat(lambda: A.detect(m, rx, truth=truth, soft=o["soft"], hard=o["hard"], errors=o["errors"])),
        "batch_train_detect_us": lat(lambda: b.train().detect()),
    }
    inst = synth.make_instance(synth.spec_paper_shape())
    p = A.Params(sigma2=0.05, eps=0.05, mu=1.0, window=20, dict_cap=2 * inst.spec.P)
    rxp, symp, rx = cu(inst.rx_pilot), cu(inst.sym_pilot), cu(inst.rx_data)
    m = A.train(rxp, symp, p)
    o = A.detect(m, rx)
    out["paper_shape"] = {
        "workload": "6 users QPSK, 16 antennas, 685 pilots (dictionary 1370), 3840 data symbols, W=20, sigma2=0.05",
        "train_ms": lat(lambda: A.train(rxp, symp, p, model=m), 5) / 1e3,
        "detect_ms": lat(lambda: A.detect(m, rx, soft=o["soft"], hard=o["hard"])) / 1e3,
        "paper_detect_ms_context": {"RTX 2060 Super": 1.25, "RTX 2080 Ti": 0.906, "Titan V": 0.403,
                                    "source": "paper Table tab:optimization_results, Balanced implementation"},
    }
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the detector has no multi-GPU path to measure.", file=sys.stderr)
        return 2

    import torch
    import paper_2201_05024_amd as A

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    A.library()  # fail loudly if the HIP library is missing

    # the two streams of the pipelined schedules, created first and shared by
    # the workloads (streams created later may share a hardware queue with them)
    s_train, s_det = torch.cuda.Stream(), torch.cuda.Stream()
    head = run_large(args, dev, s_train, s_det)
    out = {
        "metric": METRIC,
        "value": head.pop("value"),
        "unit": "user-symbols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP32 inputs, outputs and accumulation; both inner-product blocks as 3-term split-fp16 MFMA)",
        "data": "synthetic (seeded Rayleigh channel, Rapp PA, AWGN), generated on the device",
    }
    out.update(head)
    extra = set() if args.headline_only else {e for e in args.extra.split(",") if e}
    unknown = extra - {"slot", "mixed", "unrolled", "small"}
    if unknown:
        print(f"bench.py: unknown workloads {sorted(unknown)}", file=sys.stderr)
        return 2
    if "slot" in extra:
        out["slot"] = run_slot(args, dev, s_train, s_det)
    if "mixed" in extra:
        out["batched_mixed"] = run_batched_mixed(args, dev, s_train, s_det)
    if "unrolled" in extra:
        out["unrolled"] = run_unrolled(dev)
    if "small" in extra:
        out.update(run_small(dev))
    if args.copy_calibration:
        n = 64 << 20
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": 4 * n, "write": 4 * n}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
