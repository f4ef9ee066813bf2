"""Benchmark of the APSM detector hot path on one MI355X.

One step = the whole path on one realistic slot at four SNR points
(5, 10, 15, 20 dB): for each point, training on 1024 pilot symbols
(2048 real steps, window 32, dictionary cap 1024) followed by detection,
decisions and symbol-error counting on 1,048,576 data symbols of 6 users
received on 16 antennas (near-far powers in [-6, 0] dB, Rapp PA p = 2,
A_sat = 1).  Inputs are synthetic (seeded) and resident in HBM before the
timed region starts.  The four trainings run in one launch (one workgroup
each), followed by the four detections.

Prints one JSON line: whole-step throughput in detected user-symbols/s, the
roofline of the detection kernel (its average duration measured with HIP
events on its stream), and the FP64 oracle timed on a bounded sample of the
same workload on the host.
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
# Peak of the pipe that binds detection: the FP32 VALU without packed-FP32
# instructions (kept out of the build), 256 CUs x 4 SIMDs x 16 lanes x FMA
# (2 flops) x 2.4 GHz.  The exp2 of each kernel evaluation is a
# transcendental that occupies four VALU issue slots (counted as 8 flops).
# FP32 vector peak: 256 CUs x 4 SIMDs x 32 lanes x 2 flops (FMA) x 2.4 GHz.
# Plain (non-packed) FP32 FMA reaches it: a throughput probe of independent
# v_fma_f32 chains measured 111 TFLOP/s on this GPU, above half of it.
PEAK_FP32_VALU_TFLOPS = 256 * 4 * 32 * 2 * 2.4e9 / 1e12     # 157.3

# HBM bytes per launch of detect_f16_kernel<32,6> on this workload, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by a 256 MiB device copy
# (profiles/detect_f16_realistic_slot_counters.md).  Valid only for the kernel
# sources they were taken with; reported as null otherwise.
MEASURED_TRAFFIC = {
    "bytes": (138977 + 55502) * 1024,
    "sources": {"paper_2201_05024_amd/csrc/detect_f16.h": "5908371f618de0c3b04c177ce06f05ab8e87321b",
                "paper_2201_05024_amd/csrc/detect_f16_m32.hip": "d4dbc3a03f2d61d0eb05e76f679e0ec7b04f4b6c"},
}


def measured_traffic():
    import hashlib
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle timing (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (HBM counter calibration)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched mixed-shape workload")
    ap.add_argument("--serial", action="store_true",
                    help="train then detect within each step (no overlap of consecutive steps)")
    ap.add_argument("--batched-steps", type=int, default=5)
    return ap.parse_args()


def cpu_baseline(spec_fn, snr, params, S_full, n_inst):
    """Time the FP64 oracle on a bounded sample: full training of one instance
    plus detection of 1024 data symbols, extrapolated linearly to one step."""
    import oracle as O
    import synth
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        limiter = None
    inst = synth.make_instance(spec_fn(snr, S=1024))
    p = O.APSMParams(sigma2=params.sigma2, eps=params.eps, mu=params.mu, window=params.window,
                     w_lin=params.w_lin, w_gauss=params.w_gauss, dict_cap=params.dict_cap)
    t0 = time.perf_counter()
    f = O.train_from_pilots(inst.rx_pilot, inst.sym_pilot, p)
    t_train = time.perf_counter() - t0
    t0 = time.perf_counter()
    soft = O.detect_planar(f, inst.rx_data)
    O.symbol_errors(O.decide(soft, "qpsk"), inst.truth)
    t_det = time.perf_counter() - t0
    if limiter is not None:
        limiter.restore_original_limits()
    K = inst.spec.K
    t_step = n_inst * (t_train + t_det * S_full / 1024)
    return {
        "value": n_inst * S_full * K / t_step,
        "unit": "user-symbols/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"FP64 oracle, 1 thread: full training of one {snr:g} dB instance "
                   f"({t_train:.2f} s) and detection of 1024 of {S_full} data symbols "
                   f"({t_det:.2f} s), extrapolated linearly to {n_inst} instances x {S_full} symbols"),
    }


def run_batched(args, dev):
    """The batched mixed-shape workload: 256 detectors (K 2..8, 8/16/32
    antennas, dictionaries of 64..2048 entries with as many pilots, 65,536
    received vectors each, QPSK/16-QAM mixed) trained in one launch and
    detected in one launch, against the plain form (one apsm_train and one
    apsm_detect launch per detector) on the same buffers."""
    import torch
    import synth
    import paper_2201_05024_amd as A

    n = synth.BATCH_INSTANCES
    log(f"[bench] generating the batched workload ({n} detectors)")
    params = A.Params(eps=0.05, mu=1.0, window=32)
    items, evals, syms, flops = [], 0, 0, 0
    for i in range(n):
        spec, D = synth.spec_batch_mixed(i)
        inst = synth.make_instance(spec)
        K, M2, S = spec.K, 2 * spec.M, spec.S
        items.append(A.BatchItem(
            model=A.Model(M2, K, D, dev, 0.5), rx_pilot=torch.from_numpy(inst.rx_pilot).to(dev),
            sym_pilot=torch.from_numpy(inst.sym_pilot).to(dev), rx=torch.from_numpy(inst.rx_data).to(dev),
            modulation=spec.modulation, soft=torch.empty((S, K, 2), dtype=torch.float32, device=dev),
            hard=torch.empty((S, K), dtype=torch.uint8, device=dev),
            truth=torch.from_numpy(inst.truth).to(dev), errors=torch.zeros(K, dtype=torch.int64, device=dev),
            sigma2=0.5))
        evals += 2 * S * D
        flops += 2 * S * D * (2 + 8 + 2 * K)
        syms += S * K
    batch = A.Batch(params, items)
    stream = torch.cuda.current_stream()
    batch.train(stream).detect(stream)
    batch.tune(stream)
    torch.cuda.synchronize()

    def batched_step():
        for it in items:
            it.errors.zero_()
        batch.train(stream).detect(stream)

    def plain_step():
        for it in items:
            it.errors.zero_()
            p = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=32, dict_cap=it.model.dict_cap)
            A.train(it.rx_pilot, it.sym_pilot, p, model=it.model, stream=stream)
            A.detect(it.model, it.rx, modulation=it.modulation, truth=it.truth, soft=it.soft, hard=it.hard,
                     errors=it.errors, stream=stream)

    def timed(fn, steps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    log("[bench] batched form")
    t_batched = timed(batched_step, args.batched_steps)
    log("[bench] plain form")
    t_plain = timed(plain_step, 2)
    # the detection launch alone, with HIP events on its stream
    ev = []
    for _ in range(args.batched_steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        batch.detect(stream)
        e1.record(stream)
        ev.append((e0, e1))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    batch.train(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    det_s = float(np.mean([a.elapsed_time(b) for a, b in ev])) / 1e3
    train_ms = e0.elapsed_time(e1)
    achieved = flops / det_s / 1e12
    return {
        "workload": (f"{n} detectors, K 2..8, 8/16/32 antennas, dictionaries 64..2048 (= pilots), "
                     "65536 vectors each, QPSK/16-QAM mixed, SNR 5..20 dB, W=32, sigma2=0.5"),
        "batched_user_symbols_per_s": syms / t_batched,
        "plain_user_symbols_per_s": syms / t_plain,
        "speedup_vs_plain": t_plain / t_batched,
        "ms_per_step_batched": t_batched * 1e3,
        "ms_per_step_plain": t_plain * 1e3,
        "train_ms_one_launch": train_ms,
        "detect_ms_one_launch": det_s * 1e3,
        "kernel_evals_per_s": evals / det_s,
        "roofline": {"kernel": "detect_batch_kernel", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU_TFLOPS, "traffic": None},
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the detector has no multi-GPU path to measure.", file=sys.stderr)
        return 2

    import torch
    import synth
    import paper_2201_05024_amd as A

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    A.library()  # fail loudly if the HIP library is missing

    snrs = synth.SLOT_SNRS_DB
    params = A.Params(sigma2=0.5, eps=0.05, mu=1.0, window=32, w_lin=0.5, w_gauss=0.5,
                      dict_cap=1024)
    log(f"[bench] generating {len(snrs)} slot instances")
    insts = [synth.make_instance(synth.spec_slot(s)) for s in snrs]
    K, M2, P, S = insts[0].spec.K, 2 * insts[0].spec.M, insts[0].spec.P, insts[0].spec.S
    rx_p = torch.from_numpy(np.stack([i.rx_pilot for i in insts])).to(dev)
    sym_p = torch.from_numpy(np.stack([i.sym_pilot for i in insts])).to(dev)
    rx_d = [torch.from_numpy(i.rx_data).to(dev) for i in insts]
    truth = [torch.from_numpy(i.truth).to(dev) for i in insts]
    # Two model sets: in the pipelined schedule the detectors of step k are
    # trained while the detection of step k - 1 runs on the other set.
    models = [[A.Model(M2, K, params.dict_cap, dev, params.sigma2) for _ in insts] for _ in range(2)]
    # each set is trained by one batch (kernel rows of the 4 pilot blocks in
    # one data-parallel launch, then the 4 trainings in one launch)
    tbatch = [A.Batch(params, [A.BatchItem(model=ms[i], rx_pilot=rx_p[i], sym_pilot=sym_p[i])
                               for i in range(len(insts))]) for ms in models]

    def train_set(k, stream):
        tbatch[k].train(stream)
    soft = [torch.empty((S, K, 2), dtype=torch.float32, device=dev) for _ in insts]
    hard = [torch.empty((S, K), dtype=torch.uint8, device=dev) for _ in insts]
    errs = [torch.zeros(K, dtype=torch.int64, device=dev) for _ in insts]
    s_train = torch.cuda.Stream()
    s_det = torch.cuda.Stream()
    trained = [torch.cuda.Event(), torch.cuda.Event()]
    detected = [torch.cuda.Event(), torch.cuda.Event()]
    rows_ready = [torch.cuda.Event(), torch.cuda.Event()]
    torch.cuda.synchronize()

    det_events = []

    def detect_set(ms, stream, record):
        for e in errs:
            e.zero_()
        for i in range(len(insts)):
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            A.detect(ms[i], rx_d[i], modulation="qpsk", truth=truth[i], soft=soft[i],
                     hard=hard[i], errors=errs[i], stream=stream)
            if record:
                e1.record(stream)
                det_events.append((e0, e1))

    def step(k, record):
        cur, prev = k % 2, (k + 1) % 2
        if args.serial:
            with torch.cuda.stream(s_det):
                train_set(cur, s_det)
                detect_set(models[cur], s_det, record)
            return
        # the kernel rows of step k's pilots (a short launch over the whole
        # GPU) ahead of the detections on the detection stream; then the four
        # trainings of step k (one launch) beside the detection of step k - 1
        with torch.cuda.stream(s_det):
            tbatch[cur].kernel_rows(s_det)
            rows_ready[cur].record(s_det)
        with torch.cuda.stream(s_train):
            s_train.wait_event(detected[cur])
            s_train.wait_event(rows_ready[cur])
            tbatch[cur].train_prepared(s_train)
            trained[cur].record(s_train)
        with torch.cuda.stream(s_det):
            s_det.wait_event(trained[prev])
            detect_set(models[prev], s_det, record)
            detected[prev].record(s_det)

    log(f"[bench] warmup {args.warmup}")
    # the set detected first in the timed region is trained here
    with torch.cuda.stream(s_train):
        train_set(1, s_train)
        trained[1].record(s_train)
    for k in range(args.warmup):
        step(k, False)
    torch.cuda.synchronize()

    # training alone, for the report
    t_ev0, t_ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_ev0.record(s_train)
    train_set(0, s_train)
    t_ev1.record(s_train)
    torch.cuda.synchronize()
    train_ms = t_ev0.elapsed_time(t_ev1)
    # the serialized step (train, then detect) for the report
    t0 = time.perf_counter()
    for _ in range(3):
        with torch.cuda.stream(s_det):
            train_set(0, s_det)
            detect_set(models[0], s_det, False)
    torch.cuda.synchronize()
    serial_ms = (time.perf_counter() - t0) / 3 * 1e3
    # re-arm the pipeline: set 1 trained, set 0 free
    with torch.cuda.stream(s_train):
        train_set(1, s_train)
        trained[1].record(s_train)
    with torch.cuda.stream(s_det):
        detected[0].record(s_det)
    torch.cuda.synchronize()

    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k, True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log("[bench] timed region done")

    det_ms = [a.elapsed_time(b) for a, b in det_events]
    det_avg_s = float(np.mean(det_ms)) / 1e3
    n_inst = len(insts)
    sym_per_step = n_inst * S * K
    value = sym_per_step * args.steps / elapsed
    D = params.dict_cap
    S_r = 2 * S
    evals_per_launch = S_r * D
    # VALU work per kernel evaluation: one FMA for the exponent argument, one
    # exp2 (4 issue slots = 8 flop-equivalents) and K coefficient FMAs.
    valu_flops_per_eval = 2 + 8 + 2 * K
    valu_flops = evals_per_launch * valu_flops_per_eval
    achieved_tflops = valu_flops / det_avg_s / 1e12
    mfma_tflops = evals_per_launch * 2 * M2 / det_avg_s / 1e12
    ser = {f"{s:g}dB": float(e.sum().item()) / (S * K) for s, e in zip(snrs, errs)}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "user-symbols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Rayleigh channel, near-far, Rapp PA, AWGN)",
        "config": {
            "workload": ("realistic slot: K=6 users QPSK, 16 Rx antennas (2M=32), near-far "
                         "[-6,0] dB, Rapp PA p=2 A_sat=1, SNR 5/10/15/20 dB (4 instances), "
                         "1024 pilots, 1048576 data symbols, W=32, sigma2=0.5, eps=0.05, "
                         "mu=1, dictionary cap 1024"),
            "instances_per_step": n_inst,
            "data_symbols": S,
            "pilots": P,
        },
        "roofline": {
            "kernel": "detect_f16_kernel<32,6>",
            "bound": "alu",
            "achieved": achieved_tflops,
            "peak": PEAK_FP32_VALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / PEAK_FP32_VALU_TFLOPS,
            "traffic": measured_traffic(),
            "per_launch": {"real_vectors": S_r, "dictionary": D,
                           "kernel_evals": evals_per_launch,
                           "valu_flops_per_eval": valu_flops_per_eval,
                           "avg_ms": det_avg_s * 1e3, "launches_timed": len(det_ms),
                           "inner_product_tflops_on_mfma": mfma_tflops},
        },
        "detect_only": {
            "user_symbols_per_s": S * K / det_avg_s,
            "kernel_evals_per_s": evals_per_launch / det_avg_s,
        },
        "train_ms_4_instances": train_ms,
        "schedule": ("serial: train then detect within each step" if args.serial else
                     "pipelined: the kernel rows of step k's pilots (one launch) precede the detections "
                     "on the detection stream; the trainings of step k (one launch, 4 CUs) run beside "
                     "the detection of step k-1 on a second stream; every step trains 4 detectors and "
                     "detects 4 x 1048576 symbols"),
        "ms_per_step_serialized": serial_ms,
        "train_steps_per_instance": 2 * P,
        "ser_gpu": ser,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(lambda snr, S: synth.spec_slot(snr, S=S), 10.0, params,
                                           S, n_inst)
    if not args.no_batched:
        out["batched"] = run_batched(args, dev)
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
