#!/usr/bin/env python3
"""Throughput of the SFT template-bank scan on one MI355X.

Workload (the ground-based bank): 3 detectors x 3891 SFTs of 32 s at 128 Hz
(4096 slots per detector, 5% dropped), coloured non-stationary PSD, antenna
patterns, stored band bins [32, 512); 1e5 Newtonian templates with
Mc ~ U[1.0, 1.5], K = 8, automatic Dirichlet/Fresnel kernel, FP64 phase and FP32
compensated sums.  One step = one sft_template_bank_scan over the whole bank, with
data and bank already resident in device memory.

Prints one JSON line with the metric, the roofline of the scan kernel and the FP64
oracle timed on a bounded sample of the same workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "template inner products/s at ≤1e-6 rel err; surrogate+FP32 vs plain path"

# --------------------------------------------------------------------------------------
# Algorithmic VALU work of the scan per (template, SFT), in lane-operation slots
# (an add, mul or FMA = 1 slot; a transcendental v_rcp/v_sqrt/v_sin/v_exp/v_log = 4
# slots, quarter rate).  Counted from the formulas the kernel evaluates:
#   waveform at the SFT midpoint (FP64): tau, y, s = y^(-1/8) (log2 + exp2 + two
#     4-operation Newton steps), kappa, phase, A, beta, 1/tau       -> 21 + 2 T
#   phase reduction mod 2 pi + sin/cos of the reduced phase          ->  4 + 2 T
#   bin split kappa -> k0, delta                                     ->  3
#   kernel setup: Dirichlet sin(pi delta) (1 + 1 T); Fresnel sqrt(2/beta),
#     E-+ phasors, pi beta/4 reduction (~14 + 3 T)
#   per bin: Dirichlet: x = delta - j, 1/x (T), x sp, 2 FMA          ->  3 + 1 T
#            Fresnel (asymptotic endpoints, the dominant branch): two endpoint
#            terms (1/p, w, 2 x (3 FMA + 1 mul), 2 mul) = 2 x (9 + 1 T), the
#            assembly with the two phasors (8) and the complex MAC (4)  -> 30 + 2 T
#   coherent accumulation: complex rotation (6), 4 compensated adds (4 x 4),
#     norm (interpolation 3, 1/S 1 T, 4 mul, 2 compensated adds 8)     -> 37 + 1 T
# --------------------------------------------------------------------------------------
SLOT_T = 4


def alg_slots_per_unit(K: int, kernel: str) -> int:
    base = (21 + 2 * SLOT_T) + (4 + 2 * SLOT_T) + 3 + (37 + 1 * SLOT_T)
    if kernel == "dirichlet":
        return base + (1 + SLOT_T) + (2 * K + 1) * (3 + SLOT_T)
    return base + (14 + 3 * SLOT_T) + (2 * K + 1) * (30 + 2 * SLOT_T)


# peak VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (FP32 and FP64 FMA both
# full rate without packed FP32; = 78.6 TFLOP/s FP64 / 2 flops per FMA)
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--templates", type=int, default=100_000)
    p.add_argument("--cpu-sample", type=int, default=160, help="templates in the oracle sample (0 = skip)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run only a plain device copy of known size (counter calibration)")
    return p.parse_args()


def copy_calibration():
    import torch
    n = 256 << 20  # bytes
    a = torch.empty(n // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "launches": 5}))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (got --gpus %d); the scan would shard "
              "templates across GPUs with no exchange, which is not built here" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2502_11823_amd import sft, synth

    if args.copy_calibration:
        copy_calibration()
        return

    t0 = time.time()
    w = synth.ground(seed=2, n_templates=args.templates)
    K, kernel = 8, "auto"
    data = sft.SFTData.from_workload(w, storage="f32")
    bank = sft.bank_to_device(w.bank)
    opts = sft.make_opts(K=K, kernel=kernel, precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    out = sft.alloc_out(w.n_templates)
    print("setup %.1f s: %d SFTs x %d bins, %d templates" % (time.time() - t0, w.n_sft, w.n_bins, w.n_templates),
          file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        sft.template_bank_scan(data, bank, opts, out=out)
    torch.cuda.synchronize()

    sft.kernel_timing(args.steps)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        sft.template_bank_scan(data, bank, opts, out=out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ktimes = np.array(sft.kernel_times(args.steps), dtype=np.float64)
    sft.kernel_timing(0)

    value = w.n_templates * args.steps / elapsed
    ms_step = 1e3 * elapsed / args.steps
    k_ms = float(np.mean(ktimes)) if ktimes.size else float("nan")
    units = w.n_templates * w.n_sft
    slots = alg_slots_per_unit(K, kernel) * units
    achieved = slots / (k_ms * 1e-3) / 1e12
    peak = PEAK_SLOTS / 1e12

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "IP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64-phase+f32",
        "data": "synthetic",
        "config": {"workload": "ground-3det: %d SFTs x %d bins, %d Newtonian templates, K=%d, %s kernel, "
                               "FP64 phase + FP32 Kahan sums" % (w.n_sft, w.n_bins, w.n_templates, K, kernel),
                   "n_templates": w.n_templates, "n_sft": w.n_sft, "K": K, "kernel": kernel,
                   "precision": "fp32_kahan", "storage": "f32"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "scan_kernel", "kernel_ms": k_ms,
                     "alg_slots_per_template_sft": alg_slots_per_unit(K, kernel)},
    }
    print("scan: %.3f ms/step (kernel %.3f ms), %.3e IP/s" % (ms_step, k_ms, value), file=sys.stderr, flush=True)

    if not args.no_cpu_baseline and args.cpu_sample > 0:
        res["cpu_baseline"] = cpu_baseline(w, out, args.cpu_sample, K, kernel)
    print(json.dumps(res), flush=True)


def cpu_baseline(w, out, n_sample, K, kernel):
    """The FP64 oracle on a seeded template sample of the same workload, host cores."""
    import oracle
    idx = np.sort(np.random.default_rng(12345).choice(w.n_templates, n_sample, replace=False))
    b = w.subset(idx)
    od = oracle.SFTData(w.t_start, w.n_samples, w.t_sft, w.k_lo, w.x_bins, w.psd, w.fplus, w.fcross)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    ref = oracle.scan(od, b["mc"], b["t_c"], phi_c=b["phi_c"], K=K, kernel=oracle.K_AUTO,
                      a_plus=1.0, a_cross=1.0)
    dt = time.perf_counter() - t0
    zp = out["zp"].cpu().numpy()[idx]
    zp = zp[:, 0] + 1j * zp[:, 1]
    zx = out["zx"].cpu().numpy()[idx]
    zx = zx[:, 0] + 1j * zx[:, 1]
    sc = np.maximum(np.abs(ref["zp"]), np.sqrt(ref["hhp"]))
    err = float(max(np.max(np.abs(zp - ref["zp"]) / sc), np.max(np.abs(zx - ref["zx"]) / sc)))
    return {"value": n_sample / dt, "unit": "IP/s", "cores": threads, "kind": "oracle",
            "sample": "%d seeded templates of the same bank, all %d SFTs, FP64 oracle (C, OpenMP), %.1f s"
                      % (n_sample, w.n_sft, dt),
            "max_rel_err_vs_gpu": err}


if __name__ == "__main__":
    main()
