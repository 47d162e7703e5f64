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
# Algorithmic VALU work of the scan, in lane operations: every FP32/FP64 add, mul or FMA and
# every transcendental (rcp, rsqrt, log, exp) of the formulas counts once; compares, selects,
# conversions of loop indices and address arithmetic are not counted.  (An issue-rate probe on
# the MI355X: FMA/MUL streams sustain 0.97 wave-instructions per clock per CU, a v_rcp_f32
# interleaved with FMAs takes ~1.7 issue slots, and 32-bit integer instructions issue beside
# the floating-point ones; the peak below is the FP32 VALU issue rate.)
# Counted from the formulas the kernel evaluates (Fresnel kernel, asymptotic endpoint
# branch, which is the dominant one):
#   per (template, timestamp group), shared by the detectors of the group:
#     FP64 chirp at the SFT midpoint (tau, y, s = y^(-1/8) from log2/exp2 and two
#       Newton steps, kappa, phase, A, beta, Taylor residual)          34 + 2 T
#     window split kappa -> k0, delta                                    4
#     Fresnel set-up: 1/sqrt(beta), scales, endpoint offsets, the two
#       phasors exp(i pi beta/4), exp(i pi delta), E-+, 1/beta (FP64)   63 + 2 T
#     per bin: p-+ (2) and two endpoint terms (|p| sqrt(2/beta), 1/p,
#       r^2, w, w^2, two 3-FMA series, three products)                  28 + 2 T
#     phase phasor exp(i phi) and the signed amplitude                   24
#     norm set-up (floor, weight, A^2 T)                                  6
#   per (template, SFT row):
#     per bin: two complex MACs into S-, S+                              8
#     C = (E- S- - E+ S+) / 2 pi + S_stat                                12
#     term, projector and four Kahan-compensated sums                    26
#     norm term A^2 T / S(f) with interpolation, two Kahan sums          18 + T
# When a group has several detector rows (the kernel's ND >= 2) the Fresnel weights are
# combined per bin once per group, H = (E- e(p-) - E+ e(p+)) / 2 pi + stationary term   12
# per bin, and each row then takes one complex MAC per bin (4) and no final combination.
# The Dirichlet kernel replaces the Fresnel set-up by sin(pi delta) (22) and the per-bin
# group work by x = delta - j and x^-1 (1 + T), and the per-row MACs by 2 FMAs.
# --------------------------------------------------------------------------------------
SLOT_T = 1


def alg_slots(K: int, kernel: str, n_groups: int, n_rows: int, nd: int = 1) -> float:
    nb = 2 * K + 1
    if kernel == "dirichlet":
        per_group = (34 + 2 * SLOT_T) + 4 + 22 + nb * (1 + SLOT_T) + 24 + 6
        per_row = nb * 2 + 26 + (18 + SLOT_T)
    elif nd >= 2:
        per_group = (34 + 2 * SLOT_T) + 4 + (63 + 2 * SLOT_T) + nb * (28 + 2 * SLOT_T + 12) + 24 + 6
        per_row = nb * 4 + 26 + (18 + SLOT_T)
    else:
        per_group = (34 + 2 * SLOT_T) + 4 + (63 + 2 * SLOT_T) + nb * (28 + 2 * SLOT_T) + 24 + 6
        per_row = nb * 8 + 12 + 26 + (18 + SLOT_T)
    return per_group * n_groups + per_row * n_rows


# peak VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (FP32 and FP64 FMA both
# full rate without packed FP32; = 78.6 TFLOP/s FP64 counting an FMA as 2 flops)
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9


KERNEL_SOURCES = ["paper_2502_11823_amd/csrc/sft_lib.hip", "paper_2502_11823_amd/csrc/sft_device.h",
                  "paper_2502_11823_amd/csrc/fresnel_table.h"]
COUNTERS = "profiles/scan_kernel_ground_counters.md"


def measured_traffic():
    """HBM bytes per scan launch from the committed rocprofv3 counter summary, or None when
    the kernel sources have changed since the counters were taken."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    try:
        txt = open(os.path.join(ROOT, COUNTERS)).read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in txt.splitlines() if ":" in line and line[:1].isalpha()
                  and " " not in line.split(":", 1)[0])
    if fields.get("kernel_source_sha256_16", "").strip() != h.hexdigest()[:16]:
        return None
    return float(fields["traffic_bytes_per_launch"])


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--templates", type=int, default=100_000)
    p.add_argument("--cpu-sample", type=int, default=160, help="templates in the oracle sample (0 = skip)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--tuning", default="",
                   help="block,chunk_groups,persistent: use this launch shape instead of autotuning")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run only a plain device copy of known size (counter calibration)")
    p.add_argument("--surrogate-templates", type=int, default=1_000_000,
                   help="templates of the learned-surrogate leg (0 = skip the leg)")
    p.add_argument("--surrogate-samples", type=int, default=10_000_000)
    p.add_argument("--surrogate-epochs", type=int, default=8)
    p.add_argument("--surrogate-only", action="store_true", help="run only the surrogate leg")
    p.add_argument("--space-templates", type=int, default=200_000,
                   help="templates of the space-based leg (0 = skip the leg)")
    p.add_argument("--space-only", action="store_true", help="run only the space-based leg")
    p.add_argument("--paper-shapes", action="store_true",
                   help="context only: time banks shaped like the paper's timing runs and exit")
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

    if args.surrogate_only:
        print(json.dumps(surrogate_leg(args)), flush=True)
        return
    if args.space_only:
        print(json.dumps(space_leg(args)), flush=True)
        return
    if args.paper_shapes:
        print(json.dumps(paper_shapes(args)), flush=True)
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
    t0 = time.time()
    if args.tuning:
        b, c, p = (int(v) for v in args.tuning.split(","))
        sft.set_tuning(data, block=b, chunk_groups=c, persistent=p)
        best = sft.get_tuning(data)
        print("fixed tuning %s" % best.as_dict(), file=sys.stderr, flush=True)
    else:
        best, best_ms = sft.autotune(data, bank, opts, out=out, reps=2)
        torch.cuda.synchronize()
        print("autotune %.1f s: %s -> %.3f ms" % (time.time() - t0, best.as_dict(), best_ms), file=sys.stderr,
              flush=True)

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
    n_groups = int(np.unique(w.t_start).size)
    nd = int(np.max(np.unique(w.t_start, return_counts=True)[1]))   # rows per timestamp group (at most)
    slots = w.n_templates * alg_slots(K, kernel, n_groups, w.n_sft, nd)
    achieved = slots / (k_ms * 1e-3) / 1e12
    peak = PEAK_SLOTS / 1e12

    # the same scan replayed from a captured HIP graph
    plan = sft.Plan(data, bank, opts, out=out)
    for _ in range(2):
        plan.launch()
    torch.cuda.synchronize()
    tg = time.perf_counter()
    for _ in range(args.steps):
        plan.launch()
    torch.cuda.synchronize()
    graph_ms = 1e3 * (time.perf_counter() - tg) / args.steps
    plan.close()

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
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tlane-op/s",
                     "frac": achieved / peak, "traffic": measured_traffic(),
                     "kernel": "scan_kernel", "kernel_ms": k_ms,
                     "alg_lane_ops_per_template": slots / w.n_templates,
                     "units": {"templates": w.n_templates, "timestamp_groups": n_groups, "sft_rows": w.n_sft}},
        "tuning": best.as_dict(),
        "graph_ms_per_step": graph_ms,
    }
    print("scan: %.3f ms/step (kernel %.3f ms), %.3e IP/s" % (ms_step, k_ms, value), file=sys.stderr, flush=True)

    if not args.no_cpu_baseline and args.cpu_sample > 0:
        res["cpu_baseline"] = cpu_baseline(w, out, args.cpu_sample, K, kernel)
    del out, bank, data
    if args.space_templates > 0:
        res["space"] = space_leg(args)
    if args.surrogate_templates > 0:
        res["surrogate"] = surrogate_leg(args)
    print(json.dumps(res), flush=True)


def space_leg(args):
    """Space-based-like bank (one detector, 60 SFTs of 2 days at 0.2 Hz, band [0, 1792) bins):
    2e5 templates with Mc log-uniform in [1e5, 1e6], each using its last 8..60 SFTs (one
    ragged launch), K = 32, automatic kernel (Fresnel throughout: beta from ~0.01 to ~48 bins),
    FP64 phase, FP32 Kahan sums, autotuned launch shape."""
    import torch
    from paper_2502_11823_amd import sft, synth
    K, kernel = 32, "auto"
    w = synth.space(seed=3, n_templates=args.space_templates)
    data = sft.SFTData.from_workload(w, storage="f32")
    bank = sft.bank_to_device(w.bank)
    opts = sft.make_opts(K=K, kernel=kernel, precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    out = sft.alloc_out(w.n_templates)
    best, best_ms = sft.autotune(data, bank, opts, out=out, reps=2)
    for _ in range(args.warmup):
        sft.template_bank_scan(data, bank, opts, out=out)
    torch.cuda.synchronize()
    sft.kernel_timing(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sft.template_bank_scan(data, bank, opts, out=out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    k_ms = float(np.mean(sft.kernel_times(args.steps)))
    sft.kernel_timing(0)
    n_use = (w.bank["a_last"] - w.bank["a_first"] + 1).astype(np.float64)
    slots = float(np.sum(n_use)) * alg_slots(K, "fresnel", 1, 1)   # one group and one row per SFT
    achieved = slots / (k_ms * 1e-3) / 1e12
    flags = out["flags"].cpu().numpy()
    print("space: %.3f ms/step (kernel %.3f ms), %.3e IP/s" % (1e3 * elapsed / args.steps, k_ms,
          w.n_templates * args.steps / elapsed), file=sys.stderr, flush=True)
    return {"workload": "space-like: 60 SFTs x 2 d at 0.2 Hz, band 1792 bins, %d templates Mc log-U[1e5,1e6], "
                        "8-60 SFTs each (ragged), K=%d, auto kernel (Fresnel), FP64 phase + FP32 Kahan sums"
                        % (w.n_templates, K),
            "value": w.n_templates * args.steps / elapsed, "unit": "IP/s", "ms_per_step": 1e3 * elapsed / args.steps,
            "template_sfts": float(np.sum(n_use)),
            "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_SLOTS / 1e12, "unit": "Tlane-op/s",
                         "frac": achieved / (PEAK_SLOTS / 1e12), "kernel": "scan_kernel", "kernel_ms": k_ms,
                         "alg_lane_ops_per_template_sft": alg_slots(K, "fresnel", 1, 1)},
            "tuning": best.as_dict(), "flagged_templates": int(np.sum(flags != 0))}


# The paper's own timings (Sec. V.C), NVIDIA H100 with JAX vmap over batches of 1000
# waveforms, precision not stated, IMRPhenomT waveforms generated inside the timing:
# per-waveform cost in seconds.  Quoted as context beside runs of the same shapes here.
PAPER_H100_BATCH_S = {"bns": 0.4e-3, "mbbh": 0.08e-3}


def paper_shapes(args):
    """Banks shaped like the paper's timing workloads (leading-order chirp, not IMRPhenomT):
    throughput of the scan next to the paper's per-waveform H100 cost.  Context only."""
    import torch
    from paper_2502_11823_amd import sft, synth
    res = {}
    for name in ("bns", "mbbh"):
        w = synth.paper_shape(name)
        K = int(w.opts["K"])
        data = sft.SFTData.from_workload(w, storage="f32")
        bank = sft.bank_to_device(w.bank)
        opts = sft.make_opts(K=K, kernel="auto", precision="fp32_kahan")
        out = sft.alloc_out(w.n_templates)
        best, _ = sft.autotune(data, bank, opts, out=out, reps=2)
        sft.template_bank_scan(data, bank, opts, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            sft.template_bank_scan(data, bank, opts, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        flags = out["flags"].cpu().numpy()
        res[name] = {"n_sft": w.n_sft, "bins_per_sft": w.n_bins, "K": K, "templates": w.n_templates,
                     "ms_per_scan": 1e3 * dt, "value": w.n_templates / dt, "unit": "IP/s",
                     "per_waveform_s": dt / w.n_templates, "tuning": best.as_dict(),
                     "flagged_templates": int(np.sum(flags != 0)),
                     "paper_h100_batch1000_per_waveform_s": PAPER_H100_BATCH_S[name],
                     "paper_h100_ip_per_s": 1.0 / PAPER_H100_BATCH_S[name]}
        print("%s: %.3f ms per %d-template scan, %.3e IP/s (paper H100: %.3e IP/s)" % (
            name, 1e3 * dt, w.n_templates, w.n_templates / dt, 1.0 / PAPER_H100_BATCH_S[name]),
            file=sys.stderr, flush=True)
        del data, bank, out
    return {"context": "banks shaped like the paper's timing runs; leading-order chirp; not the metric", **res}


# the learned surrogate's domain on the tiny data: Mc in [1.19, 1.21], q in [1, 2],
# tau in [600, 16984] s; phase scale 2 rad, log-amplitude scale 0.01, analytic head
SUR_CFG = dict(mc=(1.19, 1.21), q=(1.0, 2.0), ln_tau=(float(np.log(600.0)), float(np.log(16984.0))),
               c_phi=2.0, c_amp=0.01, head=1)


def surrogate_leg(args):
    """Learned-surrogate form on the tiny data (256 SFTs of 64 s, one detector, K = 4
    Dirichlet): the network 3 -> 128 x 4 -> 2 is trained with the library's kernels on
    3.5PN targets, then the bank (Mc ~ U[1.19, 1.21], q ~ U[1, 2]) is scanned with the
    surrogate waveform (FP64 network evaluation, judge at 1e-4 with 3.5PN fallback) and,
    for comparison, with the plain leading-order chirp and with the 3.5PN waveform."""
    import torch
    from paper_2502_11823_amd import sft, synth
    hidden, layers = 128, 4
    w = synth.tiny(seed=1, n_templates=1, noise_series=False)
    n = args.surrogate_templates
    bank = synth.uniform_bank(n, 1.19, 1.21, 16984.0, 501, q_lo=1.0, q_hi=2.0, random_phase=True,
                              n_sft=w.n_sft)
    data = sft.SFTData.from_workload(w, storage="f32")
    bt = sft.bank_to_device(bank)
    s = sft.Surrogate(synth.mlp_init(23, hidden, layers), hidden=hidden, layers=layers, judge_tol=1e-4,
                      **SUR_CFG)
    # training set on the device
    t0 = time.perf_counter()
    mc, q, tau = synth.surrogate_samples(args.surrogate_samples, 41, 1.19, 1.21, 1.0, 2.0, 600.0, 16984.0)
    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
    u, y = s.targets(dev(mc), dev(q), dev(tau))
    del mc, q, tau
    torch.cuda.synchronize()
    t_targets = time.perf_counter() - t0
    t0 = time.perf_counter()
    hist = s.train(u, y, batch=4096, epochs=args.surrogate_epochs, lr=2e-3, lr_min=1e-5)
    t_train = time.perf_counter() - t0
    del u, y
    print("surrogate training: %d samples x %d epochs in %.1f s, loss %s" % (
        args.surrogate_samples, args.surrogate_epochs, t_train, np.array2string(hist, precision=2)),
        file=sys.stderr, flush=True)

    out = sft.alloc_out(n, mismatch=True)
    steps = max(1, min(args.steps, 3))

    def timed(opts):
        sft.template_bank_scan(data, bt, opts, out=out)    # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            sft.template_bank_scan(data, bt, opts, out=out)
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) / steps

    common = dict(K=4, kernel="dirichlet", precision="fp32_kahan")
    t_plain = timed(sft.make_opts(waveform="newton", **common))
    t_pn = timed(sft.make_opts(waveform="pn35", **common))
    t_sur = timed(sft.make_opts(waveform="surrogate", surrogate=s, **common))
    flags = out["flags"].cpu().numpy()
    mm = out["mismatch"].cpu().numpy()
    fb = float(np.mean((flags & sft.FLAG_SURROGATE_FALLBACK) > 0))
    evals = n * w.n_sft
    mlp_flop = evals * 2 * 2 * (3 * hidden + (layers - 1) * hidden * hidden + hidden * 2)
    res = {"workload": "tiny data (256 SFTs x 64 s, 1 detector, K=4 Dirichlet, FP32 Kahan sums), %d templates "
                       "Mc~U[1.19,1.21] q~U[1,2]; MLP 3-%dx%d-2 SiLU trained on %d 3.5PN samples"
                       % (n, hidden, layers, args.surrogate_samples),
           "value": n / t_sur, "unit": "IP/s", "ms_per_step": 1e3 * t_sur, "steps": steps,
           "plain_newton_value": n / t_plain, "pn35_value": n / t_pn,
           "surrogate_over_plain": t_plain / t_sur, "surrogate_over_pn35": t_pn / t_sur,
           "network_evals_per_step": evals, "network_fp64_tflop_per_step": mlp_flop / 1e12,
           "fallback_frac": fb, "judge_tol": 1e-4,
           "mismatch_median": float(np.median(mm)), "mismatch_p99": float(np.quantile(mm, 0.99)),
           "train": {"samples": args.surrogate_samples, "epochs": args.surrogate_epochs, "batch": 4096,
                     "targets_s": t_targets, "train_s": t_train, "epoch_loss": [float(v) for v in hist]}}
    print("surrogate scan %.1f ms (plain %.2f ms, 3.5PN %.2f ms), fallback %.4f" % (
        1e3 * t_sur, 1e3 * t_plain, 1e3 * t_pn, fb), file=sys.stderr, flush=True)
    s.close()
    return res


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
