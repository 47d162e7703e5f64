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
# Algorithmic VALU work of the scan, in FP32 lane-operation slots: every FP32 add, mul or FMA
# and every transcendental (rcp, rsqrt, log2, exp2) of the formulas counts 1 and every FP64
# add, mul or FMA counts 2 (the FP64 vector rate is half the FP32 one); compares, selects,
# conversions, index and address arithmetic are not counted.
# Peak: the FP32 vector rate, 157.3 TFLOP/s with an FMA as two flops, i.e. 256 CUs x 2.4 GHz
# x 128 lanes per clock = 78.6e12 slots/s.  Packed FP32 is disabled at compile time; plain
# wave64 FP32 instructions still issue faster than one per clock per CU: the library's issue-rate
# probe (16 independent FMA chains per lane, run below right after the timed scan) sustains
# about 1.5 wave-instructions per clock per CU of the 2.0 this peak implies, and the roofline
# object also reports the scan against that practical FMA ceiling.
#
# Per (template, timestamp group), shared by the detector rows of the group:
OPS_CHIRP = 2 * 34 + 2      # Newtonian chirp at the SFT midpoint in FP64 (tau, y, s = y^(-1/8)
                            # from log2/exp2 seeds and two Newton steps, kappa, phase, A, beta)
OPS_SPLIT = 2 * 2           # kappa -> k0, delta (FP64)
OPS_TAIL = 24 + 2 * 2 + 2 + 4 + 6 * 4
                            # exp(i phi) (FP64 reduction + series), norm set-up (FP64 floor and
                            # weight, A^2 T), signed amplitude, six Kahan-compensated additions
OPS_FRESNEL = 2 * 22 + 7 + 9 + 18 + 6 * 5
                            # exp(i pi beta/4), exp(i pi delta), 1/sqrt(beta) and scales, 1/beta
                            # (FP64 Newton), E-+, E-/2pi, E+/2pi and rho = E+/E-, and the six
                            # wave-uniform series-tier bounds
OPS_DIRICHLET = 23          # sin(pi delta) / pi
# Fresnel weights per bin and lane, by the series length the bin's endpoints need (two
# endpoints each; p-+ = delta -+ beta/2 - j is 2): both endpoints at v = |p| sqrt(2/beta) >= 76
# (no W term: 1/p, r^2, w, r w), >= 11 (one W term: 5 more), >= 4.5 (three W terms: 4 more),
# else the 90-interval quartic table (|p| sqrt(2/beta), the offset in the interval, two Horner
# chains of 4, the scale) and the stationary-point test
OPS_BIN = {"w0": 2 + 2 * (1 + 3), "w1": 2 + 2 * (1 + 8), "w3": 2 + 2 * (1 + 12), "table": 2 + 2 * 13 + 2}
OPS_BIN_SERIES = 24         # central bin with |beta| <= 0.04 and |delta| <= 0.125: F(delta, beta)
                            # from its series (two 4-term Horner chains in (pi delta)^2 with
                            # beta-folded coefficients)
SERIES_BETA, SERIES_DELTA = 0.04, 0.125
OPS_BIN_STAT = 2 * 3 + 2 * 3 + 16 + 5 + 6   # stationary point inside the SFT: x^2/beta and its
                                            # reduction (FP64), the phasor, the term, folded into e(p-)
OPS_BIN_DIR = 3                             # x = delta - j, 1/x, sin(pi delta)/pi x
OPS_BIN_SHARED = 4                          # several rows: H' = e(p-) - rho e(p+) once per bin
# Per (template, SFT row):
OPS_ROW_MAC = 4             # complex MAC per bin (Fresnel); Dirichlet: 2 (real weight)
OPS_ROW_EQ = 4              # several rows: E-/2pi applied to the row's sum
OPS_ROW_TAIL = 4 + 4 + 3 + 1 + 1 + 2 + 2
                            # the term, four projector products, the PSD at f interpolated,
                            # 1/S, A^2 T/S, F+^2 and Fx^2, two norm products
OPS_ROW1_MAC = 8            # one-row kernel: b e(p-) and b e(p+) per bin (no H'), then
OPS_ROW1_COMB = 10          # C = E-/2pi S- - E+/2pi S+ once
SERIES_V = (76.0, 11.0, 4.5)
# F-statistic form: per present row the cross-norm product F+ Fx and its FMA (FP32); per pair the
# three norm sums in FP64 (one FP64 add each) instead of two FP32 compensated sums
OPS_FSTAT_ROW = 2
OPS_FSTAT_PAIR = 3 * 2 - 2 * 4
# Doppler form, per (template, row): r.n, v.n, a.n (9 FP64 FMAs), then kappa (1 + v.n),
# beta (1 + v.n)^2 + kappa a.n T and the fddot scaling (8 FP64 operations)
OPS_DOPPLER = 2 * (9 + 8)
OUTER_MIN_K = 4             # narrower windows use the table for every bin


def scan_census(mc, t_c, g_tmid, g_rows, T, K, beta_switch, tsun, g_first=None, g_last=None, multi_row=True,
                stride=64, chunk=256, fstat=False, eph=None, sky=None):
    """Algorithmic slots of one scan (the counts above), from the Newtonian chirp of every
    stride-th template at every timestamp group it uses, scaled to the whole bank.  g_rows:
    SFT rows present per group; g_first/g_last: the template's group range (ragged banks);
    fstat: the F-statistic form; eph [n_groups, 9] (r/c, v/c, a/c per group, one row each) and
    sky [n, 3] (unit vectors toward the sources): the Doppler form, whose chirp is taken at the
    emission time with f and fdot scaled by the delay's rates."""
    mc = np.asarray(mc, np.float64)
    n = mc.size
    pick = np.arange(0, n, stride)
    total = 0.0
    census = {"pairs": 0, "w0": 0, "w1": 0, "w3": 0, "table": 0, "stat": 0, "series": 0, "dirichlet_pairs": 0}
    nb = 2 * K + 1
    for i0 in range(0, pick.size, chunk):
        idx = pick[i0:i0 + chunk]
        M = mc[idx, None] * tsun
        tau = np.asarray(t_c, np.float64)[idx, None] - np.asarray(g_tmid, np.float64)[None, :]
        if eph is not None:
            nv = np.asarray(sky, np.float64)[idx]
            e = np.asarray(eph, np.float64)
            dl, dl1, dl2 = nv @ e[:, 0:3].T, nv @ e[:, 3:6].T, nv @ e[:, 6:9].T
            tau = tau - dl
        use = tau > 0
        if g_first is not None:
            gi = np.arange(len(g_tmid))[None, :]
            use &= (gi >= np.asarray(g_first)[idx, None]) & (gi <= np.asarray(g_last)[idx, None])
        taus = np.where(use, tau, 1.0)
        f = (5.0 * M / taus) ** 0.375 / (8.0 * np.pi * M)
        fdot = 96.0 / 5.0 * np.pi ** (8.0 / 3.0) * M ** (5.0 / 3.0) * f ** (11.0 / 3.0)
        kap = f * T
        beta = fdot * T * T
        if eph is not None:
            g1 = 1.0 + dl1
            beta = beta * g1 * g1 + kap * dl2 * T
            kap = kap * g1
        delta = kap - np.floor(kap + 0.5)
        rows = np.broadcast_to(np.asarray(g_rows, np.float64)[None, :], use.shape)
        fres = use & (np.abs(beta) > beta_switch)
        dirp = use & ~fres
        b = np.where(fres, np.abs(beta), 1.0)
        ds = np.where(beta < 0, -delta, delta)
        dm, dp = ds - 0.5 * b, ds + 0.5 * b
        s2b = np.sqrt(2.0 / b)
        n_pairs = float(use.sum())
        n_rows = float((rows * use).sum())
        ops = n_pairs * (OPS_CHIRP + OPS_SPLIT + OPS_TAIL) + float(fres.sum()) * OPS_FRESNEL
        ops += float(dirp.sum()) * (OPS_DIRICHLET + nb * OPS_BIN_DIR) + float((rows * dirp).sum()) * nb * 2
        ops += n_rows * OPS_ROW_TAIL
        if fstat:
            ops += n_rows * OPS_FSTAT_ROW + n_pairs * OPS_FSTAT_PAIR
        if eph is not None:
            ops += n_pairs * OPS_DOPPLER
        for jj in range(-K, K + 1):
            pm, pp = dm - jj, dp - jj
            v = np.minimum(np.abs(pm), np.abs(pp)) * s2b
            same = pm * pp > 0
            if K >= OUTER_MIN_K:
                w0 = fres & same & (v >= SERIES_V[0])
                w1 = fres & same & (v >= SERIES_V[1]) & ~w0
                w3 = fres & same & (v >= SERIES_V[2]) & ~w0 & ~w1
            else:
                w0 = w1 = w3 = np.zeros_like(fres)
            tab = fres & ~w0 & ~w1 & ~w3
            if jj == 0:
                ser = fres & (b <= SERIES_BETA) & (np.abs(delta) <= SERIES_DELTA)
                census["series"] += float(ser.sum())
                ops += float(ser.sum()) * OPS_BIN_SERIES
                w0, w1, w3, tab = w0 & ~ser, w1 & ~ser, w3 & ~ser, tab & ~ser
            stat = tab & (pm < 0) & (pp >= 0)
            for key, msk in (("w0", w0), ("w1", w1), ("w3", w3), ("table", tab)):
                c_ = float(msk.sum())
                census[key] += c_
                ops += c_ * OPS_BIN[key]
            census["stat"] += float(stat.sum())
            ops += float(stat.sum()) * OPS_BIN_STAT
        if multi_row:
            ops += float(fres.sum()) * nb * OPS_BIN_SHARED + float((rows * fres).sum()) * (nb * OPS_ROW_MAC + OPS_ROW_EQ)
        else:
            ops += float(fres.sum()) * (nb * OPS_ROW1_MAC + OPS_ROW1_COMB)
        census["pairs"] += n_pairs
        census["dirichlet_pairs"] += float(dirp.sum())
        total += ops
    scale = n / pick.size
    census = {k: v * scale for k, v in census.items()}
    return total * scale, census


# peak FP32 VALU rate in lane-operation slots per second (see above)
PEAK_SLOTS = 256 * 128 * 2.4e9


KERNEL_SOURCES = ["paper_2502_11823_amd/csrc/sft_scan.h", "paper_2502_11823_amd/csrc/sft_scan_args.h",
                  "paper_2502_11823_amd/csrc/sft_device.h", "paper_2502_11823_amd/csrc/fresnel_table.h"]
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


def _alu_roofline(achieved, k_ms, slots, args):
    """Roofline object of a scan-kernel leg: census slots per second against the FP32 vector
    peak, and against the probed FP32 FMA issue ceiling when the main leg measured it."""
    ceiling = getattr(args, "fma_ceiling", None)
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_SLOTS / 1e12, "unit": "Tslot/s",
            "frac": achieved / (PEAK_SLOTS / 1e12), "kernel": "scan_kernel", "kernel_ms": k_ms,
            "alg_slots_per_launch": slots, "frac_of_fma_ceiling": (achieved / ceiling) if ceiling else None}


def issue_probe(achieved):
    """The rates that plain wave64 VALU instructions sustain on this part (probe of 16
    independent chains per lane), per clock per CU at the nominal 2.4 GHz, and the scan's census
    rate against the FP32 FMA one: the practical ceiling with packed FP32 left off."""
    from paper_2502_11823_amd import sft
    per_clk = {op: sft.probe_issue_rate(op) / (256 * 2.4e9) for op in sft.PROBE}
    ceiling = per_clk["v_fma_f32"] * 256 * 2.4e9 * 64 / 1e12   # FP32 slots/s of plain FMAs
    print("issue probe (wave-instr/clk/CU): %s; FP32 FMA ceiling %.1f Tslot/s, scan at %.3f of it"
          % ({k: round(v, 3) for k, v in per_clk.items()}, ceiling, achieved / ceiling), file=sys.stderr, flush=True)
    return {"unit": "VALU wave-instructions per clock per CU at 2.4 GHz", "rates": per_clk,
            "nominal_fp32_rate": 2.0, "fp32_fma_ceiling_tslot_s": ceiling, "frac_of_fma_ceiling": achieved / ceiling}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--templates", type=int, default=100_000)
    p.add_argument("--cpu-sample", type=int, default=160, help="templates in the oracle sample (0 = skip)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--tuning", default="",
                   help="block,chunk_groups,persistent: use this launch shape instead of autotuning "
                        "(the ground scan; with --space-only, the space scan)")
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
    p.add_argument("--no-fstat", action="store_true", help="skip the F-statistic leg")
    p.add_argument("--no-order", action="store_true", help="skip the bank-order leg")
    p.add_argument("--no-doppler", action="store_true", help="skip the Doppler leg")
    p.add_argument("--no-strain", action="store_true", help="skip the SFT-creation leg")
    p.add_argument("--no-r-study", action="store_true", help="skip the accuracy-study leg")
    p.add_argument("--no-issue-probe", action="store_true", help="skip the VALU issue-rate probe")
    p.add_argument("--strain-only", action="store_true", help="run only the SFT-creation leg")
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
        print("bench.py: runs on one GPU only (got --gpus %d); the scan would shard "
              "templates across GPUs with no exchange, which is not implemented here" % args.gpus, file=sys.stderr)
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
    if args.strain_only:
        print(json.dumps(strain_leg(args)), flush=True)
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
        best, best_ms = sft.autotune(data, bank, opts, out=out, reps=3)
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
    g_t, g_rows = np.unique(w.t_start, return_counts=True)
    n_groups = int(g_t.size)
    slots, census = scan_census(w.bank["mc"], w.bank["t_c"], g_t + 0.5 * w.t_sft, g_rows, w.t_sft, K, 1e-7,
                                sft.T_SUN, multi_row=True)
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
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                     "frac": achieved / peak, "traffic": measured_traffic(),
                     "kernel": "scan_kernel", "kernel_ms": k_ms,
                     "alg_slots_per_launch": slots, "alg_slots_per_template_group": slots / census["pairs"],
                     "units": {"templates": w.n_templates, "timestamp_groups": n_groups, "sft_rows": w.n_sft},
                     "bins_by_series": {k: census[k] / census["pairs"] for k in ("w0", "w1", "w3", "table", "stat", "series")}},
        "tuning": best.as_dict(),
        "graph_ms_per_step": graph_ms,
    }
    print("scan: %.3f ms/step (kernel %.3f ms), %.3e IP/s" % (ms_step, k_ms, value), file=sys.stderr, flush=True)
    if not args.no_issue_probe:
        res["roofline"]["issue_probe"] = issue_probe(achieved)
        args.fma_ceiling = res["roofline"]["issue_probe"]["fp32_fma_ceiling_tslot_s"]

    if not args.no_cpu_baseline and args.cpu_sample > 0:
        res["cpu_baseline"] = cpu_baseline(w, out, args.cpu_sample, K, kernel)
    if not args.no_fstat:
        res["fstat"] = fstat_leg(args, w, data, bank, opts, K)
    if not args.no_order:
        res["order"] = order_leg(args, w, data, bank, opts, out)
    del out, bank, data
    if not args.no_doppler:
        res["doppler"] = doppler_leg(args, w, opts, K)
    if not args.no_strain:
        res["strain"] = strain_leg(args)
    if not args.no_r_study:
        res["r_study"] = r_study_leg()
    if args.space_templates > 0:
        res["space"] = space_leg(args)
    if args.surrogate_templates > 0:
        res["surrogate"] = surrogate_leg(args)
    print(json.dumps(res), flush=True)


def order_leg(args, w, data, bank, opts, out):
    """The same ground bank shuffled: scanned in its given order, and sorted by track on the
    device (sort and gathers included in the time), against the sorted bank in its given order;
    whole scans per step timed with events on the stream."""
    import torch

    from paper_2502_11823_amd import sft
    t0 = time.time()
    perm = np.random.default_rng(4242).permutation(w.n_templates)
    shuf = sft.bank_to_device({k: np.ascontiguousarray(v[perm]) for k, v in w.bank.items()})
    keep = sft.get_tuning(data)
    tune = keep.as_dict()

    def timed(b, order):
        sft.set_tuning(data, block=tune["block"], chunk_groups=tune["chunk_groups"],
                       persistent=tune["persistent"], order=order)
        sft.template_bank_scan(data, b, opts, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            sft.template_bank_scan(data, b, opts, out=out)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    sorted_ms = timed(bank, "given")
    shuf_given_ms = timed(shuf, "given")
    shuf_track_ms = timed(shuf, "track")
    sft.set_tuning(data, block=keep.block, chunk_groups=keep.chunk_groups, persistent=keep.persistent,
                   order=keep.order)
    del shuf
    print("order leg %.1f s: sorted %.3f ms, shuffled %.3f ms, shuffled+track sort %.3f ms"
          % (time.time() - t0, sorted_ms, shuf_given_ms, shuf_track_ms), file=sys.stderr, flush=True)
    return {"workload": "the ground bank shuffled (seed 4242), same data, K and launch shape",
            "sorted_given_ms": sorted_ms, "shuffled_given_ms": shuf_given_ms,
            "shuffled_track_ms": shuf_track_ms, "track_over_sorted": shuf_track_ms / sorted_ms}


def fstat_leg(args, w, data, bank, opts, K):
    """The F-statistic form (Sec. II.B) on the same ground bank and launch shape: z, the three
    norms and 2F per template; a seeded sample of 40 templates is checked against the oracle."""
    import torch
    import oracle
    from paper_2502_11823_amd import sft
    out = sft.alloc_out(w.n_templates, fstat=True)
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
    f2 = out["twoF"].cpu().numpy()
    flags = out["flags"].cpu().numpy().astype(np.uint32)
    idx = np.sort(np.random.default_rng(777).choice(w.n_templates, 40, replace=False))
    b = w.subset(idx)
    od = oracle.SFTData(w.t_start, w.n_samples, w.t_sft, w.k_lo, w.x_bins, w.psd, w.fplus, w.fcross)
    ref = oracle.scan(od, b["mc"], b["t_c"], phi_c=b["phi_c"], K=K, kernel=oracle.K_AUTO, a_plus=1.0,
                      a_cross=1.0, fstat=True)
    err = float(np.max(np.abs(f2[idx] - ref["twoF"]) / np.maximum(ref["twoF"], 4.0)))
    value = w.n_templates * args.steps / elapsed
    g_t, g_rows = np.unique(w.t_start, return_counts=True)
    slots, _ = scan_census(w.bank["mc"], w.bank["t_c"], g_t + 0.5 * w.t_sft, g_rows, w.t_sft, K, 1e-7,
                           sft.T_SUN, multi_row=True, fstat=True)
    achieved = slots / (k_ms * 1e-3) / 1e12
    print("fstat census: %.3e slots, %.1f Tslot/s, %.3f of the FP32 peak"
          % (slots, achieved, achieved / (PEAK_SLOTS / 1e12)), file=sys.stderr, flush=True)
    print("fstat: %.3f ms/step (kernel %.3f ms), %.3e IP/s, max e(2F) %.2e on 40 templates"
          % (1e3 * elapsed / args.steps, k_ms, value, err), file=sys.stderr, flush=True)
    return {"workload": "F-statistic form of the ground scan (same data, bank, K, launch shape): z+, zx, "
                        "hh+, hhx, hh+x and 2F = x.M^-1.x per template",
            "value": value, "unit": "IP/s", "ms_per_step": 1e3 * elapsed / args.steps, "kernel_ms": k_ms,
            "twoF_median": float(np.median(f2)), "twoF_mean": float(np.mean(f2)),
            "degenerate_frac": float(np.mean((flags & sft.FLAG_FSTAT_DEGENERATE) != 0)),
            "max_err_2F_vs_oracle_40": err,
            "roofline": _alu_roofline(achieved, k_ms, slots, args)}


def r_study_leg():
    """The accuracy study of Sec. IV: r(delta, Delta k) for the BNS (3.5PN) and massive-BBH
    (leading-order chirp) pilot sources, every step on the device (signal series, direct
    integral, SFTs, SFT inner product)."""
    from paper_2502_11823_amd import study
    res = {}
    for case in ("bns", "mbbh"):
        r = study.r_study(case, dks=(4, 8, 12, 16, 20, 24, 32, 40, 48, 64),
                          log=lambda m: print(m, file=sys.stderr, flush=True))
        res[case] = {"waveform": r["waveform"], "duration_h": r["duration_h"], "n0": r["n0"],
                     "fddot_max": r["fddot_max"], "config": {str(k): v for k, v in r["config"].items()},
                     "r": {str(k): {str(dk): v for dk, v in row.items()} for k, row in r["r"].items()},
                     "seconds": r["seconds"]}
    return res


def strain_leg(args):
    """SFT creation from raw strain on the device (the step upstream of the scan, Sec. III.B):
    three detectors x 4096 segments of 4096 samples at 128 Hz (the ground data set before it is
    cut into SFTs, 402 MB of FP64), FFT of every segment, band bins [32, 512) and their PSD by a
    51-bin running median.  Bound: HBM (algorithmic bytes: the series read once, band bins and
    PSD written once)."""
    import torch
    from paper_2502_11823_amd import sft
    n, n_slots, n_det, k_lo, n_bins, w = 4096, 4096, 3, 32, 480, 25
    dt = 1.0 / 128.0
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1234)
    x = torch.randn((n_det, n * n_slots), dtype=torch.float64, device="cuda", generator=gen)
    sft.make_sfts(x, n, dt, k_lo, n_bins, w)            # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(max(3, min(args.steps, 10))):
        e0.record()
        sft.make_sfts(x, n, dt, k_lo, n_bins, w)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    t0 = time.perf_counter()
    data = sft.SFTData.from_strain(x, n, dt, k_lo, n_bins, w)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t0
    n_seg = n_slots * n_det
    alg_bytes = x.numel() * 8 + n_seg * n_bins * (16 + 8)
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    print("strain: %d segments in %.3f ms (%.0f GB/s of algorithmic traffic), full load %.3f s"
          % (n_seg, ms, achieved, load_s), file=sys.stderr, flush=True)
    res = {"workload": "SFT creation: 3 detectors x 4096 segments x 4096 samples (128 Hz, 32 s SFTs), band "
                       "[32, 512), running-median PSD over 51 bins",
           "segments_per_s": n_seg / (ms * 1e-3), "ms_per_launch": ms,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                        "frac": achieved / 8000.0, "alg_bytes_per_launch": alg_bytes},
           "load_strain_s": load_s, "n_rows": data.n_sft}
    data.close()
    return res


# detector sites of the Doppler leg (latitude, longitude) [rad]
SITES = [(0.81, -1.58), (0.53, -2.08), (0.76, 0.18)]


def doppler_leg(args, w, opts, K):
    """The Doppler form (Sec. III.B) on the ground bank: every template with its own sky
    position, each detector at its own site on the rotating, orbiting Earth (every SFT row then
    has its own waveform: one row per timestamp group), autotuned launch shape."""
    import torch
    from paper_2502_11823_amd import sft, synth
    tm = w.t_start + 0.5 * w.t_sft
    eph = np.empty((w.n_sft, 9))
    for d, (lat, lon) in enumerate(SITES):
        m = w.det == d
        eph[m] = synth.ground_ephemeris(tm[m], lat, lon)
    g = np.random.default_rng(99)
    bank_h = dict(w.bank)
    bank_h["sky"] = synth.sky_vector(g.uniform(0, 2 * np.pi, w.n_templates),
                                     np.arcsin(g.uniform(-1, 1, w.n_templates)))
    data = sft.SFTData.from_workload(w, storage="f32")
    data.set_ephemeris(eph)
    bank = sft.bank_to_device(bank_h)
    out = sft.alloc_out(w.n_templates)
    best, _ = sft.autotune(data, bank, opts, out=out, reps=2)
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
    value = w.n_templates * args.steps / elapsed
    print("doppler: %.3f ms/step (kernel %.3f ms), %.3e IP/s" % (1e3 * elapsed / args.steps, k_ms, value),
          file=sys.stderr, flush=True)
    # every SFT row its own group (one-row kernel), its chirp at the emission time
    slots, _ = scan_census(w.bank["mc"], w.bank["t_c"], tm, np.ones(w.n_sft), w.t_sft, K, 1e-7, sft.T_SUN,
                           multi_row=False, eph=eph, sky=bank_h["sky"], stride=128)
    achieved = slots / (k_ms * 1e-3) / 1e12
    print("doppler census: %.3e slots, %.1f Tslot/s, %.3f of the FP32 peak"
          % (slots, achieved, achieved / (PEAK_SLOTS / 1e12)), file=sys.stderr, flush=True)
    return {"workload": "Doppler form of the ground scan: 3 detector sites (Earth orbit + rotation), "
                        "random sky position per template, one SFT row per timestamp group",
            "value": value, "unit": "IP/s", "ms_per_step": 1e3 * elapsed / args.steps, "kernel_ms": k_ms,
            "tuning": best.as_dict(), "roofline": _alu_roofline(achieved, k_ms, slots, args)}


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
    if args.tuning and args.space_only:
        b, c, p = (int(v) for v in args.tuning.split(","))
        sft.set_tuning(data, block=b, chunk_groups=c, persistent=p)
        best = sft.get_tuning(data)
        print("fixed tuning %s" % best.as_dict(), file=sys.stderr, flush=True)
    else:
        best, best_ms = sft.autotune(data, bank, opts, out=out, reps=3)
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
    # one row per timestamp group (one detector): group index = SFT index
    slots, census = scan_census(w.bank["mc"], w.bank["t_c"], w.t_start + 0.5 * w.t_sft, np.ones(w.n_sft), w.t_sft,
                                K, 1e-7, sft.T_SUN, g_first=w.bank["a_first"], g_last=w.bank["a_last"],
                                multi_row=False, stride=16)
    achieved = slots / (k_ms * 1e-3) / 1e12
    flags = out["flags"].cpu().numpy()
    print("space: %.3f ms/step (kernel %.3f ms), %.3e IP/s" % (1e3 * elapsed / args.steps, k_ms,
          w.n_templates * args.steps / elapsed), file=sys.stderr, flush=True)
    return {"workload": "space-like: 60 SFTs x 2 d at 0.2 Hz, band 1792 bins, %d templates Mc log-U[1e5,1e6], "
                        "8-60 SFTs each (ragged), K=%d, auto kernel (Fresnel), FP64 phase + FP32 Kahan sums"
                        % (w.n_templates, K),
            "value": w.n_templates * args.steps / elapsed, "unit": "IP/s", "ms_per_step": 1e3 * elapsed / args.steps,
            "template_sfts": float(np.sum(n_use)),
            "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_SLOTS / 1e12, "unit": "Tslot/s",
                         "frac": achieved / (PEAK_SLOTS / 1e12), "kernel": "scan_kernel", "kernel_ms": k_ms,
                         "alg_slots_per_launch": slots, "alg_slots_per_template_sft": slots / census["pairs"],
                         "bins_by_series": {k: census[k] / census["pairs"] for k in ("w0", "w1", "w3", "table", "stat", "series")},
                         "frac_of_fma_ceiling": (achieved / args.fma_ceiling) if getattr(args, "fma_ceiling", None) else None},
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

    train = {"samples": args.surrogate_samples, "epochs": args.surrogate_epochs, "batch": 4096,
             "targets_s": t_targets, "train_s": t_train, "epoch_loss": [float(v) for v in hist]}
    if n <= 0:
        # training only (no bank to scan)
        s.close()
        return {"workload": "surrogate training only: MLP 3-%dx%d-2 SiLU on %d 3.5PN samples"
                            % (hidden, layers, args.surrogate_samples), "train": train}
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
    z64 = out["zp"].cpu().numpy()
    nz64 = np.sqrt(out["hhp"].cpu().numpy())
    # the same trained parameters evaluated on the BF16 matrix cores
    par = s.get_params()
    lowp = {}
    for mode in ("bf16x3", "bf16"):
        sb = sft.Surrogate(par, hidden=hidden, layers=layers, judge_tol=1e-4, inference=mode, **SUR_CFG)
        t_b = timed(sft.make_opts(waveform="surrogate", surrogate=sb, **common))
        fl_b = out["flags"].cpu().numpy()
        dz = np.abs(out["zp"].cpu().numpy() - z64).max(axis=1) / np.maximum(np.abs(z64).max(axis=1), nz64)
        lowp[mode] = {"value": n / t_b, "ms_per_step": 1e3 * t_b, "over_fp64_network": t_sur / t_b,
                      "fallback_frac": float(np.mean((fl_b & sft.FLAG_SURROGATE_FALLBACK) > 0)),
                      "mismatch_median": float(np.median(out["mismatch"].cpu().numpy())),
                      "max_dz_vs_fp64_network": float(dz.max()), "median_dz_vs_fp64_network": float(np.median(dz))}
        print("surrogate scan, %s network: %.1f ms, fallback %.4f, max dz %.2e" % (
            mode, 1e3 * t_b, lowp[mode]["fallback_frac"], dz.max()), file=sys.stderr, flush=True)
        sb.close()
    evals = n * w.n_sft
    mlp_flop = evals * 2 * 2 * (3 * hidden + (layers - 1) * hidden * hidden + hidden * 2)
    res = {"workload": "tiny data (256 SFTs x 64 s, 1 detector, K=4 Dirichlet, FP32 Kahan sums), %d templates "
                       "Mc~U[1.19,1.21] q~U[1,2]; MLP 3-%dx%d-2 SiLU trained on %d 3.5PN samples"
                       % (n, hidden, layers, args.surrogate_samples),
           "value": n / t_sur, "unit": "IP/s", "ms_per_step": 1e3 * t_sur, "steps": steps,
           "plain_newton_value": n / t_plain, "pn35_value": n / t_pn,
           "surrogate_over_plain": t_plain / t_sur, "surrogate_over_pn35": t_pn / t_sur,
           "network_evals_per_step": evals, "network_fp64_tflop_per_step": mlp_flop / 1e12,
           "fallback_frac": fb, "judge_tol": 1e-4, "network_bf16": lowp,
           "mismatch_median": float(np.median(mm)), "mismatch_p99": float(np.quantile(mm, 0.99)),
           "train": train}
    print("surrogate scan %.1f ms (plain %.2f ms, 3.5PN %.2f ms), fallback %.4f" % (
        1e3 * t_sur, 1e3 * t_plain, 1e3 * t_pn, fb), file=sys.stderr, flush=True)
    s.close()
    return res


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, out, n_sample, K, kernel):
    """The FP64 oracle on a seeded template sample of the same workload, host cores; the same
    oracle on one thread; the brute-force time-domain product of the tiny workload (the paper's
    non-optimised comparator, Sec. V.C); the oracle on a sample of the space-based bank."""
    import oracle
    from paper_2502_11823_amd import synth
    idx = np.sort(np.random.default_rng(12345).choice(w.n_templates, n_sample, replace=False))
    b = w.subset(idx)
    od = oracle.SFTData(w.t_start, w.n_samples, w.t_sft, w.k_lo, w.x_bins, w.psd, w.fplus, w.fcross)
    threads = oracle.get_threads()
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
    # one thread, 12 templates
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.scan(od, b["mc"][:12], b["t_c"][:12], phi_c=b["phi_c"][:12], K=K, kernel=oracle.K_AUTO,
                a_plus=1.0, a_cross=1.0)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    # brute force on the tiny workload: the template at all 524,288 samples and sum x h / sigma^2
    n_bf = 32
    t = synth.tiny(seed=1, n_templates=n_bf)
    tt = np.arange(t.n_sft * t.n_samples) * (t.t_sft / t.n_samples)
    t0 = time.perf_counter()
    for m in range(n_bf):
        wv = oracle.waveform(t.bank["mc"][m], t.bank["t_c"][m], 0.0, tt)
        h = wv[:, 0] * np.cos(wv[:, 1])
        oracle.td_product(t.series, h, 1.0)
    dtb = time.perf_counter() - t0
    # the oracle on the space-based bank (60 SFTs of 2 days, K = 32, ragged ranges)
    ws = synth.space(seed=3, n_templates=200_000)
    n_sp = 4000
    si = np.sort(np.random.default_rng(54321).choice(ws.n_templates, n_sp, replace=False))
    bs = ws.subset(si)
    ods = oracle.SFTData(ws.t_start, ws.n_samples, ws.t_sft, ws.k_lo, ws.x_bins, ws.psd, ws.fplus, ws.fcross)
    t0 = time.perf_counter()
    oracle.scan(ods, bs["mc"], bs["t_c"], phi_c=bs["phi_c"], a_first=bs["a_first"], a_last=bs["a_last"], K=32,
                kernel=oracle.K_AUTO, a_plus=1.0, a_cross=1.0)
    dts = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "IP/s", "cores": threads, "kind": "oracle",
            "sample": "%d seeded templates of the same bank, all %d SFTs, FP64 oracle (C, OpenMP), %.1f s"
                      % (n_sample, w.n_sft, dt),
            "max_rel_err_vs_gpu": err, "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
            "single_thread": {"value": 12 / dt1, "unit": "IP/s", "sample": "12 templates, %.1f s" % dt1},
            "brute_force_tiny": {"value": n_bf / dtb, "unit": "IP/s",
                                 "sample": "%d templates of the tiny workload, each the waveform at all %d samples "
                                           "and sum x h / sigma^2 (numpy + oracle), %.1f s" % (n_bf, tt.size, dtb)},
            "space_bank": {"value": n_sp / dts, "unit": "IP/s",
                           "sample": "%d seeded templates of the space-based bank (8-60 SFTs, K = 32), %.1f s"
                                     % (n_sp, dts)}}


if __name__ == "__main__":
    main()
