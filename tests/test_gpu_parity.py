"""GPU parity: the HIP bank scan against the FP64 oracle, element by element.

Metric (per template, per polarisation): e = |z_gpu - z_orc| / max(|z_orc|, sqrt(hh_orc)),
the error in units of the noise standard deviation of <n,h> when |z| is small and
relative otherwise; likewise |rho_gpu - rho_orc| / max(rho_orc, 1) for the SNR (rho is
itself in noise units).  Bars: e <= 1e-6 on z, <= 1e-5 on rho, relative <= 1e-6 on hh,
flags bit-exact.  Templates whose window
centre sits within 1e-9 bins of a rounding tie (both sides decide k0 in FP64 but
by different formulae) are excluded from the flag/z comparison and counted.
"""
import numpy as np
import pytest

import oracle
from paper_2502_11823_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_11823_amd import sft  # noqa: E402

from parity_helpers import KERN, compare, compare_fstat, gpu_scan, orc_scan  # noqa: E402,F401


# ----------------------------------------------------------------------------- fixtures
@pytest.fixture(scope="module")
def tiny():
    """The tiny workload with a Newtonian injection at SNR 20 (Mc = 1.2, t_c = 16984 s)."""
    w = synth.tiny(seed=1)
    dt = w.t_sft / w.n_samples
    t = np.arange(w.n_sft * w.n_samples) * dt
    wf = oracle.waveform(1.2, 16984.0, 0.0, t)
    h = wf[:, 0] * np.cos(wf[:, 1])
    h *= 20.0 / np.sqrt(np.sum(h**2) / w.sigma**2)
    w.x_bins = synth.sfts_from_series(w.series + h, w.n_samples, w.n_sft, dt)
    return w


@pytest.fixture(scope="module")
def ground_small():
    return synth.ground(seed=6, n_templates=777, n_slots=96, n_det=3, k_lo=40, k_hi=470,
                        t_end_pad=300.0)


# ----------------------------------------------------------------------------- tiny workload
def test_tiny_fp64_dirichlet_full_bank(tiny):
    data = sft.SFTData.from_workload(tiny, storage="f64")
    kw = dict(K=4, kernel="dirichlet", precision="fp64")
    g = gpu_scan(data, tiny.bank, **kw)
    o = orc_scan(tiny, tiny.bank, **kw)
    e = compare(g, o, label="tiny fp64")
    assert e < 1e-9                       # FP64 throughout: far inside the bar
    # the loudest template sits at the injected chirp mass (the K = 4 Dirichlet window
    # loses part of the SNR-20 injection in the late, fast-drifting SFTs)
    m = int(np.argmax(g["rho"]))
    assert abs(tiny.bank["mc"][m] - 1.2) < 1e-3 and g["rho"][m] > 8


@pytest.mark.parametrize("precision", ["fp32_kahan", "fp32_naive"])
def test_tiny_fp32_dirichlet_full_bank(tiny, precision):
    data = sft.SFTData.from_workload(tiny, storage="f32")
    kw = dict(K=4, kernel="dirichlet", precision=precision)
    compare(gpu_scan(data, tiny.bank, **kw), orc_scan(tiny, tiny.bank, **kw), label="tiny " + precision)


def test_tiny_bf16_storage_is_reported_not_exact(tiny):
    """BF16 data bins carry ~3e-3 relative rounding: the error is measured, not hidden."""
    data = sft.SFTData.from_workload(tiny, storage="bf16")
    kw = dict(K=4, kernel="dirichlet", precision="fp32_kahan")
    g = gpu_scan(data, tiny.bank, **kw)
    o = orc_scan(tiny, tiny.bank, **kw)
    e = np.abs(g["zp"] - o["zp"]) / np.maximum(np.abs(o["zp"]), np.sqrt(o["hhp"]))
    print("tiny bf16: max e = %.3e" % e.max())
    assert 1e-5 < e.max() < 3e-2
    assert np.array_equal(g["flags"], o["flags"])


# ----------------------------------------------------------------------------- Fresnel / multi-detector
@pytest.mark.parametrize("K,kernel", [(8, "auto"), (5, "auto"), (8, "fresnel"), (4, "dirichlet")])
def test_ground_small_multidetector(ground_small, K, kernel):
    """3 detectors, gaps, coloured non-stationary PSD, antenna patterns; 777 templates
    (three 256-lane tiles and a ragged tail), compile-time and run-time K."""
    w = ground_small
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=K, kernel=kernel, precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    compare(gpu_scan(data, w.bank, **kw), orc_scan(w, w.bank, **kw), label="ground-small K=%d %s" % (K, kernel))


@pytest.mark.parametrize("K,kernel", [(8, "auto"), (32, "fresnel")])
def test_shuffled_bank_mixes_staged_and_gathered_windows(ground_small, K, kernel):
    """The bank in a seeded random order: the lanes of a wavefront hold chirp masses across
    [1.0, 1.5], so their windows spread over tens of bins.  Groups whose window union exceeds
    the wavefront's LDS stage take the checked gather path, the others the stage, and the
    series-tier bounds are set by the widest lanes."""
    w = ground_small
    p = np.random.default_rng(17).permutation(w.n_templates)
    bank = {k: np.ascontiguousarray(v[p]) for k, v in w.bank.items()}
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=K, kernel=kernel, precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    g = gpu_scan(data, bank, **kw)
    compare(g, orc_scan(w, bank, **kw), label="shuffled K=%d %s" % (K, kernel))
    # the same templates in bank order give the same results up to FP32 summation order
    gs = gpu_scan(data, w.bank, **kw)
    e = np.abs(g["zp"] - gs["zp"][p]) / np.maximum(np.abs(gs["zp"][p]), np.sqrt(gs["hhp"][p]))
    assert e.max() < 1e-6


@pytest.mark.parametrize("n_det,pad", [(3, 1.5e5), (1, 1.5e5), (3, 100.0), (1, 100.0), (3, 60.0), (1, 60.0)])
def test_largest_window_full_band(n_det, pad):
    """K = 64 (the largest window), band from DC to Nyquist.  Far from merger (pad 1.5e5 s,
    k0 ~ 43-49, drift ~0.004 bins) the windows reach below DC and take the mirrored bins, and
    the central bin takes the small-drift series; near merger (pad 100 s, k0 ~ 250-725, drifts
    up to 75 bins, inside beta/2 + 8 <= K) the lanes of a wavefront spread by tens of bins, so
    some groups fit the LDS stage and others fall back to gathers.  Pad 60 s: the last SFTs
    drift by up to ~134 bins, past beta/2 + 8 <= K, where the window no longer holds the track
    (the result is still the same truncated sum on both sides, with its flags)."""
    with np.errstate(divide="ignore"):   # the coloured PSD is infinite at DC: that bin is masked
        w = synth.ground(seed=12, n_templates=300, n_slots=40, n_det=n_det, k_lo=0, k_hi=2049,
                         t_end_pad=pad, mc_lo=1.2, mc_hi=1.5)
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=sft.K_MAX, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    compare(gpu_scan(data, w.bank, **kw), orc_scan(w, w.bank, **kw),
            label="K=64 full band, %d det, pad %g s" % (n_det, pad))


@pytest.mark.parametrize("K,n_det", [(8, 3), (8, 1), (32, 1), (32, 3)])
def test_small_drift_central_bin(K, n_det):
    """Far from merger (pad 1.5e5 s: drift ~0.004 bins, k0 ~ 43-49) every lane with
    |delta| <= 1/8 takes its central bin from the small-drift series; K = 8 and K = 32 run
    the compile-time windows (the one-row K = 32 kernel among them), with one and three rows
    per timestamp group."""
    w = synth.ground(seed=13, n_templates=300, n_slots=40, n_det=n_det, k_lo=1, k_hi=400,
                     t_end_pad=1.5e5, mc_lo=1.2, mc_hi=1.5)
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=K, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    compare(gpu_scan(data, w.bank, **kw), orc_scan(w, w.bank, **kw),
            label="small drift K=%d, %d det" % (K, n_det))


def test_fresnel_large_drift():
    """Templates close to merger: beta = fdot T^2 up to tens of bins, K = 32."""
    w = synth.ground(seed=8, n_templates=300, n_slots=40, n_det=1, k_lo=20, k_hi=1500,
                     t_end_pad=15.0, mc_lo=1.3, mc_hi=1.5)
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=32, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=0.0)
    o = orc_scan(w, w.bank, **kw)
    compare(gpu_scan(data, w.bank, **kw), o, label="large drift")


# ----------------------------------------------------------------------------- edge cases
def _edge_workload(k_lo, k_hi):
    w = synth.ground(seed=9, n_templates=333, n_slots=50, n_det=2, k_lo=k_lo, k_hi=k_hi,
                     t_end_pad=-400.0, mc_lo=1.0, mc_hi=1.5)
    g0 = np.random.default_rng(1)
    w.bank["a_first"] = g0.integers(0, w.n_sft // 2, w.n_templates).astype(np.int32)
    w.bank["a_last"] = (w.bank["a_first"] + g0.integers(-3, w.n_sft, w.n_templates)).astype(np.int32)
    return w


def test_edges_tau_band_ragged_empty():
    """t_c inside the data (tau <= 0 SFTs), windows leaving the band, ragged and empty
    SFT ranges, a masked PSD bin and a single template.  The stored band [100, 300)
    cuts the norm bins of many SFTs whose windows still reach into the band, so the
    error scale is the norm computed from the same PSD over the full band."""
    w = _edge_workload(100, 300)
    w.psd[5, 17] = 0.0
    w.psd[6, 30] = np.inf
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=8, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0, delta_max=1e-3)
    g = gpu_scan(data, w.bank, **kw)
    o = orc_scan(w, w.bank, **kw)
    wide = _edge_workload(20, 2049)
    assert np.array_equal(wide.psd[:, 80:280][:, [i for i in range(200) if i not in (17, 30)]],
                          w.psd[:, [i for i in range(200) if i not in (17, 30)]])
    ow = orc_scan(wide, w.bank, **kw)
    assert np.any(o["flags"] & oracle.F_TAU_NONPOSITIVE)
    assert np.any(o["flags"] & oracle.F_OUT_OF_BAND)
    assert np.any(o["flags"] & oracle.F_EMPTY)
    assert np.any(o["flags"] & oracle.F_TAYLOR_INVALID)
    compare(g, o, label="edges", noise_scale=(ow["hhp"], ow["hhx"]))
    one = {k: v[:1] for k, v in w.bank.items()}
    compare(gpu_scan(data, one, **kw), orc_scan(w, one, **kw), label="single template")


def test_dc_mirror_and_nonfinite():
    """A band starting at DC: windows reaching k < 0 use conj(d~[-k]); NaN data -> NONFINITE."""
    w = synth.tiny(seed=4, n_templates=64, n_sft=16)
    w.bank["t_c"][:] = 1.4e9                 # f ~ 0.05 Hz: kappa ~ 3 bins at T = 64 s
    w.bank["mc"][:] = np.linspace(1.0, 1.6, 64)
    kw = dict(K=6, kernel="dirichlet", precision="fp64")
    data = sft.SFTData.from_workload(w, storage="f64")
    compare(gpu_scan(data, w.bank, **kw), orc_scan(w, w.bank, **kw), label="dc mirror")
    xb = w.x_bins.copy()
    xb[3, :] = np.nan
    w2 = synth.tiny(seed=4, n_templates=64, n_sft=16)
    w2.x_bins = xb
    w2.bank = w.bank
    d2 = sft.SFTData.from_workload(w2, storage="f64")
    g = gpu_scan(d2, w.bank, **kw)
    o = orc_scan(w2, w.bank, **kw)
    assert np.all(g["flags"] & oracle.F_NONFINITE) and np.array_equal(g["flags"], o["flags"])


def test_zero_templates_and_determinism(ground_small):
    w = ground_small
    data = sft.SFTData.from_workload(w, storage="f32")
    opts = sft.make_opts(K=8, kernel="auto", a_plus=1.0, a_cross=1.0)
    bt = sft.bank_to_device(w.bank)
    out = sft.alloc_out(1)
    sft.template_bank_scan(data, bt, opts, out=out, n=0)       # no-op
    r1 = sft.template_bank_scan(data, bt, opts)
    r2 = sft.template_bank_scan(data, bt, opts)
    torch.cuda.synchronize()
    for k in r1:
        assert torch.equal(r1[k], r2[k]), k


def test_inner_product_single_call(ground_small):
    w = ground_small
    data = sft.SFTData.from_workload(w, storage="f32")
    opts = sft.make_opts(K=8, kernel="auto", a_plus=1.0, a_cross=1.0)
    m = 123
    r = sft.inner_product(data, w.bank["mc"][m], w.bank["t_c"][m], opts=opts)
    one = {k: v[m:m + 1] for k, v in w.bank.items()}
    o = orc_scan(w, one, K=8, kernel="auto", a_plus=1.0, a_cross=1.0)
    e = abs(r["zp"] - o["zp"][0]) / max(abs(o["zp"][0]), np.sqrt(o["hhp"][0]))
    assert e < 1e-6 and r["flags"] == o["flags"][0]
    assert abs(r["rho"] / o["rho"][0] - 1) < 1e-5


# ----------------------------------------------------------------------------- full ground workload
@pytest.mark.slow
def test_ground_full_size_sampled():
    """The full ground-based workload (3 x 3891 SFTs, 1e5 templates, K = 8, automatic
    kernel, FP32 compensated) in the bench's launch configuration, checked on a seeded
    sample of templates the oracle computes one by one."""
    w = synth.ground(seed=2)
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=8, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    g = gpu_scan(data, w.bank, **kw)
    idx = np.sort(np.random.default_rng(0).choice(w.n_templates, 24, replace=False))
    idx = np.concatenate([[0, w.n_templates - 1], idx])
    o = orc_scan(w, w.subset(idx), **kw)
    compare(g, o, idx=idx, label="ground full (sampled)")
    assert np.all(np.isfinite(g["rho"])) and np.all(g["flags"] == 0)


# ----------------------------------------------------------------------------- launch shapes, autotuner, graphs
@pytest.mark.parametrize("block,nchunk,persistent", [(64, 1, 0), (128, 7, 1), (256, 3, 1), (256, 40, 0), (64, 200, 1)])
def test_tunings_match_oracle_and_repeat_bitwise(ground_small, block, nchunk, persistent):
    """Every launch shape (workgroup size, chunking of timestamp groups, plain or
    persistent work-queue grid) gives oracle parity and bitwise-repeatable results."""
    w = ground_small
    data = sft.SFTData.from_workload(w, storage="f32")
    n_groups = len(np.unique(w.t_start))
    sft.set_tuning(data, block=block, chunk_groups=max(1, -(-n_groups // nchunk)), persistent=persistent)
    kw = dict(K=8, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    g1 = gpu_scan(data, w.bank, **kw)
    g2 = gpu_scan(data, w.bank, **kw)
    for k in g1:
        assert np.array_equal(g1[k], g2[k]), k
    compare(g1, orc_scan(w, w.bank, **kw), label="tuning %d/%d/%d" % (block, nchunk, persistent))


def test_autotune_then_scan(ground_small):
    w = ground_small
    data = sft.SFTData.from_workload(w, storage="f32")
    opts = sft.make_opts(K=8, kernel="auto", a_plus=1.0, a_cross=1.0)
    bt = sft.bank_to_device(w.bank)
    best, ms = sft.autotune(data, bt, opts, reps=1)
    assert best.block in (64, 128, 256) and best.chunk_groups >= 1 and ms > 0
    assert sft.get_tuning(data).as_dict() == best.as_dict()
    kw = dict(K=8, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    compare(gpu_scan(data, w.bank, **kw), orc_scan(w, w.bank, **kw), label="autotuned")


@pytest.mark.parametrize("persistent", [0, 1])
def test_graph_plan_replays(ground_small, persistent):
    """A captured plan replays bitwise-identically to the eager scan with the same
    launch shape, several times with eager work and synchronisations in between, and
    follows changes of the bank contents behind its fixed pointers."""
    w = ground_small
    data = sft.SFTData.from_workload(w, storage="f32")
    n_groups = len(np.unique(w.t_start))
    sft.set_tuning(data, block=128, chunk_groups=max(1, n_groups // 5), persistent=persistent)
    opts = sft.make_opts(K=8, kernel="auto", a_plus=1.0, a_cross=1.0)
    bt = sft.bank_to_device(w.bank)
    eager = sft.template_bank_scan(data, bt, opts)
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in eager.items()}
    plan = sft.Plan(data, bt, opts)
    for rep in range(4):
        out = plan.launch()
        torch.cuda.synchronize()
        for k in eager:
            assert torch.equal(out[k], eager[k]), (rep, k)
        junk = torch.randn(1 << 16, device="cuda").sum()     # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
    # new bank contents behind the same pointers
    bt["mc"].mul_(1.001)
    out = plan.launch()
    torch.cuda.synchronize()
    ref = sft.template_bank_scan(data, bt, opts)
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(out[k], ref[k]), k
    plan.close()


# ----------------------------------------------------------------------------- ragged space-based bank
def test_space_ragged_small_all_templates():
    """Ragged SFT ranges (each template its last 8..60 of 60 two-day SFTs), Fresnel drift
    up to ~30 bins, K = 32 (run-time K) with the DC mirror, every template checked."""
    w = synth.space(n_templates=999)
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=32, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0, delta_max=3.0)
    o = orc_scan(w, w.bank, **kw)
    assert np.all(o["flags"] == 0)
    for tune in [(256, 0, 1), (64, 3, 0)]:
        sft.set_tuning(data, block=tune[0], chunk_groups=tune[1], persistent=tune[2])
        compare(gpu_scan(data, w.bank, **kw), o, label="space ragged %s" % (tune,))


@pytest.mark.slow
def test_space_ragged_full_size_sampled():
    """The full ragged space-based bank (2e5 templates) in one launch, sampled."""
    w = synth.space()
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=32, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0, delta_max=3.0)
    g = gpu_scan(data, w.bank, **kw)
    idx = np.sort(np.random.default_rng(3).choice(w.n_templates, 48, replace=False))
    idx = np.concatenate([[0, w.n_templates - 1], idx])
    compare(g, orc_scan(w, w.subset(idx), **kw), idx=idx, label="space full (sampled)")


# ----------------------------------------------------------------------------- precision sweep
@pytest.mark.slow
def test_precision_sweep_tiny_data_1e5_templates(tiny):
    """The tiny workload's data (with its SNR-20 injection) against 1e5 templates, four
    arithmetic variants, every template compared with the FP64 oracle.  FP64 sums and
    FP32 compensated sums meet the 1e-6 bar; plain FP32 sums and BF16-stored bins are
    measured and reported."""
    bank = synth.uniform_bank(100_000, 1.19, 1.21, 16984.0, 4242, n_sft=tiny.n_sft)
    kw = dict(K=4, kernel="dirichlet")
    o = orc_scan(tiny, bank, **kw)
    ok = o["tie"] > 1e-9
    rows = []
    for storage, prec in [("f64", "fp64"), ("f32", "fp32_naive"), ("f32", "fp32_kahan"), ("bf16", "fp32_kahan")]:
        data = sft.SFTData.from_workload(tiny, storage=storage)
        g = gpu_scan(data, bank, precision=prec, **kw)
        e = np.abs(g["zp"] - o["zp"]) / np.maximum(np.abs(o["zp"]), np.sqrt(o["hhp"]))
        er = np.abs(g["rho"] - o["rho"]) / np.maximum(o["rho"], 1.0)
        e, er = e[ok], er[ok]
        rows.append((storage, prec, e.max(), np.percentile(e, 99), np.median(e), er.max()))
        print("precision %-4s %-10s e: max %.3e p99 %.3e median %.3e | rho: max %.3e"
              % (storage, prec, e.max(), np.percentile(e, 99), np.median(e), er.max()))
        assert np.array_equal(g["flags"][ok], o["flags"][ok])
    assert rows[0][2] < 1e-9
    assert rows[2][2] <= 1e-6 and rows[2][5] <= 1e-5
    assert rows[1][2] < 1e-5
    assert rows[3][2] < 3e-2


@pytest.mark.parametrize("workload", ["ground_small", "space"])
def test_precision_sweep_fresnel_data(ground_small, workload):
    """The four arithmetic variants on Fresnel data: the three-detector ground bank (K = 8,
    AUTO kernel, drifts of a few bins) and the ragged space-based bank (K = 32, drifts up to
    ~30 bins, DC mirror), every template against the FP64 oracle.  FP64 (Fresnel weights
    from FP64 Fresnel integrals) within 1e-9, FP32 compensated sums within the 1e-6 bar, plain
    FP32 sums within 1e-5, BF16-stored bins reported (bound 3e-2)."""
    if workload == "space":
        w = synth.space(n_templates=999)
        kw = dict(K=32, kernel="auto", a_plus=1.0, a_cross=1.0)
    else:
        w = ground_small
        kw = dict(K=8, kernel="auto", a_plus=1.0, a_cross=1.0)
    o = orc_scan(w, w.bank, **kw)
    ok = o["tie"] > 1e-9
    rows = []
    for storage, prec in [("f64", "fp64"), ("f32", "fp32_naive"), ("f32", "fp32_kahan"), ("bf16", "fp32_kahan")]:
        data = sft.SFTData.from_workload(w, storage=storage)
        g = gpu_scan(data, w.bank, precision=prec, **kw)
        e = np.abs(g["zp"] - o["zp"]) / np.maximum(np.abs(o["zp"]), np.sqrt(o["hhp"]))
        er = np.abs(g["rho"] - o["rho"]) / np.maximum(o["rho"], 1.0)
        e, er = e[ok], er[ok]
        rows.append((storage, prec, e.max(), er.max()))
        print("%s precision %-4s %-10s e: max %.3e median %.3e | rho: max %.3e"
              % (workload, storage, prec, e.max(), np.median(e), er.max()))
        assert np.array_equal(g["flags"][ok], o["flags"][ok])
        data.close()
    assert rows[0][2] < 1e-9 and rows[0][3] < 1e-9
    assert rows[2][2] <= 1e-6 and rows[2][3] <= 1e-5
    assert rows[1][2] < 1e-5
    assert rows[3][2] < 3e-2


def test_fp64_fresnel_forms(ground_small):
    """FP64 Fresnel weights in every scan form that has them: the 3.5PN waveform (the
    four-row group kernel), the F-statistic, and the start reference (both waveforms),
    against the oracle within 1e-9 on z, rho, the norms and 2F."""
    w = ground_small
    data = sft.SFTData.from_workload(w, storage="f64")
    tight = dict(tol_z=1e-9, tol_rho=1e-9, tol_hh=1e-9)
    base = dict(K=8, kernel="auto", precision="fp64", a_plus=1.0, a_cross=1.0)
    bank = _with_q(w.bank, 9)
    for label, extra, fstat in [("pn35", dict(waveform="pn35"), False),
                                ("fstat", dict(), True),
                                ("start newton", dict(t_ref="start"), False),
                                ("start pn35", dict(t_ref="start", waveform="pn35"), False)]:
        kw = dict(base, **extra)
        g = gpu_scan(data, bank, fstat=fstat, **kw)
        o = orc_scan(w, bank, fstat=fstat, **kw)
        compare(g, o, label="fp64 fresnel " + label, **tight)
        if fstat:
            compare_fstat(g, o, tol_f=1e-9, tol_hh=1e-9, label="fp64 fresnel 2F")


# ----------------------------------------------------------------------------- 3.5PN waveform
def _with_q(bank, seed):
    b = dict(bank)
    b["q"] = np.random.default_rng(seed).uniform(1.0, 2.0, b["mc"].size)
    return b


@pytest.mark.parametrize("K,kernel", [(8, "auto"), (5, "fresnel")])
def test_pn35_multidetector(ground_small, K, kernel):
    """The 3.5PN closed-form waveform (mass ratio per template) against the oracle's
    independently written series, three detectors, Fresnel kernels."""
    w = ground_small
    bank = _with_q(w.bank, 5)
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=K, kernel=kernel, precision="fp32_kahan", a_plus=1.0, a_cross=1.0, waveform="pn35",
              delta_max=0.05)
    o = orc_scan(w, bank, **kw)
    compare(gpu_scan(data, bank, **kw), o, label="pn35 ground-small K=%d %s" % (K, kernel))


def test_pn35_fp64_tiny(tiny):
    bank = _with_q(tiny.bank, 6)
    data = sft.SFTData.from_workload(tiny, storage="f64")
    kw = dict(K=4, kernel="dirichlet", precision="fp64", waveform="pn35")
    e = compare(gpu_scan(data, bank, **kw), orc_scan(tiny, bank, **kw), label="pn35 tiny fp64")
    assert e < 1e-8


# ----------------------------------------------------------------------------- paper-shaped banks
@pytest.mark.parametrize("name", ["bns", "mbbh"])
def test_paper_shaped_banks_sampled(name):
    """Banks shaped like the paper's timing runs: BNS (6384 SFTs of 73 s, K = 50, drift up to
    a few bins near 10 Hz) and MBBH (1540 SFTs of 2502 s, K = 15, windows centred a quarter bin
    above DC so that most bins reflect through DC).  Full bank on the GPU, a seeded sample of
    templates against the oracle."""
    w = synth.paper_shape(name, n_templates=1000)
    K = int(w.opts["K"])
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=K, kernel="auto", precision="fp32_kahan")
    g = gpu_scan(data, w.bank, **kw)
    idx = np.sort(synth.rng(21).choice(w.n_templates, 24, replace=False))
    o = orc_scan(w, w.subset(idx), **kw)
    compare(g, o, idx=idx, label="paper-shaped " + name)


# ----------------------------------------------------------------------------- remaining instantiations
def test_fp32_naive_fresnel_ground(ground_small):
    """Plain FP32 sums with the Fresnel kernels (groups of three rows, K = 8 compile-time window)."""
    data = sft.SFTData.from_workload(ground_small, storage="f32")
    kw = dict(K=8, kernel="auto", precision="fp32_naive", a_plus=1.0, a_cross=1.0)
    compare(gpu_scan(data, ground_small.bank, **kw), orc_scan(ground_small, ground_small.bank, **kw),
            label="ground-small fp32 naive")


def test_bf16_fresnel_multirow_is_reported_not_exact(ground_small):
    """BF16 data bins with the Fresnel kernels and three rows per group: the 8-bit mantissa of
    the data (relative 4e-3) bounds the error, which is measured and reported; flags are exact."""
    data = sft.SFTData.from_workload(ground_small, storage="bf16")
    kw = dict(K=8, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    g = gpu_scan(data, ground_small.bank, **kw)
    o = orc_scan(ground_small, ground_small.bank, **kw)
    e = np.abs(g["zp"] - o["zp"]) / np.maximum(np.abs(o["zp"]), np.sqrt(o["hhp"]))
    print("ground-small bf16 fresnel: max e = %.3e, median %.3e" % (e.max(), np.median(e)))
    assert 1e-5 < e.max() < 3e-2
    assert np.array_equal(g["flags"], o["flags"])
    # the norm does not read the data bins: FP32 accuracy
    assert np.max(np.abs(g["hhp"] - o["hhp"]) / o["hhp"]) < 1e-6


def test_newton_four_detectors_per_group():
    """Four detectors sharing every start time: the width-4 group kernel (weights shared by four
    rows) with gaps, K = 8 and a run-time window."""
    w = synth.ground(seed=21, n_templates=400, n_slots=64, n_det=4, k_lo=40, k_hi=470, t_end_pad=300.0)
    data = sft.SFTData.from_workload(w, storage="f32")
    for K in (8, 6):
        kw = dict(K=K, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
        compare(gpu_scan(data, w.bank, **kw), orc_scan(w, w.bank, **kw), label="4 detectors K=%d" % K)


@pytest.mark.parametrize("K", [8, 32])
def test_pn35_fp32_one_row_fresnel(K):
    """The 3.5PN waveform in FP32 sums on one detector (one row per group), Fresnel kernels."""
    w = synth.ground(seed=22, n_templates=300, n_slots=96, n_det=1, k_lo=20, k_hi=700, t_end_pad=200.0)
    bank = _with_q(w.bank, 9)
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=K, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0, waveform="pn35")
    compare(gpu_scan(data, bank, **kw), orc_scan(w, bank, **kw), label="pn35 one row K=%d" % K)


# ----------------------------------------------------------------------------- start reference
def test_start_reference_fp64_tiny(tiny):
    """The paper's own expansion point (Sec. III.B: Taylor expansion at the SFT start, Fig. 1):
    FP64 Dirichlet on the tiny data against the oracle's start form."""
    data = sft.SFTData.from_workload(tiny, storage="f64")
    kw = dict(K=4, kernel="dirichlet", precision="fp64", t_ref="start", delta_max=1.0)
    e = compare(gpu_scan(data, tiny.bank, **kw), orc_scan(tiny, tiny.bank, **kw), label="tiny fp64 start")
    assert e < 1e-9


@pytest.mark.parametrize("waveform,K", [("newton", 8), ("pn35", 8), ("newton", 24)])
def test_start_reference_fresnel_ground(ground_small, waveform, K):
    """Start reference with the Fresnel kernels, three rows per group, both closed-form
    waveforms, compile-time and run-time windows; the validity flag uses the lever T."""
    bank = _with_q(ground_small.bank, 11)
    data = sft.SFTData.from_workload(ground_small, storage="f32")
    kw = dict(K=K, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0, waveform=waveform,
              t_ref="start", delta_max=0.05)
    g = gpu_scan(data, bank, **kw)
    o = orc_scan(ground_small, bank, **kw)
    compare(g, o, label="ground-small start %s K=%d" % (waveform, K))
    assert np.any(o["flags"] & sft.FLAG_TAYLOR_INVALID)
    # the two references differ (second order of the Taylor model), by far more than the bar
    m = gpu_scan(data, bank, **dict(kw, t_ref="mid"))
    assert np.max(np.abs(m["zp"] - g["zp"]) / np.sqrt(g["hhp"])) > 1e-3


def test_issue_probe_rates():
    """The VALU issue-rate probe runs and orders its instructions as the hardware does: a
    quarter-rate transcendental below the plain FP32 FMA, FP64 FMA below FP32 FMA."""
    per_clk = {op: sft.probe_issue_rate(op) / (256 * 2.4e9) for op in sft.PROBE}
    print("issue probe, wave-instructions per clock per CU:", per_clk, flush=True)
    assert all(0.05 < v < 8.0 for v in per_clk.values())
    assert per_clk["v_rcp_f32"] < per_clk["v_fma_f32"]
    assert per_clk["v_fma_f64"] < per_clk["v_fma_f32"]
