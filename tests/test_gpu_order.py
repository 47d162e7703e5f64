"""Bank order on the device: with the tuning's order "track" the scan sorts the bank by its
frequency track, scans it in that order and writes every result back to its template's given
position.  A shuffled bank then has oracle parity element by element at its given positions
(the bars of parity_helpers.compare), every bank field (mass ratio, phase, SFT range, sky
vector) travels with its template, graph plans and the autotuner keep their contracts, and a
shuffled bank of the full ground size runs at the speed of the sorted one."""
import time

import numpy as np
import pytest

from paper_2502_11823_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_11823_amd import sft  # noqa: E402

from parity_helpers import compare, compare_fstat, gpu_scan, orc_scan  # noqa: E402

KW = dict(K=8, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)


def _small(seed=6, n=777):
    return synth.ground(seed=seed, n_templates=n, n_slots=96, n_det=3, k_lo=40, k_hi=470, t_end_pad=300.0)


def _shuffled(bank, seed):
    p = np.random.default_rng(seed).permutation(len(bank["mc"]))
    return {k: np.ascontiguousarray(v[p]) for k, v in bank.items()}


def test_shuffled_ground_bank_parity_at_given_positions():
    w = _small()
    g = np.random.default_rng(11)
    bank = dict(w.bank)
    bank["phi_c"] = g.uniform(0, 2 * np.pi, w.n_templates)
    bank["t_c"] = bank["t_c"] + g.uniform(-200.0, 200.0, w.n_templates)
    sb = _shuffled(bank, 12)
    data = sft.SFTData.from_workload(w, storage="f32")
    sft.set_tuning(data, order="track")
    assert sft.get_tuning(data).as_dict()["order"] == "track"
    g1 = gpu_scan(data, sb, **KW)
    g2 = gpu_scan(data, sb, **KW)
    for k in g1:
        assert np.array_equal(g1[k], g2[k]), k            # the sorted order is deterministic
    compare(g1, orc_scan(w, sb, **KW), label="shuffled ground, track order")
    # the same templates in the given order agree within the bars (rounding-level differences)
    sft.set_tuning(data, order="given")
    g0 = gpu_scan(data, sb, **KW)
    assert np.array_equal(g0["flags"], g1["flags"])
    assert np.max(np.abs(g0["zp"] - g1["zp"]) / np.sqrt(g0["hhp"])) < 1e-6
    assert np.max(np.abs(g0["hhp"] - g1["hhp"]) / g0["hhp"]) < 1e-6


def test_shuffled_ragged_pn35_bank_keeps_every_field():
    """Mass ratio, phase and a ragged SFT range per template (3.5PN waveform) travel with it."""
    w = _small(seed=7, n=500)
    g = np.random.default_rng(21)
    n = w.n_templates
    bank = dict(w.bank)
    bank["q"] = g.uniform(1.0, 3.0, n)
    bank["phi_c"] = g.uniform(0, 2 * np.pi, n)
    af = g.integers(0, w.n_sft // 2, n).astype(np.int32)
    bank["a_first"] = af
    bank["a_last"] = np.minimum(af + g.integers(10, w.n_sft, n), w.n_sft - 1).astype(np.int32)
    sb = _shuffled(bank, 22)
    data = sft.SFTData.from_workload(w, storage="f32")
    sft.set_tuning(data, order="track")
    kw = dict(KW, waveform="pn35")
    compare(gpu_scan(data, sb, **kw), orc_scan(w, sb, **kw), label="shuffled ragged pn35, track order")


def test_shuffled_doppler_fstat_bank():
    """Sky vectors (three values per template) travel with their templates; F-statistic too."""
    from test_gpu_doppler import _ground_eph, _sky
    w = _small(seed=6, n=600)
    eph = _ground_eph(w)
    bank = dict(w.bank)
    bank["sky"] = _sky(600, 1)
    sb = _shuffled(bank, 31)
    data = sft.SFTData.from_workload(w, storage="f32")
    data.set_ephemeris(eph)
    sft.set_tuning(data, order="track")
    g = gpu_scan(data, sb, fstat=True, **KW)
    o = orc_scan(w, sb, eph=eph, sky=sb["sky"], fstat=True, **KW)
    compare(g, o, label="shuffled doppler+fstat, track order")
    compare_fstat(g, o, label="shuffled doppler+fstat 2F")


def test_plan_with_track_order():
    """A plan fixes the order at creation and gathers the bank at every launch: it replays
    bitwise like the eager track-order scan, and stays correct when the contents change."""
    w = _small()
    sb = _shuffled(w.bank, 41)
    data = sft.SFTData.from_workload(w, storage="f32")
    sft.set_tuning(data, order="track")
    opts = sft.make_opts(**KW)
    bt = sft.bank_to_device(sb)
    eager = sft.template_bank_scan(data, bt, opts)
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in eager.items()}
    plan = sft.Plan(data, bt, opts)
    for rep in range(3):
        out = plan.launch()
        torch.cuda.synchronize()
        for k in eager:
            assert torch.equal(out[k], eager[k]), (rep, k)
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
    # new contents behind the same pointers: the bank reversed (the plan's order is now stale)
    for k in bt:
        bt[k].copy_(torch.flip(bt[k], dims=[0]).clone())
    out = plan.launch()
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["zp"] = res["zp"][:, 0] + 1j * res["zp"][:, 1]
    res["zx"] = res["zx"][:, 0] + 1j * res["zx"][:, 1]
    res["flags"] = res["flags"].astype(np.uint32)
    rb = {k: np.ascontiguousarray(v[::-1]) for k, v in sb.items()}
    compare(res, orc_scan(w, rb, **KW), label="plan, track order, changed contents")
    plan.close()


def test_autotune_weighs_the_track_order():
    w = _small()
    sb = _shuffled(w.bank, 51)
    data = sft.SFTData.from_workload(w, storage="f32")
    best, ms = sft.autotune(data, sft.bank_to_device(sb), sft.make_opts(**KW), reps=1)
    assert best.order in (0, 1) and ms > 0
    assert sft.get_tuning(data).as_dict() == best.as_dict()
    compare(gpu_scan(data, sb, **KW), orc_scan(w, sb, **KW), label="autotuned (order %d)" % best.order)


def test_noalloc_scan_keeps_the_given_order():
    """The allocation-free scan ignores the order and matches the given-order scan bitwise."""
    w = _small()
    sb = _shuffled(w.bank, 61)
    data = sft.SFTData.from_workload(w, storage="f32")
    opts = sft.make_opts(**KW)
    bt = sft.bank_to_device(sb)
    ref = sft.template_bank_scan(data, bt, opts)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in ref.items()}
    sft.set_tuning(data, order="track")
    out = sft.template_bank_scan_noalloc(data, bt, opts, sft.alloc_out(w.n_templates))
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(out[k], ref[k]), k


def test_bad_order_is_rejected():
    w = _small(n=10)
    data = sft.SFTData.from_workload(w, storage="f32")
    with pytest.raises(sft.SFTError):
        sft.set_tuning(data, order=2)


def _median_ms(data, bt, opts, out, reps=5):
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sft.template_bank_scan(data, bt, opts, out=out)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def test_shuffled_full_ground_bank_runs_at_sorted_speed():
    """1e5 templates on the three-detector ground data: the shuffled bank in track order
    (sort included) takes at most 5% longer than the sorted bank in its given order."""
    t0 = time.perf_counter()
    w = synth.ground(seed=2)
    data = sft.SFTData.from_workload(w, storage="f32")
    opts = sft.make_opts(**KW)
    bt = sft.bank_to_device(w.bank)
    st = sft.bank_to_device(_shuffled(w.bank, 71))
    out = sft.alloc_out(w.n_templates)
    print("setup %.1f s" % (time.perf_counter() - t0), flush=True)
    sft.template_bank_scan(data, bt, opts, out=out)       # warm-up
    t_sorted = _median_ms(data, bt, opts, out)
    t_shuf_given = _median_ms(data, st, opts, out)
    sft.set_tuning(data, order="track")
    sft.template_bank_scan(data, st, opts, out=out)
    t_shuf_track = _median_ms(data, st, opts, out)
    print("sorted bank %.3f ms, shuffled given order %.3f ms, shuffled track order %.3f ms"
          % (t_sorted, t_shuf_given, t_shuf_track), flush=True)
    assert t_shuf_track <= 1.05 * t_sorted
