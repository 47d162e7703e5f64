"""GPU parity of the F-statistic form (Sec. II.B, Eq. det_long and the maximisation over the
four amplitudes c_nu; reading R25) against the FP64 oracle, element by element.

Bars (parity_helpers.compare and compare_fstat): z and the norms as in the plain scan; the
cross norm to 1e-6 of sqrt(hh+ hhx); 2F to 2e-5 in noise units; flags (the degenerate bit
included) bit-exact.
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

from parity_helpers import compare, compare_fstat, gpu_scan, orc_scan  # noqa: E402


def _both(w, bank, data, **kw):
    g = gpu_scan(data, bank, fstat=True, **kw)
    o = orc_scan(w, bank, fstat=True, **kw)
    return g, o


def test_fstat_ground_three_detectors_all_templates():
    w = synth.ground(seed=6, n_templates=777, n_slots=96, n_det=3, k_lo=40, k_hi=470, t_end_pad=300.0)
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=8, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    g, o = _both(w, w.bank, data, **kw)
    compare(g, o, label="fstat ground z")
    compare_fstat(g, o, label="fstat ground 2F")
    # z of the F-statistic form are bitwise those of the plain scan
    p = gpu_scan(data, w.bank, **kw)
    assert np.array_equal(p["zp"], g["zp"]) and np.array_equal(p["zx"], g["zx"])
    assert np.array_equal(p["flags"], g["flags"] & ~np.uint32(sft.FLAG_FSTAT_DEGENERATE))
    assert np.all(np.isfinite(g["twoF"])) and np.median(g["twoF"]) < 20


def test_fstat_one_detector_long_and_short_spans():
    """One detector over 1.5 days (amplitudes resolved) and over a few SFTs (degenerate:
    the dominant-pattern branch), ragged ranges."""
    w = synth.ground(seed=7, n_templates=200, n_slots=4096, n_det=1, k_lo=40, k_hi=470, t_end_pad=300.0)
    g_ = np.random.default_rng(4)
    n = w.n_sft
    first = np.where(np.arange(200) % 2 == 0, 0, g_.integers(0, n - 40, 200)).astype(np.int32)
    last = np.where(np.arange(200) % 2 == 0, n - 1, first + g_.integers(2, 30, 200)).astype(np.int32)
    w.bank["a_first"], w.bank["a_last"] = first, last
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=8, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    idx = np.arange(0, 200, 3)
    b = w.subset(idx)
    g, o = _both(w, b, data, **kw)
    compare(g, o, label="fstat 1-det z")
    compare_fstat(g, o, label="fstat 1-det 2F")
    deg = (o["flags"] & oracle.F_FSTAT_DEGENERATE) != 0
    assert deg.any() and (~deg).any()


def test_fstat_fp64_tiny_with_antenna_patterns():
    w = synth.tiny(seed=1, n_templates=300)
    tm = w.t_start + 0.5 * w.t_sft
    w.fplus = np.cos(2 * np.pi * tm / 9000.0)
    w.fcross = 0.7 * np.sin(2 * np.pi * tm / 9000.0) + 0.2
    data = sft.SFTData.from_workload(w, storage="f64")
    kw = dict(K=4, kernel="dirichlet", precision="fp64")
    g, o = _both(w, w.bank, data, **kw)
    compare(g, o, label="fstat fp64 z")
    e = compare_fstat(g, o, label="fstat fp64 2F")
    assert e < 1e-9


def test_fstat_space_ragged_k32():
    w = synth.space(n_templates=999)
    data = sft.SFTData.from_workload(w, storage="f32")
    kw = dict(K=32, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    g, o = _both(w, w.bank, data, **kw)
    compare(g, o, label="fstat space z")
    compare_fstat(g, o, label="fstat space 2F")


def test_fstat_plan_and_noalloc_and_rejections():
    w = synth.ground(seed=8, n_templates=3000, n_slots=64, n_det=3, k_lo=40, k_hi=470, t_end_pad=300.0)
    data = sft.SFTData.from_workload(w, storage="f32")
    opts = sft.make_opts(K=8, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    bt = sft.bank_to_device(w.bank)
    ref = sft.template_bank_scan(data, bt, opts, out=sft.alloc_out(3000, fstat=True))
    out = sft.alloc_out(3000, fstat=True)
    plan = sft.Plan(data, bt, opts, out=out)
    for _ in range(3):
        for v in out.values():
            v.fill_(-3)
        plan.launch()
        torch.cuda.synchronize()
        for k in ("twoF", "hhpx", "zp", "flags"):
            assert torch.equal(out[k], ref[k]), k
    plan.close()
    na = sft.template_bank_scan_noalloc(data, bt, opts, sft.alloc_out(3000, fstat=True))
    torch.cuda.synchronize()
    assert torch.allclose(na["twoF"], ref["twoF"], rtol=1e-9, atol=1e-9)
    # unsupported forms are refused
    for bad in (sft.make_opts(K=8, precision="fp32_naive"), sft.make_opts(K=8, waveform="pn35")):
        with pytest.raises(sft.SFTError) as ei:
            sft.template_bank_scan(data, bt, bad, out=sft.alloc_out(3000, fstat=True))
        assert ei.value.status == -5
