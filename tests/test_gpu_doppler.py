"""GPU parity of the Doppler form (Sec. III.B: chirp at the emission time t + r.n/c of each SFT
row's detector, f and fdot through dt_s/dt; reading R26) against the FP64 oracle, element by
element, with the bars of the plain scan (parity_helpers.compare)."""
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

SITES = [(0.81, -1.58), (0.53, -2.08), (0.76, 0.18)]   # latitude, longitude [rad]


def _ground_eph(w):
    tm = w.t_start + 0.5 * w.t_sft
    eph = np.empty((w.n_sft, 9))
    for d, (lat, lon) in enumerate(SITES):
        m = w.det == d
        eph[m] = synth.ground_ephemeris(tm[m], lat, lon)
    return eph


def _sky(n, seed):
    g = np.random.default_rng(seed)
    return synth.sky_vector(g.uniform(0, 2 * np.pi, n), np.arcsin(g.uniform(-1, 1, n)))


def test_doppler_ground_three_sites():
    w = synth.ground(seed=6, n_templates=600, n_slots=96, n_det=3, k_lo=40, k_hi=470, t_end_pad=300.0)
    eph = _ground_eph(w)
    w.bank["sky"] = _sky(600, 1)
    data = sft.SFTData.from_workload(w, storage="f32")
    data.set_ephemeris(eph)
    kw = dict(K=8, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    g = gpu_scan(data, w.bank, **kw)
    o = orc_scan(w, w.bank, eph=eph, sky=w.bank["sky"], **kw)
    compare(g, o, label="doppler ground")
    # with the F-statistic as well
    g = gpu_scan(data, w.bank, fstat=True, **kw)
    o = orc_scan(w, w.bank, eph=eph, sky=w.bank["sky"], fstat=True, **kw)
    compare(g, o, label="doppler+fstat ground")
    compare_fstat(g, o, label="doppler+fstat ground 2F")
    # the Doppler shift matters: the same bank without it differs by far more than the bar
    wp = dict(w.bank)
    wp.pop("sky")
    o0 = orc_scan(w, wp, **kw)
    assert np.max(np.abs(o0["zp"] - o["zp"]) / np.sqrt(o["hhp"])) > 1e-2


def test_doppler_fp64_fresnel_ground():
    """The Doppler form with FP64 Fresnel weights (and the F-statistic) on the three-site
    ground data, against the oracle within 1e-9."""
    w = synth.ground(seed=6, n_templates=300, n_slots=96, n_det=3, k_lo=40, k_hi=470, t_end_pad=300.0)
    eph = _ground_eph(w)
    w.bank["sky"] = _sky(300, 2)
    data = sft.SFTData.from_workload(w, storage="f64")
    data.set_ephemeris(eph)
    kw = dict(K=8, kernel="auto", precision="fp64", a_plus=1.0, a_cross=1.0)
    for fs in (False, True):
        g = gpu_scan(data, w.bank, fstat=fs, **kw)
        o = orc_scan(w, w.bank, eph=eph, sky=w.bank["sky"], fstat=fs, **kw)
        compare(g, o, label="doppler fp64 fresnel fstat=%d" % fs, tol_z=1e-9, tol_rho=1e-9, tol_hh=1e-9)
        if fs:
            compare_fstat(g, o, tol_f=1e-9, tol_hh=1e-9, label="doppler fp64 fresnel 2F")


def test_doppler_fp64_fast_orbit_and_zero_limit():
    w = synth.tiny(seed=1, n_templates=400)
    tm = w.t_start + 0.5 * w.t_sft
    data = sft.SFTData.from_workload(w, storage="f64")
    kw = dict(K=4, kernel="dirichlet", precision="fp64")
    plain = gpu_scan(data, {k: v for k, v in w.bank.items()}, **kw)
    w.bank["sky"] = _sky(400, 2)
    # zero ephemeris: bit for bit the plain scan (one detector: the groups do not change)
    data.set_ephemeris(np.zeros((w.n_sft, 9)))
    z = gpu_scan(data, w.bank, **kw)
    for k in ("zp", "zx", "hhp", "rho", "flags"):
        assert np.array_equal(z[k], plain[k]), k
    eph = synth.circular_orbit(tm, 0.05, 3000.0, 0.3, 0.2)
    data.set_ephemeris(eph)
    g = gpu_scan(data, w.bank, **kw)
    o = orc_scan(w, w.bank, eph=eph, sky=w.bank["sky"], **kw)
    e = compare(g, o, label="doppler fp64 tiny")
    assert e < 1e-9


def test_doppler_space_k32_annual_orbit():
    w = synth.space(n_templates=999)
    eph = synth.circular_orbit(w.t_start + 0.5 * w.t_sft, synth.AU_S, synth.YEAR, 0.0, synth.OBLIQUITY)
    w.bank["sky"] = _sky(999, 3)
    data = sft.SFTData.from_workload(w, storage="f32")
    data.set_ephemeris(eph)
    kw = dict(K=32, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    g = gpu_scan(data, w.bank, **kw)
    o = orc_scan(w, w.bank, eph=eph, sky=w.bank["sky"], **kw)
    compare(g, o, label="doppler space")


def test_doppler_rejections():
    w = synth.ground(seed=8, n_templates=64, n_slots=16, n_det=1, k_lo=40, k_hi=470, t_end_pad=300.0)
    w.bank["sky"] = _sky(64, 4)
    data = sft.SFTData.from_workload(w, storage="f32")
    bt = sft.bank_to_device(w.bank)
    with pytest.raises(sft.SFTError) as ei:          # no ephemeris yet
        sft.template_bank_scan(data, bt, sft.make_opts(K=8))
    assert ei.value.status == -1
    data.set_ephemeris(np.zeros((w.n_sft, 9)))
    with pytest.raises(sft.SFTError) as ei:
        sft.template_bank_scan(data, bt, sft.make_opts(K=8, waveform="pn35"))
    assert ei.value.status == -5
    bad = np.zeros((w.n_sft, 9))
    bad[3, 4] = np.nan
    with pytest.raises(sft.SFTError):
        data.set_ephemeris(bad)
