"""GPU parity of the accuracy-study path (Sec. IV): the template's strain at every sample,
the direct integral <d,h>, SFTs of segments whose length is not a power of two (the paper's SFT
lengths), and r = 1 - sqrt(([d,h]) / <d,h>) against the oracle on a reduced configuration;
then the paper's qualitative claims on the full pilot configurations (Sec. IV.B, IV.C)."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_11823_amd import sft, study  # noqa: E402


@pytest.mark.parametrize("wf", ["newton", "pn35"])
def test_waveform_series_matches_oracle(wf):
    mc, q, t_c = 1.2188, 1.3, 5000.0
    t0, dt, n = 100.0, 1 / 40.0, 190_000        # up to 4850 s, before t_c
    g = np.random.default_rng(1)
    fp_h = g.uniform(-1, 1, n)
    fx_h = g.uniform(-1, 1, n)
    fp, fx = torch.as_tensor(fp_h, device="cuda"), torch.as_tensor(fx_h, device="cuda")
    h, qv = sft.waveform_series(mc, t_c, t0, dt, n, waveform=wf, q=q, phi_c=0.3, fplus=fp, fcross=fx,
                                a_plus=1.1, a_cross=0.7, quantities=True)
    h, qv = h.cpu().numpy(), qv.cpu().numpy()
    idx = np.arange(0, n, 997)
    t = t0 + idx * dt
    ref = oracle.waveform(mc, t_c, 0.3, t, q=q, wf=oracle.WF_PN35 if wf == "pn35" else oracle.WF_NEWTON)
    for k, tol in ((0, 1e-12), (2, 1e-12), (3, 1e-11), (4, 1e-10)):
        assert np.max(np.abs(qv[idx, k] - ref[:, k]) / np.abs(ref[:, k])) <= tol, k
    assert np.max(np.abs(qv[idx, 1] - ref[:, 1])) <= 1e-12 * np.abs(ref[:, 1]).max()
    want = ref[:, 0] * (fp_h[idx] * 1.1 * np.cos(ref[:, 1]) + fx_h[idx] * 0.7 * np.sin(ref[:, 1]))
    assert np.max(np.abs(h[idx] - want)) <= 1e-9 * np.abs(ref[:, 0]).max()
    # past coalescence the strain is zero
    h2 = sft.waveform_series(mc, 120.0, 100.0, dt, 2000, waveform=wf, q=q).cpu().numpy()
    assert np.all(h2[int(20 / dt) + 1:] == 0) and np.all(np.isfinite(h2))


def test_td_product_matches_oracle():
    g = np.random.default_rng(2)
    n, dt, S = 3_000_001, 1 / 64.0, 0.37
    x, y = g.normal(size=n), g.normal(size=n)
    got = sft.td_product(torch.as_tensor(x, device="cuda"), torch.as_tensor(y, device="cuda"), dt, S)
    want = oracle.td_product(2 * x / S, y, dt)        # dt sum d_j y_j with whitened d = 2 x / S
    assert abs(got - want) <= 1e-12 * math.sqrt(n) * dt * 2 / S
    again = sft.td_product(torch.as_tensor(x, device="cuda"), torch.as_tensor(y, device="cuda"), dt, S)
    assert again == got


@pytest.mark.parametrize("n", [4240, 5004, 2922])
def test_make_sfts_non_power_of_two(n):
    g = np.random.default_rng(n)
    dt, n_seg, S = 1 / 40.0, 6, 0.05
    x = g.normal(size=(1, n * n_seg + 11))
    x[0, 3 * n + 5] = np.nan
    bins, psd, keep = sft.make_sfts(torch.as_tensor(x, device="cuda"), n, dt, 3, n // 2 - 2, 0, s_white=S)
    torch.cuda.synchronize()
    bins, psd, keep = bins.cpu().numpy()[0], psd.cpu().numpy()[0], keep.cpu().numpy()[0]
    assert keep.tolist() == [1, 1, 1, 0, 1, 1]
    ref = oracle.make_sfts(np.nan_to_num(x[0]), n, n_seg, dt)
    for a in range(n_seg):
        if not keep[a]:
            assert not bins[a].any()
            continue
        r = ref[a, 3:3 + n // 2 - 2]
        assert np.max(np.abs(bins[a] - r)) <= 1e-12 * np.abs(ref[a]).max()
        assert np.all(psd[a] == S)
    with pytest.raises(sft.SFTError):       # the PSD estimate needs a power of two
        sft.make_sfts(torch.as_tensor(x, device="cuda"), n, dt, 3, 100, 10)


def _oracle_r(res, waveform, dks, span_scale):
    """The same reduced study with the oracle: its waveform series, its SFTs (own DFT), its scan."""
    c = study.CASES[res["case"]]
    fs = c["fs"]
    dt = 1 / fs
    n0 = res["n0"]
    delta = list(res["config"])[0]
    n = res["config"][delta]["n_samples"]
    t = np.arange(n0) * dt
    t_c = res["t_c"]
    w = oracle.waveform(res["mc"], t_c, 0.0, t, q=res["q"], wf=oracle.WF_PN35 if waveform == "pn35" else oracle.WF_NEWTON)
    ab = np.cos(2 * np.pi * t / c["period"]) + np.sin(2 * np.pi * t / c["period"])
    h = np.where(np.isfinite(w[:, 0]), w[:, 0] * ab * (np.cos(w[:, 1]) + np.sin(w[:, 1])), 0.0)
    S = 2 * dt
    hh = oracle.td_product(2 * h / S, h, dt)
    n_sft = n0 // n
    xb = oracle.make_sfts(h, n, n_sft, dt)
    tm = (np.arange(n_sft) + 0.5) * n * dt
    abm = np.cos(2 * np.pi * tm / c["period"]) + np.sin(2 * np.pi * tm / c["period"])
    od = oracle.SFTData(np.arange(n_sft) * n * dt, n, n * dt, 0, xb, np.full(xb.shape, S), abm, abm)
    out = {}
    for dk in dks:
        r = oracle.scan(od, [res["mc"]], [t_c], q=[res["q"]], K=dk // 2, kernel=oracle.K_AUTO,
                        wf=oracle.WF_PN35 if waveform == "pn35" else oracle.WF_NEWTON, a_plus=1.0, a_cross=1.0)
        dh = r["zp"][0].real + r["zx"][0].imag
        out[dk] = 1 - math.sqrt(dh / hh)
    return out, hh


def test_r_study_matches_oracle_on_a_reduced_configuration():
    dks = (8, 20, 32)
    res = study.r_study("bns", deltas=(3.0,), dks=dks, span_scale=0.004, log=lambda m: print(m, flush=True))
    ro, hh = _oracle_r(res, "pn35", dks, 0.004)
    print("reduced BNS (%d samples, %d SFTs): GPU %s oracle %s" % (res["n0"], res["config"][3.0]["n_sft"],
          res["r"][3.0], ro), flush=True)
    assert abs(res["hh"] - hh) <= 1e-9 * hh
    for dk in dks:
        assert abs(res["r"][3.0][dk] - ro[dk]) <= 1e-6


def test_r_study_paper_claims():
    """Sec. IV.B: delta <~ 3 and Delta k >~ 20 give r < 1% for the BNS; Sec. IV.C: r ~ 1% at
    delta = 3, Delta k ~ 30 for the massive BBH (here with the 3.5PN inspiral for the BNS and
    the leading-order chirp for the massive BBH instead of IMRPhenomT)."""
    log = lambda m: print(m, flush=True)
    bns = study.r_study("bns", dks=(8, 20, 32, 64), log=log)
    mbbh = study.r_study("mbbh", dks=(8, 20, 30, 64), log=log)
    for d in (3.0, 2.0, 1.0):
        print("bns  delta %.0f: T %g s, %d SFTs, r %s" % (d, bns["config"][d]["T_sft"], bns["config"][d]["n_sft"],
              {k: "%.4f" % v for k, v in bns["r"][d].items()}), flush=True)
        print("mbbh delta %.0f: T %g s, %d SFTs, r %s" % (d, mbbh["config"][d]["T_sft"], mbbh["config"][d]["n_sft"],
              {k: "%.4f" % v for k, v in mbbh["r"][d].items()}), flush=True)
    for d in (3.0, 2.0, 1.0):
        for dk in (20, 32, 64):
            assert bns["r"][d][dk] < 0.01
    assert mbbh["r"][3.0][30] < 0.02
    # smaller delta (shorter SFTs) and wider windows lose less
    assert bns["r"][1.0][64] <= bns["r"][3.0][64] + 1e-4
    assert bns["r"][3.0][8] > bns["r"][3.0][64]


def test_tsft_regions_of_the_ground_bank():
    """T_SFT per chirp-mass region (Sec. III.F): the heaviest mass of a region sets its largest
    fddot at the band's top frequency, so heavier regions get shorter SFTs; each region's T_SFT
    is Eq. max_tsft of the oracle's fddot at that mass and frequency."""
    regions = study.tsft_regions([1.0, 1.1, 1.2, 1.3, 1.4, 1.5], 16.0, 1.0, waveform="newton")
    T = [r[3] for r in regions]
    assert all(a > b for a, b in zip(T[:-1], T[1:]))
    for lo, hi, fdd, t in regions:
        tau = study.time_of_frequency(hi, 1.0, 16.0, "newton")
        ref = oracle.waveform(hi, 0.0, 0.0, [tau])[0]
        assert abs(ref[2] - 16.0) < 1e-9 * 16.0
        assert abs(fdd - ref[4]) <= 1e-9 * ref[4]
        assert t == math.floor(oracle.tsft_max(1.0, ref[4]))
