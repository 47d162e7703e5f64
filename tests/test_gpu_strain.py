"""GPU parity of SFT creation from raw strain and of the per-SFT PSD estimate (Sec. III.B,
Eq. d_SFT; reading R27) against the FP64 oracle, and of the scan over SFTs made that way.

Bars: SFT bins to 1e-12 of the segment's largest bin (FP64 FFTs in different orders), PSD
estimates to 1e-12 relative (the same block median up to rounding), keep flags bit-exact;
the scan over the device-made data handle with the bars of the plain scan."""
import numpy as np
import pytest

import oracle
from paper_2502_11823_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_11823_amd import sft  # noqa: E402

from parity_helpers import compare  # noqa: E402


def _check(x, n, dt, k_lo, n_bins, w):
    xt = torch.as_tensor(x, device="cuda")
    bins, psd, keep = sft.make_sfts(xt, n, dt, k_lo, n_bins, w)
    torch.cuda.synchronize()
    bins, psd, keep = bins.cpu().numpy(), psd.cpu().numpy(), keep.cpu().numpy()
    for d in range(x.shape[0]):
        ob, op, ok = oracle.strain_sfts(x[d], n, dt, w, k_lo, n_bins)
        assert np.array_equal(keep[d], ok)
        scale = np.abs(ob).max(axis=1, keepdims=True) + 1e-300
        eb = np.max(np.abs(bins[d] - ob) / scale)
        ep = np.max(np.abs(psd[d] - op) / np.maximum(op, 1e-300))
        print("n=%d det %d: %d segments (%d gaps), max e(bins)=%.2e e(psd)=%.2e"
              % (n, d, ok.size, int(np.sum(ok == 0)), eb, ep), flush=True)
        assert eb <= 1e-12 and ep <= 1e-12
    return keep


@pytest.mark.parametrize("n,w", [(16, 3), (256, 10), (4096, 25), (16384, 40)])
def test_make_sfts_matches_oracle(n, w):
    g = np.random.default_rng(n)
    dt = 1.0 / 128.0
    n_seg = max(4, min(40, (1 << 17) // n))
    x = g.normal(size=(2, n * n_seg + 7)) * np.array([[1.0], [2.5]])
    x[0, 2 * n + 3] = np.nan                  # a gap in detector 0
    x[1, (n_seg - 1) * n] = np.inf            # the last segment of detector 1
    keep = _check(x, n, dt, 0, n // 2 + 1, w)  # full band: DC and Nyquist included
    assert keep[0, 2] == 0 and keep[1, -1] == 0 and keep.sum() == keep.size - 2
    _check(x, n, dt, n // 8, n // 4, w)        # an inner band


@pytest.mark.parametrize("n", [16, 2048, 16384])
def test_make_sfts_power_of_two_white_psd(n):
    """A known white level (no estimate) on the FFT path: the band bins as with the estimate,
    the PSD the given level everywhere, a gap zeroed; two calls in a row, the second with the
    segment length's cached twiddle tables."""
    g = np.random.default_rng(n + 1)
    dt, S = 1.0 / 64.0, 0.25
    n_seg = max(3, min(12, (1 << 16) // n))
    x = g.normal(size=(1, n * n_seg))
    x[0, n + 1] = np.nan
    xt = torch.as_tensor(x, device="cuda")
    ref = oracle.make_sfts(np.nan_to_num(x[0]), n, n_seg, dt)
    for _ in range(2):
        bins, psd, keep = sft.make_sfts(xt, n, dt, 1, n // 2 - 1, 0, s_white=S)
        torch.cuda.synchronize()
        bins, psd, keep = bins.cpu().numpy()[0], psd.cpu().numpy()[0], keep.cpu().numpy()[0]
        assert keep[1] == 0 and keep.sum() == n_seg - 1
        assert not bins[1].any() and not psd[1].any()
        for a in np.nonzero(keep)[0]:
            assert np.max(np.abs(bins[a] - ref[a, 1:n // 2])) <= 1e-12 * np.abs(ref[a]).max()
            assert np.all(psd[a] == S)


def test_scan_over_device_made_sfts():
    """Three detectors of white noise at 128 Hz with a Newtonian injection of network SNR ~20
    (about 1 per SFT, the regime of long-duration signals), 32 s SFTs made and whitened on the
    device (gaps in one detector), then scanned; the oracle makes its own SFTs and PSD estimates
    from the same series and scans them.  (The bar is in noise units, reading R14: an injection
    loud within single SFTs raises the FP32 rounding of its signal-dominated terms above that
    scale for templates next to it.)"""
    g = np.random.default_rng(11)
    fs, n, n_slots, n_det = 128.0, 4096, 96, 3
    dt = 1.0 / fs
    N = n * n_slots
    t = np.arange(N) * dt
    t_c = N * dt + 300.0
    wf = oracle.waveform(1.25, t_c, 0.0, t)
    # each detector sees F+ A cos(phi) + Fx A sin(phi) with its own daily antenna patterns (the
    # projector with A+ = Ax = 1 that the scan uses)
    ph = 2 * np.pi * t[None, :] / 86400 + 2 * np.pi * np.arange(n_det)[:, None] / 3
    h = wf[:, 0] * (np.cos(ph) * np.cos(wf[:, 1]) + np.sin(ph) * np.sin(wf[:, 1]))
    x = g.normal(size=(n_det, N)) + h * 20.0 / np.sqrt(np.sum(h**2))
    x[2, 10 * n:12 * n] = np.nan              # two missing SFTs in detector 2
    k_lo, n_bins, w = 32, 480, 25
    tm = np.arange(n_slots) * n * dt + 0.5 * n * dt
    fp = np.stack([np.cos(2 * np.pi * tm / 86400 + 2 * np.pi * d / 3) for d in range(n_det)])
    fx = np.stack([np.sin(2 * np.pi * tm / 86400 + 2 * np.pi * d / 3) for d in range(n_det)])
    data = sft.SFTData.from_strain(torch.as_tensor(x, device="cuda"), n, dt, k_lo, n_bins, w, fplus=fp, fcross=fx)
    assert data.n_sft == n_det * n_slots - 2
    # the oracle's own SFTs and PSDs of the kept segments
    rows_b, rows_p, rows_t, rows_fp, rows_fx = [], [], [], [], []
    for d in range(n_det):
        ob, op, ok = oracle.strain_sfts(x[d], n, dt, w, k_lo, n_bins)
        for a in np.nonzero(ok)[0]:
            rows_b.append(ob[a]); rows_p.append(op[a]); rows_t.append(a * n * dt)
            rows_fp.append(fp[d, a]); rows_fx.append(fx[d, a])
    od = oracle.SFTData(np.array(rows_t), n, n * dt, k_lo, np.array(rows_b), np.array(rows_p),
                        np.array(rows_fp), np.array(rows_fx))
    bank = synth.uniform_bank(300, 1.0, 1.5, t_c, 5, n_sft=data.n_sft)
    bank["mc"][-1] = 1.25                      # the injected chirp mass, as the last template
    from parity_helpers import gpu_scan
    kw = dict(K=8, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    gres = gpu_scan(data, bank, **kw)
    ores = oracle.scan(od, bank["mc"], bank["t_c"], phi_c=bank["phi_c"], a_first=bank["a_first"],
                       a_last=bank["a_last"], K=8, kernel=oracle.K_AUTO, a_plus=1.0, a_cross=1.0)
    compare(gres, ores, label="scan over device-made SFTs")
    # the template of the injected chirp mass is the loudest, near the injected SNR of 20
    assert int(np.argmax(gres["rho"])) == 299 and gres["rho"][299] > 12
