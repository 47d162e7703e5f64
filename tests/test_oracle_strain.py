"""Pins of the oracle's SFT creation from raw strain and its per-SFT PSD estimate (Sec. III.B,
Eq. d_SFT; reading R27: bias-corrected running median of the SFT's own periodogram), CPU only."""
import math
from fractions import Fraction

import numpy as np


def test_median_bias_closed_forms_and_limit(orc):
    """B(N) is the mean of the middle order statistic of N unit exponentials: 1 for N = 1,
    5/6 for N = 3, 47/60 for N = 5 (sums of reciprocals), and ln 2 (the median of one
    exponential) as N grows; a Monte Carlo mean of sample medians agrees."""
    assert orc.median_bias(0) == 1.0
    assert abs(orc.median_bias(1) - float(Fraction(5, 6))) < 1e-15
    assert abs(orc.median_bias(2) - float(Fraction(47, 60))) < 1e-15
    assert abs(orc.median_bias(5000) - math.log(2)) < 1e-4
    g = np.random.default_rng(3)
    med = np.median(g.exponential(size=(200_000, 51)), axis=1)
    assert abs(med.mean() - orc.median_bias(25)) < 4 * med.std() / math.sqrt(med.size)


def test_running_median_is_the_block_median(orc):
    """Every output is 2 median(block) / (T B) with numpy's median of the 2w+1-bin block,
    centred on k and shifted (not clipped) at both ends of [0, n/2]."""
    g = np.random.default_rng(4)
    n, T, w = 256, 8.0, 7
    pw = g.exponential(size=n // 2 + 1) * np.linspace(1, 3, n // 2 + 1)
    out = orc.psd_running_median(pw, n, T, w, 0, n // 2 + 1)
    B = orc.median_bias(w)
    for k in range(n // 2 + 1):
        s = min(max(k - w, 0), n // 2 - 2 * w)
        assert out[k] == 2 * np.median(pw[s:s + 2 * w + 1]) / (T * B)
    # a sub-band gives the same values
    sub = orc.psd_running_median(pw, n, T, w, 30, 40)
    assert np.array_equal(sub, out[30:70])


def test_strain_sfts_match_numpy_and_gaps(orc):
    """The band bins are dt times numpy's real FFT of each segment; a segment holding a NaN is a
    gap (keep = 0, zero outputs) and does not disturb its neighbours."""
    g = np.random.default_rng(5)
    n, dt, n_seg = 512, 1 / 64.0, 6
    x = g.normal(size=n * n_seg + 100)
    x[3 * n + 17] = np.nan
    bins, psd, keep = orc.strain_sfts(x, n, dt, 10, 20, 100)
    assert keep.tolist() == [1, 1, 1, 0, 1, 1]
    for a in range(n_seg):
        if not keep[a]:
            assert not bins[a].any() and not psd[a].any()
            continue
        ref = dt * np.fft.rfft(x[a * n:(a + 1) * n])
        assert np.allclose(bins[a], ref[20:120], rtol=0, atol=1e-13 * np.abs(ref).max())
        B = orc.median_bias(10)
        pw = np.abs(ref)**2
        want = [2 * np.median(pw[min(max(k - 10, 0), n // 2 - 20):][:21]) / (n * dt * B) for k in range(20, 120)]
        assert np.allclose(psd[a], want, rtol=1e-12)


def test_psd_estimate_is_unbiased_on_white_noise(orc):
    """White Gaussian noise of variance sigma^2 has the one-sided PSD S = 2 sigma^2 dt; the
    estimate averaged over many segments and bins recovers it, while the uncorrected ln 2
    (or no) bias factor misses by more than the statistical error."""
    g = np.random.default_rng(6)
    n, dt, sigma, n_seg, w = 1024, 1 / 128.0, 1.7, 400, 25
    x = sigma * g.normal(size=n * n_seg)
    _, psd, keep = orc.strain_sfts(x, n, dt, w, 50, 400)
    S = 2 * sigma**2 * dt
    est = psd[keep == 1].ravel() / S
    # blocks 51 bins wide, bins 50..449: about 8 independent blocks per segment
    err = est.std() / math.sqrt(8 * n_seg)
    assert abs(est.mean() - 1.0) < 4 * err
    wrong = est * orc.median_bias(w) / math.log(2)
    assert abs(wrong.mean() - 1.0) > 4 * err


def test_study_tsft_is_eq_max_tsft(orc):
    """The study's T_SFT (Eq. max_tsft, floored to whole seconds) is the oracle's, and reproduces
    Table 1 for max fddot = 5e-6 Hz/s^2 (pinned against the paper by P9)."""
    from paper_2502_11823_amd import study
    for delta, want in ((3.0, 106), (2.0, 92), (1.0, 73)):
        assert study.tsft(delta, 5e-6) == want == math.floor(orc.tsft_max(delta, 5e-6))
        assert abs(study.tsft(delta, 5e-6, floor_seconds=False) - orc.tsft_max(delta, 5e-6)) < 1e-12
