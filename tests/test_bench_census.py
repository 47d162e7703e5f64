"""Host logic of the benchmark's work census (the algorithmic FP32 slots behind the roofline
fraction): every window bin of every Fresnel pair is classified exactly once, the central-bin
series class only ever takes bin 0, and the classes respect the window and drift limits."""
import numpy as np
import pytest

import bench

TSUN = 4.925490947641267e-06   # G M_sun / c^3 in seconds


def _bank(n=40, n_groups=200, T=8.0, pad=50.0, seed=3):
    rng = np.random.default_rng(seed)
    mc = rng.uniform(1.0, 1.5, n)
    g_tmid = (np.arange(n_groups) + 0.5) * T
    t_c = np.full(n, g_tmid[-1] + pad) + rng.uniform(0.0, 200.0, n)
    g_rows = rng.integers(1, 4, n_groups)
    return mc, t_c, g_tmid, g_rows, T


@pytest.mark.parametrize("K", [4, 8, 32])
@pytest.mark.parametrize("multi_row", [True, False])
def test_every_window_bin_classified_once(K, multi_row):
    mc, t_c, g_tmid, g_rows, T = _bank()
    ops, c = bench.scan_census(mc, t_c, g_tmid, g_rows, T, K, 0.0, TSUN, multi_row=multi_row, stride=1)
    assert c["dirichlet_pairs"] == 0 and c["pairs"] > 0
    classified = c["w0"] + c["w1"] + c["w3"] + c["table"] + c["series"]
    assert classified == c["pairs"] * (2 * K + 1)
    assert c["series"] <= c["pairs"]          # bin 0 only
    assert c["stat"] <= c["table"]            # a stationary point is a table bin with a sign change
    assert ops > 0


def test_drift_switch_sends_every_pair_to_dirichlet():
    mc, t_c, g_tmid, g_rows, T = _bank()
    _, c = bench.scan_census(mc, t_c, g_tmid, g_rows, T, 8, 1e30, TSUN, stride=1)
    assert c["dirichlet_pairs"] == c["pairs"] > 0
    assert c["w0"] == c["w1"] == c["w3"] == c["table"] == c["series"] == c["stat"] == 0


def test_narrow_window_uses_the_table_for_every_bin():
    mc, t_c, g_tmid, g_rows, T = _bank()
    K = bench.OUTER_MIN_K - 1
    _, c = bench.scan_census(mc, t_c, g_tmid, g_rows, T, K, 0.0, TSUN, stride=1)
    assert c["w0"] == c["w1"] == c["w3"] == 0
    assert c["table"] + c["series"] == c["pairs"] * (2 * K + 1)


def test_series_class_needs_small_drift():
    # close to merger with long SFTs every drift is far above the series bound: no series bins
    mc, t_c, g_tmid, g_rows, T = _bank(n_groups=20, T=16.0, pad=20.0)
    _, c = bench.scan_census(mc, t_c, g_tmid, g_rows, T, 32, 0.0, TSUN, stride=1)
    assert c["series"] == 0 and c["pairs"] > 0
    # far from merger with short SFTs the drift is tiny; the pairs with |delta| <= 1/8 of a bin
    # (a quarter for a uniform delta) take the series
    mc, t_c, g_tmid, g_rows, T = _bank(n_groups=400, T=2.0, pad=1e5)
    _, c = bench.scan_census(mc, t_c, g_tmid, g_rows, T, 8, 0.0, TSUN, stride=1)
    assert 0.05 * c["pairs"] < c["series"] < 0.5 * c["pairs"]


def test_stride_sample_scales_to_the_bank():
    mc, t_c, g_tmid, g_rows, T = _bank(n=256)
    full, cf = bench.scan_census(mc, t_c, g_tmid, g_rows, T, 8, 0.0, TSUN, stride=1)
    samp, cs = bench.scan_census(mc, t_c, g_tmid, g_rows, T, 8, 0.0, TSUN, stride=4)
    assert cs["pairs"] == pytest.approx(cf["pairs"], rel=0.05)
    assert samp == pytest.approx(full, rel=0.05)


def test_fstat_census_adds_the_cross_norm():
    mc, t_c, g_tmid, g_rows, T = _bank()
    plain, c = bench.scan_census(mc, t_c, g_tmid, g_rows, T, 8, 0.0, TSUN, stride=1)
    fs, cf = bench.scan_census(mc, t_c, g_tmid, g_rows, T, 8, 0.0, TSUN, stride=1, fstat=True)
    use = (t_c[:, None] - g_tmid[None, :]) > 0
    rows = float((use * g_rows[None, :]).sum())
    assert cf == c
    assert fs - plain == pytest.approx(rows * bench.OPS_FSTAT_ROW + c["pairs"] * bench.OPS_FSTAT_PAIR)


def test_doppler_census_limits():
    """A zero ephemeris is the one-row census plus the delay arithmetic; a constant delay r.n is
    the one-row census of the bank with t_c - r.n; the rates move the frequency and the drift."""
    mc, t_c, g_tmid, _, T = _bank()
    ones = np.ones(g_tmid.size)
    rng = np.random.default_rng(5)
    sky = rng.normal(size=(mc.size, 3))
    sky /= np.linalg.norm(sky, axis=1, keepdims=True)
    base, c0 = bench.scan_census(mc, t_c, g_tmid, ones, T, 8, 0.0, TSUN, multi_row=False, stride=1)
    eph = np.zeros((g_tmid.size, 9))
    dop, c1 = bench.scan_census(mc, t_c, g_tmid, ones, T, 8, 0.0, TSUN, multi_row=False, stride=1,
                                eph=eph, sky=sky)
    assert c1 == c0
    assert dop - base == pytest.approx(c0["pairs"] * bench.OPS_DOPPLER)
    # a constant delay along x: t_c - r n_x for every template
    r = 3.0
    eph[:, 0] = r
    dop, c2 = bench.scan_census(mc, t_c, g_tmid, ones, T, 8, 0.0, TSUN, multi_row=False, stride=1,
                                eph=eph, sky=sky)
    shifted, c3 = bench.scan_census(mc, t_c - r * sky[:, 0], g_tmid, ones, T, 8, 0.0, TSUN,
                                    multi_row=False, stride=1)
    assert c2 == c3
    assert dop - shifted == pytest.approx(c3["pairs"] * bench.OPS_DOPPLER)
    # a large v.n shifts every frequency: the classification of the bins changes
    eph[:, 0] = 0.0
    eph[:, 3] = 0.3
    _, c4 = bench.scan_census(mc, t_c, g_tmid, ones, T, 8, 0.0, TSUN, multi_row=False, stride=1,
                              eph=eph, sky=np.tile([1.0, 0.0, 0.0], (mc.size, 1)))
    assert c4["pairs"] == c0["pairs"] and c4 != c0
