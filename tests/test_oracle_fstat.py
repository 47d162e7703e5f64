"""Pins of the oracle's F-statistic (Sec. II.B, Eq. det_long and the maximisation over the
four amplitudes c_nu that follows it; reading R25), CPU only.

The four functions are h_nu = A (a cos phi, b cos phi, a sin phi, b sin phi) with a = F+ and
b = Fx of each SFT row; x_nu = <x, h_nu>, M_nu,mu = <h_nu, h_mu> and
2F = max_c 2 (c.x - c.M.c / 2) = x.M^{-1}.x.  Each pin fixes a different part:
the amplitude assembly (exact time-domain products), the maximisation (a numerical
optimiser), the norm matrix (time-domain products of the h_nu), the physics (recovery of
injected amplitudes built with the paper's c_nu), the noise normalisation (chi^2 with four
degrees of freedom) and the degenerate branch (Eq. det_short's statistic).
"""
import math

import numpy as np
import pytest
import scipy.optimize as so
import scipy.stats as st

from paper_2502_11823_amd import synth


def _c_paper(a_plus, a_cross, phi0, psi):
    """Amplitudes c_nu of Sec. II.B in terms of A+, Ax, the initial phase and polarisation."""
    c2, s2 = math.cos(2 * psi), math.sin(2 * psi)
    cp, sp_ = math.cos(phi0), math.sin(phi0)
    return np.array([a_plus * cp * c2 - a_cross * sp_ * s2,
                     a_plus * cp * s2 + a_cross * sp_ * c2,
                     -a_plus * sp_ * c2 - a_cross * cp * s2,
                     -a_plus * sp_ * s2 + a_cross * cp * c2])


def _block_M(hhp, hhx, hhpx):
    return np.array([[hhp, hhpx, 0, 0], [hhpx, hhx, 0, 0], [0, 0, hhp, hhpx], [0, 0, hhpx, hhx]])


def _x(r):
    return np.array([r["zp"].real, r["zx"].real, r["zp"].imag, r["zx"].imag])


def test_fstat_amplitudes_are_exact_time_domain_products(orc):
    """With all bins and the discrete kernel the SFT sums are exact (P1), so the oracle's 2F
    equals xTD.M^{-1}.xTD with xTD_nu = dt sum_j d_j h_nu(t_j) of the four piecewise-quadratic
    functions of Eq. det_long; a swapped or mis-signed amplitude fails."""
    g = np.random.default_rng(41)
    n, n_sft, dt = 64, 8, 0.5
    T = n * dt
    x = g.normal(size=n * n_sft)
    xb = synth.sfts_from_series(x, n, n_sft, dt)
    psd = np.full(xb.shape, 2.0)
    A = g.uniform(0.5, 2.0, n_sft)
    phi = g.uniform(-50, 50, n_sft)
    f = g.uniform(3, 28, n_sft) / T
    fdot = g.uniform(-4, 4, n_sft) / T**2
    a = g.uniform(-1, 1, n_sft)
    b = g.uniform(-1, 1, n_sft)
    data = orc.SFTData(np.arange(n_sft) * T, n, T, 0, xb, psd, a, b)
    r = orc.ip_params(data, A, phi, f, fdot, K=-1, kernel=orc.K_DISCRETE, fstat=True, full=True)
    hs = np.zeros((4, x.size))
    for al in range(n_sft):
        t = al * T + np.arange(n) * dt
        s = t - (al * T + 0.5 * T)
        Phi = phi[al] + 2 * np.pi * f[al] * s + np.pi * fdot[al] * s * s
        sl = slice(al * n, (al + 1) * n)
        hs[0, sl] = A[al] * a[al] * np.cos(Phi)
        hs[1, sl] = A[al] * b[al] * np.cos(Phi)
        hs[2, sl] = A[al] * a[al] * np.sin(Phi)
        hs[3, sl] = A[al] * b[al] * np.sin(Phi)
    xtd = np.array([orc.td_product(x, h, dt) for h in hs])
    assert np.allclose(_x(r), xtd, rtol=0, atol=1e-11 * np.abs(xtd).max())
    M = _block_M(r["hhp"], r["hhx"], r["hhpx"])
    want = xtd @ np.linalg.solve(M, xtd)
    assert r["flags"] & orc.F_FSTAT_DEGENERATE == 0
    assert abs(r["twoF"] - want) <= 1e-10 * want
    # the cross norm is sum a b A^2 T / S at flat S = 2
    assert abs(r["hhpx"] - np.sum(a * b * A**2 * T / 2.0)) <= 1e-13 * np.sum(np.abs(a * b) * A**2 * T)


def test_fstat_is_the_maximum_over_the_four_amplitudes(orc):
    """2F = 2 max_c (c.x - c.M.c / 2), found here by a quasi-Newton optimiser from c = 0."""
    w = synth.ground(seed=5, n_templates=6, n_slots=40, n_det=3, k_lo=40, k_hi=470, t_end_pad=300.0)
    od = orc.SFTData(w.t_start, w.n_samples, w.t_sft, w.k_lo, w.x_bins, w.psd, w.fplus, w.fcross)
    r = orc.scan(od, w.bank["mc"], w.bank["t_c"], phi_c=w.bank["phi_c"], K=8, kernel=orc.K_AUTO,
                 fstat=True)
    for m in range(6):
        x = np.array([r["zp"][m].real, r["zx"][m].real, r["zp"][m].imag, r["zx"][m].imag])
        M = _block_M(r["hhp"][m], r["hhx"][m], r["hhpx"][m])
        s = math.sqrt(r["hhp"][m])
        # in units where M is O(1)
        xs, Ms = x / s, M / s**2
        res = so.minimize(lambda c: -(c @ xs - 0.5 * c @ Ms @ c), np.zeros(4),
                          jac=lambda c: -(xs - Ms @ c), method="BFGS", options={"gtol": 1e-12})
        assert r["flags"][m] & orc.F_FSTAT_DEGENERATE == 0
        assert abs(r["twoF"][m] - 2 * (-res.fun)) <= 1e-8 * max(r["twoF"][m], 1.0)


def _chirp_network(orc, n_det=2, n_slots=48, period=8000.0, seed=3):
    """Two detectors, white noise level sigma = 1 at 32 Hz, 64 s SFTs, and the antenna
    functions a_d(t) = cos(W t + th_d), b_d(t) = 0.7 sin(W t + th_d) + 0.2 (a fast
    modulation period so that the amplitudes are well resolved over 3072 s)."""
    fs, T = 32.0, 64.0
    n = int(fs * T)
    dt = 1.0 / fs
    t = np.arange(n * n_slots) * dt
    W = 2 * np.pi / period
    th = [0.3, 2.1, 4.0][:n_det]
    mc, t_c = 1.2, n_slots * T + 2000.0
    wf = orc.waveform(mc, t_c, 0.0, t)
    amp, phase = wf[:, 0], wf[:, 1]
    hs = []
    for d in range(n_det):
        a = np.cos(W * t + th[d])
        b = 0.7 * np.sin(W * t + th[d]) + 0.2
        hs.append(np.stack([amp * a * np.cos(phase), amp * b * np.cos(phase),
                            amp * a * np.sin(phase), amp * b * np.sin(phase)]))
    tmid = np.arange(n_slots) * T + 0.5 * T
    rows_a = np.concatenate([np.cos(W * tmid + th[d]) for d in range(n_det)])
    rows_b = np.concatenate([0.7 * np.sin(W * tmid + th[d]) + 0.2 for d in range(n_det)])
    t_start = np.concatenate([np.arange(n_slots) * T for _ in range(n_det)])
    return dict(n=n, dt=dt, T=T, n_slots=n_slots, hs=hs, a=rows_a, b=rows_b, t_start=t_start,
                mc=mc, t_c=t_c, sigma=1.0)


def _sft_rows(net, series_per_det):
    xb = np.concatenate([synth.sfts_from_series(s, net["n"], net["n_slots"], net["dt"])
                         for s in series_per_det])
    psd = np.full(xb.shape, 2.0 * net["sigma"]**2 * net["dt"])
    return xb, psd


def test_fstat_norm_matrix_matches_time_domain_products(orc):
    """M of the oracle (reading R11 norms, cos-sin blocks zero) against the brute-force
    <h_nu, h_mu> = sum_j h_nu h_mu / sigma^2 of the four functions (Eq. td_product)."""
    net = _chirp_network(orc)
    xb, psd = _sft_rows(net, [np.zeros(net["n"] * net["n_slots"])] * 2)
    od = orc.SFTData(net["t_start"], net["n"], net["T"], 0, xb, psd, net["a"], net["b"])
    r = orc.scan(od, [net["mc"]], [net["t_c"]], K=16, kernel=orc.K_AUTO, fstat=True)
    Msft = _block_M(r["hhp"][0], r["hhx"][0], r["hhpx"][0])
    Mtd = sum(np.array([[np.sum(hi * hj) for hj in h] for hi in h]) for h in net["hs"]) / net["sigma"]**2
    scale = math.sqrt(Mtd[0, 0] * Mtd[1, 1])
    assert np.abs(Msft - Mtd).max() <= 2e-3 * scale
    # the time-domain cos-sin products are small (they oscillate with the phase)
    assert abs(Mtd[0, 2]) <= 2e-3 * scale and abs(Mtd[1, 3]) <= 2e-3 * scale


def test_fstat_recovers_injected_amplitudes(orc):
    """Noise-free data d = sum_nu c_nu h_nu with c_nu from A+, Ax, phi0, psi by the formula of
    Sec. II.B: the maximiser c* = M^{-1} x recovers c, and 2F equals <h, h> to the accuracy of
    the SFT approximation (2F ~ (1 - r)^2 <h, h>; the paper's bound r < 1e-2, Sec. IV); 2F is
    at least the log-likelihood ratio at the true amplitudes."""
    net = _chirp_network(orc)
    c = _c_paper(1.3, 0.9, 0.4, 0.3)
    series = [np.tensordot(c, h, axes=1) for h in net["hs"]]
    xb, psd = _sft_rows(net, series)
    od = orc.SFTData(net["t_start"], net["n"], net["T"], 0, xb, psd, net["a"], net["b"])
    r = orc.scan(od, [net["mc"]], [net["t_c"]], K=32, kernel=orc.K_AUTO, fstat=True)
    x = np.array([r["zp"][0].real, r["zx"][0].real, r["zp"][0].imag, r["zx"][0].imag])
    M = _block_M(r["hhp"][0], r["hhx"][0], r["hhpx"][0])
    cstar = np.linalg.solve(M, x)
    hh = sum(np.sum(s**2) for s in series) / net["sigma"]**2
    assert r["flags"][0] == 0
    assert np.linalg.norm(cstar - c) <= 5e-3 * np.linalg.norm(c)
    assert abs(r["twoF"][0] - hh) <= 2e-2 * hh
    assert r["twoF"][0] >= (2 * c @ x - c @ M @ c) * (1 - 1e-12)
    # a mis-assembled amplitude vector (sin and cos parts swapped) recovers something else
    xs = np.array([x[2], x[3], x[0], x[1]])
    assert np.linalg.norm(np.linalg.solve(M, xs) - c) > 0.1 * np.linalg.norm(c)


def test_fstat_noise_is_chi_squared_with_four_degrees(orc):
    """On Gaussian noise alone x is Gaussian with covariance M, so 2F follows chi^2 with four
    degrees of freedom (mean 4, variance 8).  A bin-centred monochromatic template has the
    single kernel weight 1, so the narrow-band norm is exact here."""
    g = np.random.default_rng(8)
    n, T, k0, n_rows = 128, 16.0, 20, 12
    nb = n // 2 + 1
    S = 0.5
    tm = np.arange(n_rows) * T + 0.5 * T
    a = np.cos(2 * np.pi * tm / 120.0)
    b = np.sin(2 * np.pi * tm / 120.0 + 0.4)
    phi = g.uniform(-20, 20, n_rows)
    vals = []
    for _ in range(1500):
        sd = math.sqrt(T * S / 4)
        xb = sd * (g.standard_normal((n_rows, nb)) + 1j * g.standard_normal((n_rows, nb)))
        od = orc.SFTData(np.arange(n_rows) * T, n, T, 0, xb, np.full((n_rows, nb), S), a, b)
        r = orc.ip_params(od, 1.0, phi, k0 / T, 0.0, K=4, kernel=orc.K_DIRICHLET, fstat=True, full=True)
        vals.append(r["twoF"])
    vals = np.array(vals)
    assert abs(vals.mean() - 4.0) <= 3 * math.sqrt(8.0 / vals.size)
    assert st.kstest(vals, st.chi2(4).cdf).pvalue > 1e-3
    # a norm twice too large (or amplitudes half as large) would halve the mean
    assert abs(vals.mean() / 2 - 4.0) > 5 * math.sqrt(8.0 / vals.size)


def test_fstat_degenerate_patterns_reduce_to_rho_squared(orc):
    """Reading R25: with b = 0.5 a in every row the four functions span two dimensions; the
    statistic is the phase-maximised one of Eq. det_short with the pattern a, i.e. rho^2 of
    the A+ = 1, Ax = 0 projector, and the template is flagged FSTAT_DEGENERATE."""
    w = synth.ground(seed=9, n_templates=5, n_slots=32, n_det=1, k_lo=40, k_hi=470, t_end_pad=300.0)
    a = np.cos(np.arange(w.n_sft) * 0.01)
    od = orc.SFTData(w.t_start, w.n_samples, w.t_sft, w.k_lo, w.x_bins, w.psd, a, 0.5 * a)
    r = orc.scan(od, w.bank["mc"], w.bank["t_c"], K=8, kernel=orc.K_AUTO, fstat=True)
    assert np.all(r["flags"] & orc.F_FSTAT_DEGENERATE)
    assert np.allclose(r["twoF"], r["rho"]**2, rtol=1e-12, atol=0)
    # a detector with b = 0: same statistic
    od0 = orc.SFTData(w.t_start, w.n_samples, w.t_sft, w.k_lo, w.x_bins, w.psd, a, np.zeros_like(a))
    r0 = orc.scan(od0, w.bank["mc"], w.bank["t_c"], K=8, kernel=orc.K_AUTO, fstat=True)
    assert np.allclose(r0["twoF"], r["rho"]**2, rtol=1e-12, atol=0)
