"""Pins of the oracle's Doppler form (Sec. III.B: the phase as a function of the emission
time t_s(t; n), and the frequency (1/2 pi)(dphi/dt_s)(dt_s/dt); reading R26), CPU only."""
import math

import numpy as np

from paper_2502_11823_amd import synth


def _phase_at(orc, mc, t_c, t, orbit, n):
    """Detector-frame phase phi(t + r(t).n/c) from the source-frame waveform (pinned by P10)."""
    e = orbit(np.atleast_1d(t))
    ts = np.atleast_1d(t) + e[:, :3] @ n
    return orc.waveform(mc, t_c, 0.0, ts)[:, 1]


def test_doppler_frequency_and_drift_are_derivatives_of_the_delayed_phase(orc):
    """f and fdot of the oracle equal (1/2 pi) dPhi/dt and (1/2 pi) d^2Phi/dt^2 of the delayed
    phase Phi(t) = phi(t + r(t).n/c), by central differences; a fast synthetic orbit makes the
    velocity and acceleration terms large (about 1% of fdot, fifty times the tolerance)."""
    mc, t_c = 1.2, 6000.0
    orbit = lambda t: synth.circular_orbit(t, 0.5, 2000.0, 0.7, 0.4)
    n = synth.sky_vector(1.1, -0.3)
    for t in (1000.0, 2500.0, 4200.0):
        got = orc.doppler_waveform(mc, t_c, 0.0, t, orbit(np.array([t]))[0], n)
        h = 0.5
        ph = _phase_at(orc, mc, t_c, np.array([t - h, t, t + h]), orbit, n)
        f_fd = (ph[2] - ph[0]) / (2 * h) / (2 * math.pi)
        fd_fd = (ph[2] - 2 * ph[1] + ph[0]) / h**2 / (2 * math.pi)
        assert abs(got[2] - f_fd) <= 1e-7 * abs(f_fd)
        assert abs(got[3] - fd_fd) <= 2e-4 * abs(fd_fd)
        # the phase and amplitude are those of the source at the emission time
        e = orbit(np.array([t]))[0]
        src = orc.waveform(mc, t_c, 0.0, t + e[:3] @ n)[0]
        assert got[1] == src[1] and got[0] == src[0]
        # and the Doppler terms matter at this size
        assert abs(got[3] - src[3]) > 5e-3 * abs(src[3])


def _tiny_data(orc, x, n=2048, n_sft=32, fs=32.0):
    dt = 1.0 / fs
    T = n * dt
    xb = synth.sfts_from_series(x, n, n_sft, dt)
    psd = np.full(xb.shape, 2.0 * dt)
    return orc.SFTData(np.arange(n_sft) * T, n, T, 0, xb, psd), T, dt


def test_doppler_limits_zero_and_constant_offset(orc):
    """eph = 0 gives the plain scan bit for bit; a constant offset r (v = a = 0) is a shift of
    the arrival times, i.e. the plain scan with t_c - r.n."""
    g = np.random.default_rng(2)
    od, T, dt = _tiny_data(orc, g.normal(size=2048 * 32))
    mc = np.linspace(1.19, 1.21, 7)
    t_c = np.full(7, 2600.0)
    sky = synth.sky_vector(g.uniform(0, 2 * np.pi, 7), g.uniform(-1, 1, 7))
    base = orc.scan(od, mc, t_c, K=8, kernel=orc.K_AUTO)
    zero = orc.scan(od, mc, t_c, K=8, kernel=orc.K_AUTO, eph=np.zeros((32, 9)), sky=sky)
    for k in ("zp", "hhp", "rho", "flags"):
        assert np.array_equal(base[k], zero[k]), k
    eph = np.zeros((32, 9))
    eph[:, :3] = [3.0, -1.0, 2.0]
    off = orc.scan(od, mc, t_c, K=8, kernel=orc.K_AUTO, eph=eph, sky=sky)
    shifted = orc.scan(od, mc, t_c - sky @ np.array([3.0, -1.0, 2.0]), K=8, kernel=orc.K_AUTO)
    # equal up to the rounding of t_c - t - D against (t_c - D) - t (1e-12 s, 1e-10 rad of phase)
    assert np.allclose(off["zp"], shifted["zp"], rtol=0, atol=1e-9 * np.sqrt(base["hhp"]).max())
    assert np.allclose(off["rho"], shifted["rho"], rtol=1e-9)


def test_doppler_template_recovers_a_doppler_modulated_signal(orc):
    """Noise-free data x(t) = A(t_s) cos phi(t_s(t)) of a source seen through a moving detector
    (synthetic orbit of 0.05 light-seconds, 3000 s period: a phase modulation of ~2.5 rad at
    8 Hz): the Doppler template recovers <h, h> within the SFT approximation (r < 1e-2), the
    template without Doppler, or with the source in the opposite direction, does not."""
    n, n_sft, fs = 2048, 32, 32.0
    dt = 1.0 / fs
    t = np.arange(n * n_sft) * dt
    mc, t_c = 1.2, n_sft * n * dt + 1500.0
    n_src = synth.sky_vector(0.4, 0.2)
    orbit = lambda tt: synth.circular_orbit(tt, 0.05, 3000.0, 0.3, 0.2)
    e = orbit(t)
    w = orc.waveform(mc, t_c, 0.0, t + e[:, :3] @ n_src)
    x = w[:, 0] * np.cos(w[:, 1])
    od, T, _ = _tiny_data(orc, x, n, n_sft, fs)
    eph = orbit(np.arange(n_sft) * T + 0.5 * T)
    hh = np.sum(x**2)                       # sigma = 1
    dop = orc.scan(od, [mc], [t_c], K=16, kernel=orc.K_AUTO, eph=eph, sky=n_src)
    plain = orc.scan(od, [mc], [t_c], K=16, kernel=orc.K_AUTO)
    wrong = orc.scan(od, [mc], [t_c], K=16, kernel=orc.K_AUTO, eph=eph, sky=-n_src)
    rho_opt = math.sqrt(hh)
    assert abs(dop["zp"][0].real / hh - 1.0) <= 2e-2
    assert abs(dop["rho"][0] / rho_opt - 1.0) <= 2e-2
    assert plain["rho"][0] < 0.6 * rho_opt and wrong["rho"][0] < 0.6 * rho_opt
