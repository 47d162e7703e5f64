"""Accuracy study of the SFT inner product (Sec. IV): the relative error
r = 1 - sqrt(([d,h]) / <d,h>) of Sec. IV.A for a noise-free signal, as a function of the
Taylor-validity fraction delta (which sets T_SFT by Eq. max_tsft) and the window width
Delta k = 2K, for the two pilot sources of Sec. IV.B (BNS in a third-generation ground-based
detector) and Sec. IV.C (massive BBH in a space-based detector).  Also T_SFT selection per
parameter-space region (the closing remark of Sec. III.F).

Every numerical step runs in libsft.so on the device: the strain of the signal at every sample
(sft_waveform_series), the direct integral <d,h> (sft_td_product), the SFTs of the series
(sft_load_strain, with the known white PSD) and the SFT inner product (sft_template_bank_scan).
This module only chooses the configurations and marshals arguments.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import sft

DAY = 86400.0
YEAR = 3.15576e7

# The pilot sources: component masses, band, sampling rate, the period of the antenna
# modulation a(t) = cos(2 pi t / P), b(t) = sin(2 pi t / P), and the SFT lengths of the paper's
# tables (context only; the study derives its own from its waveform).
# The waveform: the 3.5PN inspiral for the BNS; the leading-order chirp for the massive BBH,
# whose 3.5PN (TaylorT3) frequency peaks at ~1.2e-3 Hz about 1500 s before coalescence and never
# reaches the band edge of 1.9e-3 Hz (the paper's IMRPhenomT does).
CASES = {
    "bns": dict(m1=1.4, m2=1.4, f_lo=1.0, f_hi=10.0, fs=40.0, period=DAY, waveform="pn35",
                paper_tsft={3.0: 106, 2.0: 92, 1.0: 73}),
    "mbbh": dict(m1=1e6, m2=1e6, f_lo=1e-4, f_hi=1.9e-3, fs=2.0, period=YEAR, waveform="newton",
                 paper_tsft={3.0: 2502, 2.0: 2185, 1.0: 1735}),
}


def chirp_mass(m1, m2):
    return (m1 * m2) ** 0.6 / (m1 + m2) ** 0.2


def _quantities(mc, q, t_c, t, waveform):
    """(A, phi, f, fdot, fddot) of the library's waveform at the host times t (device evaluation)."""
    t = np.atleast_1d(np.asarray(t, np.float64))
    out = []
    for tt in t:
        _, qv = sft.waveform_series(mc, t_c, float(tt), 1.0, 1, waveform=waveform, q=q, quantities=True)
        out.append(qv.cpu().numpy()[0])
    return np.array(out)


def time_of_frequency(mc, q, f, waveform="pn35", t_c=0.0):
    """The time before t_c at which the waveform's frequency is f: tau halved from 1e12 s until
    the frequency passes f (the post-Newtonian series are not evaluated closer to coalescence
    than needed), then bisection on tau."""
    def freq(tau):
        return _quantities(mc, q, t_c, [t_c - tau], waveform)[0, 2]
    hi = 1e12
    lo = hi / 2
    f_prev = 0.0
    while True:
        fl = freq(lo)
        if not np.isfinite(fl) or fl <= f_prev or lo < 1e-3:
            raise ValueError("the waveform's frequency does not reach %g Hz (it peaks near %g Hz)" % (f, f_prev))
        if fl >= f:
            break
        f_prev = fl
        hi, lo = lo, lo / 2
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if freq(mid) > f:
            lo = mid
        else:
            hi = mid
        if hi / lo < 1 + 1e-13:
            break
    return t_c - math.sqrt(lo * hi)


def tsft(delta, fddot_max, floor_seconds=True):
    """Eq. max_tsft: T_SFT(delta) = (2 delta / max fddot)^(1/3), floored to whole seconds as in the
    paper's tables."""
    T = (2.0 * delta / fddot_max) ** (1.0 / 3.0)
    return float(math.floor(T)) if floor_seconds else T


def tsft_regions(mc_edges, f_hi, delta, q=1.0, waveform="pn35"):
    """T_SFT per chirp-mass region (Sec. III.F: different parameter-space regions may use
    different SFT lengths): in each region [mc_i, mc_i+1] the largest fddot at the band's upper
    frequency f_hi is the one of the heaviest chirp mass (fddot grows with the mass at fixed f),
    and sets T_SFT by Eq. max_tsft.  Returns a list of (mc_lo, mc_hi, fddot_max, T_SFT)."""
    res = []
    for a, b in zip(mc_edges[:-1], mc_edges[1:]):
        t_hi = time_of_frequency(b, q, f_hi, waveform)
        fdd = _quantities(b, q, 0.0, [t_hi], waveform)[0, 4]
        res.append((float(a), float(b), float(fdd), tsft(delta, fdd)))
    return res


def r_study(case="bns", deltas=(3.0, 2.0, 1.0), dks=(4, 8, 12, 16, 20, 24, 32, 40, 48, 64), waveform=None,
            span_scale=1.0, storage="f32", precision="fp32_kahan", log=None):
    """r(delta, Delta k) for the pilot source `case` (noise-free signal, white PSD, the
    projector Lambda = [a(t) + b(t)](Re + Im) of Sec. IV.B, i.e. c_nu = 1).  The data span the
    band [f_lo, f_hi] of the source; span_scale < 1 keeps only the last fraction of it (smaller
    test configurations).  Returns a dict with the table r[delta][dk] and the configuration."""
    import torch
    c = CASES[case]
    waveform = waveform or c["waveform"]
    say = log or (lambda msg: None)
    mc = chirp_mass(c["m1"], c["m2"])
    q = max(c["m1"], c["m2"]) / min(c["m1"], c["m2"])
    t0 = time.perf_counter()
    # time axis: t_c at 0; the data run from f_lo to f_hi
    t_lo = time_of_frequency(mc, q, c["f_lo"], waveform)
    t_hi = time_of_frequency(mc, q, c["f_hi"], waveform)
    t_start = t_hi - span_scale * (t_hi - t_lo)
    say("%s: band %g-%g Hz spans %.1f h (%.1f s of setup)" % (case, c["f_lo"], c["f_hi"], (t_hi - t_lo) / 3600.0,
                                                           time.perf_counter() - t0))
    fs = c["fs"]
    dt = 1.0 / fs
    n0 = int(math.floor((t_hi - t_start) * fs))
    t_c = -t_start          # shift: sample 0 at t = 0
    tt = torch.arange(n0, dtype=torch.float64, device="cuda") * dt
    ph = 2.0 * math.pi * tt / c["period"]
    ab = torch.cos(ph) + torch.sin(ph)
    h = sft.waveform_series(mc, t_c, 0.0, dt, n0, waveform=waveform, q=q, fplus=ab, fcross=ab,
                            a_plus=1.0, a_cross=1.0)
    S = 2.0 * dt           # white PSD of unit-variance samples
    hh = sft.td_product(h, h, dt, S)
    fdd_max = float(_quantities(mc, q, t_c, [(n0 - 1) * dt], waveform)[0, 4])
    say("%s: %d samples, <h,h> = %.6g, max fddot %.4g Hz/s^2 (%.1f s)" % (case, n0, hh, fdd_max,
                                                                          time.perf_counter() - t0))
    rows = {}
    cfg = {}
    for delta in deltas:
        T = tsft(delta, fdd_max)
        n = int(round(T * fs))
        n -= n % 2
        n_sft = n0 // n
        # the antenna patterns at the SFT midpoints
        tm = (np.arange(n_sft) + 0.5) * n * dt
        abm = np.cos(2 * math.pi * tm / c["period"]) + np.sin(2 * math.pi * tm / c["period"])
        data = sft.SFTData.from_strain(h.reshape(1, -1), n, dt, 0, n // 2 + 1, 0, s_white=S,
                                       fplus=abm[None, :], fcross=abm[None, :], storage=storage)
        bank = sft.bank_to_device({"mc": np.array([mc]), "q": np.array([q]), "t_c": np.array([t_c]),
                                   "phi_c": np.zeros(1)})
        rr = {}
        for dk in dks:
            opts = sft.make_opts(K=dk // 2, kernel="auto", precision=precision, waveform=waveform, a_plus=1.0,
                                 a_cross=1.0)
            out = sft.template_bank_scan(data, bank, opts)
            torch.cuda.synchronize()
            zp = out["zp"].cpu().numpy()[0]
            zx = out["zx"].cpu().numpy()[0]
            dh = zp[0] + zx[1]                 # A+ Re z+ + Ax Im zx
            rr[int(dk)] = float(1.0 - math.sqrt(dh / hh)) if dh > 0 else float("nan")
        rows[float(delta)] = rr
        say("%s: delta %g, T_SFT %g s, %d SFTs: r %s (%.1f s)" % (case, delta, T, n_sft,
            {k: round(v, 5) for k, v in rr.items()}, time.perf_counter() - t0))
        cfg[float(delta)] = {"T_sft": T, "n_samples": n, "n_sft": n_sft,
                             "paper_T_sft": c["paper_tsft"].get(delta)}
        data.close()
    return {"case": case, "waveform": waveform, "mc": mc, "q": q, "fs": fs, "n0": n0, "hh": hh, "t_c": t_c,
            "duration_h": (t_hi - t_start) / 3600.0, "fddot_max": fdd_max, "config": cfg, "r": rows,
            "seconds": time.perf_counter() - t0}
