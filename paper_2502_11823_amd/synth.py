"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the GPU path's tests/benchmark and by the oracle's
tests.  It draws random numbers and lays out arrays; it contains none of the
method's arithmetic (no waveform, kernel, whitening or inner product).  The one
transform it applies, the per-segment DFT that turns a time series into raw SFT
bins with the normalisation of Eq. d_SFT (dt times numpy's forward FFT), is the
input convention of the method, not a step of it.

Workloads (all synthetic; the paper's data are simulated signals too):
  * ``tiny``   : one detector, white noise sigma = 1 at 32 Hz, 16384 s, 256 SFTs of
                 64 s (1025 bins), 1024 templates with Mc ~ U[1.19, 1.21], t_c =
                 16984 s, K = 4, Dirichlet, FP64.
  * ``ground`` : three detectors, 4096 SFT slots of 32 s at 128 Hz each, 5% of
                 slots dropped per detector, coloured PSD (f/5)^-4 + 1 + (f/50)^2
                 with a U[0.8, 1.2] scale per SFT, antenna patterns with a one-day
                 period, stored band bins [32, 512), 1e5 templates with
                 Mc ~ U[1.0, 1.5], t_c = 131672 s, K = 8, automatic kernel.
  * ``space``  : one detector, 60 SFTs of 2 days at 0.2 Hz (34560 samples, band
                 bins [0, 1792) = 0 .. 1.04e-2 Hz), white noise, antenna patterns with
                 a one-year period; 2e5 templates with Mc log-uniform in [1e5, 1e6]
                 Msun, each using its last n_use ~ U{8..60} SFTs (ragged), K = 32.
                 t_c puts the last SFT midpoint tau_end = 3.5e5 s (Mc/1e5)^(-5/19)
                 before coalescence (the recipe constant is derived in the design
                 notes so that the last SFT keeps the Taylor residual below 3 bins
                 and the drift below 48 bins).
Noise in the ``ground`` workload is drawn directly in the SFT domain (independent
Gaussian bins of variance T S / 4 per quadrature), which is the exact law of the
SFT of stationary Gaussian noise under a rectangular window when leakage is
ignored.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Optional

import numpy as np

DAY = 86400.0


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.PCG64(seed))


@dataclass
class Workload:
    """Raw SFT data (host, FP64) plus a template bank and evaluation options."""
    name: str
    t_start: np.ndarray          # [n_sft] segment start times [s]
    det: np.ndarray              # [n_sft] detector index
    n_samples: int               # samples per SFT
    t_sft: float                 # T_SFT [s]
    k_lo: int                    # first stored bin
    x_bins: np.ndarray           # [n_sft, n_bins] complex128 raw SFT bins (Eq. d_SFT)
    psd: np.ndarray              # [n_sft, n_bins] one-sided PSD
    fplus: Optional[np.ndarray]  # [n_sft] or None
    fcross: Optional[np.ndarray]  # [n_sft] or None
    bank: Dict[str, np.ndarray]  # mc, q, t_c, phi_c (f64), a_first, a_last (i32)
    opts: Dict[str, float] = field(default_factory=dict)

    @property
    def n_sft(self) -> int:
        return int(self.x_bins.shape[0])

    @property
    def n_bins(self) -> int:
        return int(self.x_bins.shape[1])

    @property
    def n_templates(self) -> int:
        return int(self.bank["mc"].size)

    def subset(self, idx) -> Dict[str, np.ndarray]:
        return {k: np.ascontiguousarray(v[idx]) for k, v in self.bank.items()}


# ----------------------------------------------------------------------------- primitives
def white_series(n_total: int, sigma: float, seed: int) -> np.ndarray:
    return rng(seed).normal(0.0, sigma, n_total)


def sfts_from_series(x: np.ndarray, n: int, n_sft: int, dt: float) -> np.ndarray:
    """Raw SFT bins of consecutive segments: dt * rfft (Eq. d_SFT convention)."""
    seg = np.asarray(x[: n * n_sft], dtype=np.float64).reshape(n_sft, n)
    return dt * np.fft.rfft(seg, axis=1)


def sft_domain_noise(psd: np.ndarray, t_sft: float, seed: int) -> np.ndarray:
    """Complex bins with independent Re, Im ~ N(0, T S / 4)."""
    sd = np.sqrt(t_sft * psd / 4.0)
    g = rng(seed)
    return sd * (g.standard_normal(psd.shape) + 1j * g.standard_normal(psd.shape))


def uniform_bank(n: int, mc_lo: float, mc_hi: float, t_c, seed: int, sort: bool = True,
                 q_lo: float = 1.0, q_hi: float = 1.0, random_phase: bool = False,
                 a_first=None, a_last=None, n_sft: int = 0) -> Dict[str, np.ndarray]:
    g = rng(seed)
    mc = g.uniform(mc_lo, mc_hi, n)
    q = g.uniform(q_lo, q_hi, n) if q_hi > q_lo else np.full(n, q_lo)
    phi = g.uniform(0.0, 2 * np.pi, n) if random_phase else np.zeros(n)
    if sort:
        o = np.argsort(mc, kind="stable")
        mc, q, phi = mc[o], q[o], phi[o]
    tc = np.broadcast_to(np.asarray(t_c, dtype=np.float64), (n,)).copy()
    af = np.zeros(n, np.int32) if a_first is None else np.broadcast_to(a_first, (n,)).astype(np.int32)
    al = (np.full(n, n_sft - 1, np.int32) if a_last is None
          else np.broadcast_to(a_last, (n,)).astype(np.int32))
    return {"mc": mc, "q": q, "t_c": tc, "phi_c": phi, "a_first": af.copy(), "a_last": al.copy()}


def coloured_psd_shape(f: np.ndarray) -> np.ndarray:
    """Ground-detector PSD shape of the ``ground`` workload: (f/5)^-4 + 1 + (f/50)^2."""
    return (f / 5.0) ** -4 + 1.0 + (f / 50.0) ** 2


# ----------------------------------------------------------------------------- workloads
def tiny(seed: int = 1, n_templates: int = 1024, n_sft: int = 256, noise_series: bool = True) -> Workload:
    """One detector, white noise (sigma = 1 per sample) at 32 Hz, 64 s SFTs."""
    fs, t_sft = 32.0, 64.0
    n = int(fs * t_sft)
    dt = 1.0 / fs
    sigma = 1.0
    x = white_series(n * n_sft, sigma, seed)
    xb = sfts_from_series(x, n, n_sft, dt)
    psd = np.full(xb.shape, 2.0 * sigma * sigma * dt)      # S_n = 2 sigma^2 dt
    bank = uniform_bank(n_templates, 1.19, 1.21, 16384.0 + 600.0, seed + 1000, n_sft=n_sft)
    w = Workload("tiny", np.arange(n_sft) * t_sft, np.zeros(n_sft, np.int32), n, t_sft, 0, xb, psd,
                 None, None, bank, dict(K=4, kernel="dirichlet", precision="fp64"))
    w.series = x if noise_series else None  # type: ignore[attr-defined]
    w.sigma = sigma  # type: ignore[attr-defined]
    return w


def ground(seed: int = 2, n_templates: int = 100_000, n_slots: int = 4096, n_det: int = 3,
           gap_frac: float = 0.05, k_lo: int = 32, k_hi: int = 512, t_end_pad: float = 600.0,
           mc_lo: float = 1.0, mc_hi: float = 1.5) -> Workload:
    """Three-detector ground-based bank with coloured, non-stationary noise and gaps."""
    fs, t_sft = 128.0, 32.0
    n = int(fs * t_sft)
    g = rng(seed)
    n_drop = int(round(gap_frac * n_slots))
    rows_t, rows_d = [], []
    for d in range(n_det):
        keep = np.sort(g.permutation(n_slots)[: n_slots - n_drop])
        rows_t.append(keep * t_sft)
        rows_d.append(np.full(keep.size, d, np.int32))
    t_start = np.concatenate(rows_t)
    det = np.concatenate(rows_d)
    n_sft = t_start.size
    f = np.arange(k_lo, k_hi) / t_sft
    scale = g.uniform(0.8, 1.2, n_sft)
    psd = scale[:, None] * coloured_psd_shape(f)[None, :]
    xb = sft_domain_noise(psd, t_sft, seed + 17)
    ph = 2.0 * np.pi * (t_start + 0.5 * t_sft) / DAY + 2.0 * np.pi * det / 3.0
    fplus, fcross = np.cos(ph), np.sin(ph)
    t_c = n_slots * t_sft + t_end_pad
    bank = uniform_bank(n_templates, mc_lo, mc_hi, t_c, seed + 1000, n_sft=n_sft)
    return Workload("ground", t_start, det, n, t_sft, k_lo, xb, psd, fplus, fcross, bank,
                    dict(K=8, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0))


YEAR = 3.15576e7


def space(seed: int = 3, n_templates: int = 200_000, n_sft: int = 60, n_use_lo: int = 8,
          n_use_hi: int = 60) -> Workload:
    """Space-based-like massive-BBH bank with ragged SFT ranges (one detector)."""
    fs, t_sft = 0.2, 2 * DAY
    n = int(round(fs * t_sft))
    k_lo, k_hi = 0, 1792
    g = rng(seed)
    t_start = np.arange(n_sft) * t_sft
    psd = np.ones((n_sft, k_hi - k_lo))
    xb = sft_domain_noise(psd, t_sft, seed + 17)
    ph = 2.0 * np.pi * (t_start + 0.5 * t_sft) / YEAR
    fplus, fcross = np.cos(ph), np.sin(ph)
    mc = np.exp(g.uniform(np.log(1e5), np.log(1e6), n_templates))
    n_use = g.integers(n_use_lo, n_use_hi + 1, n_templates)
    a_first = (n_sft - n_use).astype(np.int32)
    o = np.lexsort((mc, a_first))             # group templates of equal range, then by mass
    mc, a_first = mc[o], a_first[o]
    t_mid_last = t_start[-1] + 0.5 * t_sft
    t_c = t_mid_last + 3.5e5 * (mc / 1e5) ** (-5.0 / 19.0)
    bank = {"mc": mc, "q": np.ones(n_templates), "t_c": t_c, "phi_c": np.zeros(n_templates),
            "a_first": a_first, "a_last": np.full(n_templates, n_sft - 1, np.int32)}
    return Workload("space", t_start, np.zeros(n_sft, np.int32), n, t_sft, k_lo, xb, psd, fplus, fcross,
                    bank, dict(K=32, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0))


# ----------------------------------------------------------------------------- ephemerides
AU_S = 499.00478383615643     # astronomical unit / c [s]
R_EARTH_S = 6.371e6 / 299792458.0
SIDEREAL_DAY = 86164.0905
OBLIQUITY = np.deg2rad(23.4393)


def circular_orbit(t, radius: float, period: float, phase: float = 0.0, tilt: float = 0.0):
    """Position, velocity and acceleration over c ([n, 9]: r/c [s], v/c, a/c [1/s]) of a
    point on a circle of radius `radius` (light-seconds) in a plane tilted by `tilt` about the
    x axis, angular position W t + phase."""
    t = np.asarray(t, np.float64)
    W = 2.0 * np.pi / period
    th = W * t + phase
    c, s = np.cos(th), np.sin(th)
    ct, st_ = np.cos(tilt), np.sin(tilt)
    r = radius * np.stack([c, s * ct, s * st_], -1)
    v = radius * W * np.stack([-s, c * ct, c * st_], -1)
    a = -(W * W) * r
    return np.concatenate([r, v, a], -1)


def ground_ephemeris(t, latitude: float, longitude: float):
    """A ground detector: the Earth on a circular orbit of 1 AU in the ecliptic (tilted by the
    obliquity against the equatorial frame) plus the Earth's rotation at the detector's
    latitude and longitude (sidereal day).  [n, 9] as circular_orbit."""
    orb = circular_orbit(t, AU_S, 3.15576e7, 0.0, OBLIQUITY)
    rot = circular_orbit(t, R_EARTH_S * np.cos(latitude), SIDEREAL_DAY, longitude, 0.0)
    rot[..., 2] += R_EARTH_S * np.sin(latitude)
    return orb + rot


def sky_vector(ra, dec):
    """Unit vectors toward (right ascension, declination), [n, 3]."""
    ra, dec = np.broadcast_arrays(np.asarray(ra, np.float64), np.asarray(dec, np.float64))
    return np.stack([np.cos(dec) * np.cos(ra), np.cos(dec) * np.sin(ra), np.sin(dec)], -1)


def mlp_init(seed: int, hidden: int = 128, layers: int = 4) -> np.ndarray:
    """Seeded initial parameters of the surrogate network, packed layer by layer
    (W [n_in][n_out] input-major, then b [n_out]): W ~ N(0, 1/n_in), b = 0, the output
    layer scaled by 0.1.  FP32 values returned as float64."""
    g = rng(seed)
    dims = [3] + [hidden] * layers + [2]
    parts = []
    for i in range(len(dims) - 1):
        W = g.standard_normal((dims[i], dims[i + 1])) / np.sqrt(dims[i])
        if i == len(dims) - 2:
            W *= 0.1
        parts += [W.ravel(), np.zeros(dims[i + 1])]
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def surrogate_samples(n: int, seed: int, mc_lo: float, mc_hi: float, q_lo: float, q_hi: float,
                      tau_lo: float, tau_hi: float):
    """Training inputs: Mc, q uniform, ln(tau) uniform."""
    g = rng(seed)
    mc = g.uniform(mc_lo, mc_hi, n)
    q = g.uniform(q_lo, q_hi, n)
    tau = np.exp(g.uniform(np.log(tau_lo), np.log(tau_hi), n))
    return mc, q, tau


def paper_shape(name: str, seed: int = 5, n_templates: int = 1000) -> Workload:
    """Context workloads shaped like the paper's timing runs (Sec. V.C): one detector, white
    noise drawn in the SFT domain (unit PSD), every bin of each SFT stored, and a bank of
    templates whose chirp mass lies within 0.5% of the nominal system; t_c puts the end of
    the data where the nominal chirp reaches its upper frequency.
      * ``bns``  : 1.4 + 1.4 Msun, 1 -> 10 Hz, fs = 40 Hz, 6384 SFTs of 73 s, K = 50.
      * ``mbbh`` : 1e6 + 1e6 Msun, 1e-4 -> 1.9e-3 Hz, fs = 2 Hz, 1540 SFTs of 2502 s, K = 15."""
    if name == "bns":
        fs, t_sft, n_sft, m1, f_hi, K = 40.0, 73.0, 6384, 1.4, 10.0, 50
    elif name == "mbbh":
        fs, t_sft, n_sft, m1, f_hi, K = 2.0, 2502.0, 1540, 1.0e6, 1.9e-3, 15
    else:
        raise ValueError(name)
    n = int(round(fs * t_sft))
    mc0 = (m1 * m1) ** 0.6 / (2.0 * m1) ** 0.2
    M = mc0 * 4.925490947641267e-6
    tau_end = 5.0 * M * (8.0 * np.pi * M * f_hi) ** (-8.0 / 3.0)   # leading-order time to coalescence
    t_start = np.arange(n_sft) * t_sft
    psd = np.ones((n_sft, n // 2 + 1))
    xb = sft_domain_noise(psd, t_sft, seed + 17)
    bank = uniform_bank(n_templates, 0.995 * mc0, 1.005 * mc0, n_sft * t_sft + tau_end, seed + 1000, n_sft=n_sft)
    return Workload("paper-" + name, t_start, np.zeros(n_sft, np.int32), n, t_sft, 0, xb, psd, None, None,
                    bank, dict(K=K, kernel="auto", precision="fp32_kahan"))

