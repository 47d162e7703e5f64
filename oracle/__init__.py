"""FP64 CPU oracle for the SFT inner product (arXiv:2502.11823).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product (the HIP library and its
binding) never imports this package, and this package imports nothing from the
product.  The arithmetic lives in ``sft_oracle.c`` (plain C, FP64), compiled with
gcc into ``_liboracle.so`` next to this file; this module only marshals numpy
arrays.  See the C file for the equations each routine follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sft_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")

# kernel / reference / waveform / flag codes (mirror the enums in sft_oracle.c)
K_DIRICHLET, K_FRESNEL, K_AUTO, K_DISCRETE, K_QUAD = 0, 1, 2, 3, 4
REF_MID, REF_START = 0, 1
WF_NEWTON, WF_PN35, WF_SURROGATE = 0, 1, 2
F_OUT_OF_BAND, F_TAU_NONPOSITIVE, F_TAYLOR_INVALID, F_NONFINITE, F_EMPTY = 1, 2, 4, 8, 64
F_SURROGATE_FALLBACK = 32
F_FSTAT_DEGENERATE = 128

# GM_sun / c^3 in seconds (IAU 2015 nominal solar mass parameter)
T_SUN = 4.925490947641267e-6

_lib = None


def build(force: bool = True) -> str:
    """Compile sft_oracle.c with gcc (-O2, OpenMP, IEEE arithmetic)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    L = ctypes.c_long
    D = ctypes.c_double
    Int = ctypes.c_int
    lib.orc_kernel_eval.argtypes = [Int, Int, L, D, L, P, P, P]
    lib.orc_kernel_eval.restype = None
    lib.orc_fresnel_E_eval.argtypes = [L, P, P]
    lib.orc_fresnel_aux_eval.argtypes = [L, P, P]
    lib.orc_faddeeva_eval.argtypes = [L, P, P]
    lib.orc_rdft.argtypes = [P, L, P]
    lib.orc_make_sfts.argtypes = [P, L, L, L, D, P]
    lib.orc_median_bias.argtypes = [Int]
    lib.orc_median_bias.restype = D
    lib.orc_psd_running_median.argtypes = [P, L, D, Int, L, L, P]
    lib.orc_strain_sfts.argtypes = [P, L, L, D, Int, L, L, P, P, P]
    lib.orc_waveform.argtypes = [Int, D, D, D, D, D, D, P]
    lib.orc_waveform_array.argtypes = [Int, D, D, D, D, P, L, D, P]
    lib.orc_ip_params.argtypes = [L, L, D, L, L, P, P, P, P, P, P, P, P, P, P,
                                  Int, Int, Int, D, D, D, D, Int, Int, P, P, P]
    lib.orc_scan.argtypes = [L, L, D, L, L, P, P, P, P, P,
                             L, Int, P, P, P, P, P, P,
                             Int, Int, Int, D, D, D, D, D, Int, Int, P, P, P, P, P, P, P]
    lib.orc_doppler_waveform.argtypes = [Int, D, D, D, D, D, D, P, P, P]
    lib.orc_set_surrogate.argtypes = [Int, Int, P, P]
    lib.orc_mlp_param_count.argtypes = [Int, Int]
    lib.orc_mlp_param_count.restype = L
    lib.orc_mlp_forward_eval.argtypes = [P, Int, Int, L, P, P, P]
    lib.orc_mlp_forward_eval.restype = None
    lib.orc_surrogate_targets.argtypes = [L, P, P, P, D, Int, D, D, P]
    lib.orc_td_product.argtypes = [P, P, L, D]
    lib.orc_td_product.restype = D
    lib.orc_fd_product.argtypes = [P, P, L, D, P]
    lib.orc_fd_product.restype = D
    lib.orc_pn35_consistency.argtypes = [D, D, D, D]
    lib.orc_pn35_consistency.restype = D
    lib.orc_set_pn_order.argtypes = [Int]
    lib.orc_set_pn_order.restype = None
    lib.orc_set_threads.argtypes = [Int]
    lib.orc_set_threads.restype = None
    lib.orc_get_threads.argtypes = []
    lib.orc_get_threads.restype = Int
    lib.orc_tsft_max.argtypes = [D, D]
    lib.orc_tsft_max.restype = D
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _cplx(out):
    return out[0::2] + 1j * out[1::2]


# --------------------------------------------------------------------------- kernels
def kernel(x, beta, kernel=K_FRESNEL, t_ref=REF_MID, beta_switch=0.0, n=0):
    """Kernel F(x, beta) in bins (Sec. III.C); complex ndarray shaped like x."""
    x = np.asarray(x, dtype=np.float64)
    xb, bb = np.broadcast_arrays(x, np.asarray(beta, dtype=np.float64))
    xb = np.ascontiguousarray(xb.ravel())
    bb = np.ascontiguousarray(bb.ravel())
    out = np.empty(2 * xb.size)
    _load().orc_kernel_eval(kernel, t_ref, int(n), float(beta_switch), xb.size, _ptr(xb), _ptr(bb), _ptr(out))
    return _cplx(out).reshape(np.broadcast(x, beta).shape)


def fresnel_E(v):
    """E(v) = C(v) + i S(v) = int_0^v exp(i pi t^2/2) dt."""
    v = np.ascontiguousarray(np.ravel(v), dtype=np.float64)
    out = np.empty(2 * v.size)
    _load().orc_fresnel_E_eval(v.size, _ptr(v), _ptr(out))
    return _cplx(out)


def fresnel_aux(v):
    """G(v), v >= 0, with E(v) = (1+i)/2 - G(v) exp(i pi v^2/2)."""
    v = np.ascontiguousarray(np.ravel(v), dtype=np.float64)
    out = np.empty(2 * v.size)
    _load().orc_fresnel_aux_eval(v.size, _ptr(v), _ptr(out))
    return _cplx(out)


def faddeeva(z):
    """w(z) for Im z > 0 by continued fraction."""
    z = np.ravel(np.asarray(z, dtype=np.complex128))
    zz = np.ascontiguousarray(np.stack([z.real, z.imag], axis=1).ravel())
    out = np.empty(2 * z.size)
    _load().orc_faddeeva_eval(z.size, _ptr(zz), _ptr(out))
    return _cplx(out)


# --------------------------------------------------------------------------- transforms
def rdft(x):
    """sum_j x_j exp(-2 pi i jk/n), k = 0..n/2 (own FFT)."""
    x = _f64(x)
    out = np.empty(2 * (x.size // 2 + 1))
    _load().orc_rdft(_ptr(x), x.size, _ptr(out))
    return _cplx(out)


def make_sfts(x, n, n_sft, dt):
    """Eq. d_SFT for consecutive segments: complex [n_sft, n/2+1]."""
    x = _f64(x)
    nb = n // 2 + 1
    out = np.empty(2 * nb * n_sft)
    rc = _load().orc_make_sfts(_ptr(x), x.size, n, n_sft, float(dt), _ptr(out))
    if rc != 0:
        raise ValueError("series shorter than n_sft * n")
    return _cplx(out).reshape(n_sft, nb)


def median_bias(w):
    """Expected median of 2w+1 exponential variables of unit mean (reading R27)."""
    return _load().orc_median_bias(int(w))


def psd_running_median(power, n, T, w, k_lo, n_bins):
    """Per-SFT PSD from the periodogram power[0..n/2] by the bias-corrected running median."""
    p = _f64(power)
    out = np.empty(int(n_bins))
    if _load().orc_psd_running_median(_ptr(p), int(n), float(T), int(w), int(k_lo), int(n_bins), _ptr(out)) != 0:
        raise ValueError("band or block outside [0, n/2]")
    return out


def strain_sfts(x, n, dt, w, k_lo, n_bins):
    """SFTs (band bins, complex [n_seg, n_bins]), PSDs [n_seg, n_bins] and the keep flags of the
    consecutive segments of a strain series (Eq. d_SFT; reading R27)."""
    x = _f64(x)
    n_seg = x.size // int(n)
    bins = np.empty(2 * n_seg * int(n_bins))
    psd = np.empty(n_seg * int(n_bins))
    keep = np.empty(n_seg, np.int32)
    if _load().orc_strain_sfts(_ptr(x), x.size, int(n), float(dt), int(w), int(k_lo), int(n_bins), _ptr(bins),
                               _ptr(psd), _ptr(keep)) != 0:
        raise ValueError("band or block outside [0, n/2]")
    return _cplx(bins).reshape(n_seg, int(n_bins)), psd.reshape(n_seg, int(n_bins)), keep


# --------------------------------------------------------------------------- waveform
def waveform(mc, t_c, phi_c, t, q=1.0, wf=WF_NEWTON, tsun=T_SUN):
    """Waveform quantities (A, phi, f, fdot, fddot) at times t; NaN where tau <= 0."""
    t = np.ascontiguousarray(np.atleast_1d(np.asarray(t, dtype=np.float64)))
    res = np.empty((t.size, 5))
    rc = _load().orc_waveform_array(wf, float(mc), float(q), float(t_c), float(phi_c), _ptr(t), t.size,
                                    float(tsun), _ptr(res))
    if rc == -2:
        raise NotImplementedError("waveform model %d" % wf)
    return res


def doppler_waveform(mc, t_c, phi_c, t, eph, sky, q=1.0, wf=WF_NEWTON, tsun=T_SUN):
    """(A, phi, f, fdot, fddot) at detector time t of a source in direction sky seen by a
    detector with eph = (r/c, v/c, a/c) at t (Sec. III.B, reading R26)."""
    e = _f64(np.reshape(eph, 9))
    n = _f64(np.reshape(sky, 3))
    out = np.empty(5)
    rc = _load().orc_doppler_waveform(wf, float(mc), float(q), float(t_c), float(phi_c), float(t), float(tsun),
                                      _ptr(e), _ptr(n), _ptr(out))
    if rc != 0:
        out[:] = np.nan
    return out


def pn35_consistency(mc, q, tau, tsun=T_SUN):
    """(d phi/dt) / (2 pi f) - 1 of the 3.5PN waveform, analytic."""
    return _load().orc_pn35_consistency(float(mc), float(q), float(tau), float(tsun))


def set_pn_order(order: int):
    """Half PN orders kept by the 3.5PN waveform (7 = all; 0 = the Newtonian chirp)."""
    _load().orc_set_pn_order(int(order))


# --------------------------------------------------------------------------- inner products
class SFTData:
    """Raw SFT bins of a stored band plus per-SFT metadata (host, FP64)."""

    def __init__(self, t_start, n_samples, t_sft, k_lo, x_bins, psd, fplus=None, fcross=None):
        self.t_start = _f64(t_start)
        self.n_samples = int(n_samples)
        self.t_sft = float(t_sft)
        self.k_lo = int(k_lo)
        xb = np.asarray(x_bins)
        if np.iscomplexobj(xb):
            xb = np.stack([xb.real, xb.imag], axis=-1)
        self.x_bins = np.ascontiguousarray(xb, dtype=np.float64)
        self.n_sft, self.n_bins = self.x_bins.shape[0], self.x_bins.shape[1]
        self.psd = np.ascontiguousarray(np.broadcast_to(psd, (self.n_sft, self.n_bins)), dtype=np.float64)
        self.fplus = _f64(fplus)
        self.fcross = _f64(fcross)

    def _args(self):
        return (self.n_sft, self.n_samples, self.t_sft, self.k_lo, self.n_bins)


def ip_params(data: SFTData, A, phi, f, fdot, use=None, fddot=None, K=4, kernel=K_AUTO,
              t_ref=REF_MID, beta_switch=1e-7, a_plus=1.0, a_cross=0.0, delta_max=0.0,
              compensated=True, fstat=False, full=False):
    """Coherent sum for one template from per-SFT waveform quantities (Eq. efficient).

    Returns (z_plus, z_cross, hh_plus, hh_cross, rho, flags, tie); with full=True a dict
    that also holds the cross norm hhpx and 2F (when fstat)."""
    n = data.n_sft
    use = np.ones(n, np.uint8) if use is None else np.ascontiguousarray(use, dtype=np.uint8)
    A, phi, f, fdot = (_f64(np.broadcast_to(v, (n,))) for v in (A, phi, f, fdot))
    fddot = None if fddot is None else _f64(np.broadcast_to(fddot, (n,)))
    out = np.empty(9)
    fl = np.zeros(1, np.uint32)
    tie = np.zeros(1)
    _load().orc_ip_params(*data._args(), _ptr(data.x_bins), _ptr(data.psd), _ptr(data.fplus),
                          _ptr(data.fcross), _ptr(A), _ptr(phi), _ptr(f), _ptr(fdot), _ptr(fddot),
                          _ptr(use), int(K), int(kernel), int(t_ref), float(beta_switch),
                          float(a_plus), float(a_cross), float(delta_max), int(compensated),
                          int(bool(fstat)), _ptr(out), _ptr(fl), _ptr(tie))
    if full:
        return {"zp": out[0] + 1j * out[1], "zx": out[2] + 1j * out[3], "hhp": out[4], "hhx": out[5],
                "rho": out[6], "hhpx": out[7], "twoF": out[8], "flags": int(fl[0]), "tie": float(tie[0])}
    return (out[0] + 1j * out[1], out[2] + 1j * out[3], out[4], out[5], out[6], int(fl[0]), float(tie[0]))


def scan(data: SFTData, mc, t_c, phi_c=None, q=None, a_first=None, a_last=None, K=4,
         kernel=K_AUTO, t_ref=REF_MID, beta_switch=1e-7, a_plus=1.0, a_cross=0.0,
         tsun=T_SUN, delta_max=0.0, compensated=True, wf=WF_NEWTON, fstat=False, eph=None, sky=None):
    """Template-bank SFT inner products (Eq. efficient), one template per entry.

    Doppler (Sec. III.B, reading R26): eph [n_sft, 9] = (r/c, v/c, a/c) of each SFT row's
    detector at the SFT midpoint, sky [n, 3] unit vectors toward the sources.

    Returns a dict of numpy arrays: zp, zx (complex), hhp, hhx, rho, flags, tie, mismatch,
    n_used (SFT rows in the template's sum), and with fstat=True the cross norm hhpx and the F-statistic twoF (Sec. II.B)."""
    mc = _f64(np.atleast_1d(mc))
    m = mc.size
    t_c = _f64(np.broadcast_to(t_c, (m,)))
    phi_c = None if phi_c is None else _f64(np.broadcast_to(phi_c, (m,)))
    q = None if q is None else _f64(np.broadcast_to(q, (m,)))
    af = None if a_first is None else np.ascontiguousarray(np.broadcast_to(a_first, (m,)), dtype=np.int32)
    al = None if a_last is None else np.ascontiguousarray(np.broadcast_to(a_last, (m,)), dtype=np.int32)
    out = np.empty((m, 9))
    fl = np.zeros(m, np.uint32)
    tie = np.zeros(m)
    mm = np.zeros(m)
    nu = np.zeros(m, np.int32)
    eph = None if eph is None else np.ascontiguousarray(np.reshape(eph, (data.n_sft, 9)), dtype=np.float64)
    sky = None if sky is None else np.ascontiguousarray(np.broadcast_to(np.reshape(sky, (-1, 3)), (m, 3)),
                                                        dtype=np.float64)
    rc = _load().orc_scan(*data._args(), _ptr(data.t_start), _ptr(data.x_bins), _ptr(data.psd),
                          _ptr(data.fplus), _ptr(data.fcross), m, int(wf), _ptr(mc), _ptr(q),
                          _ptr(t_c), _ptr(phi_c), _ptr(af), _ptr(al), int(K), int(kernel),
                          int(t_ref), float(beta_switch), float(a_plus), float(a_cross),
                          float(tsun), float(delta_max), int(compensated), int(bool(fstat)),
                          _ptr(eph), _ptr(sky), _ptr(out), _ptr(fl), _ptr(tie), _ptr(mm), _ptr(nu))
    if rc == -2:
        raise ValueError("Doppler needs eph and sky, the midpoint reference and a closed-form waveform")
    if rc != 0:
        raise MemoryError("oracle scan failed")
    res = {"zp": out[:, 0] + 1j * out[:, 1], "zx": out[:, 2] + 1j * out[:, 3],
           "hhp": out[:, 4], "hhx": out[:, 5], "rho": out[:, 6], "flags": fl, "tie": tie,
           "mismatch": mm, "n_used": nu}
    if fstat:
        res["hhpx"] = out[:, 7]
        res["twoF"] = out[:, 8]
    return res


# --------------------------------------------------------------------------- surrogate
def mlp_param_count(hidden=128, layers=4):
    return int(_load().orc_mlp_param_count(int(hidden), int(layers)))


def set_surrogate(params, cfg, hidden=128, layers=4):
    """Install surrogate parameters (FP64 values) and its configuration dict with keys
    mc_lo, mc_hi, q_lo, q_hi, lt_lo, lt_hi, c_phi, c_amp, judge_tol, head."""
    params = _f64(params)
    assert params.size == mlp_param_count(hidden, layers)
    c = _f64([cfg["mc_lo"], cfg["mc_hi"], cfg["q_lo"], cfg["q_hi"], cfg["lt_lo"], cfg["lt_hi"],
              cfg["c_phi"], cfg["c_amp"], cfg.get("judge_tol", 1e-4), 1.0 if cfg.get("head") else 0.0])
    if _load().orc_set_surrogate(int(hidden), int(layers), _ptr(params), _ptr(c)) != 0:
        raise MemoryError("surrogate")


def mlp_forward(params, u, hidden=128, layers=4):
    """Outputs y [n, 2] and their derivatives along the third input dy [n, 2] (FP64)."""
    params = _f64(params)
    u = _f64(np.atleast_2d(u))
    y = np.empty((u.shape[0], 2))
    dy = np.empty((u.shape[0], 2))
    _load().orc_mlp_forward_eval(_ptr(params), int(hidden), int(layers), u.shape[0], _ptr(u), _ptr(y), _ptr(dy))
    return y, dy


def surrogate_targets(mc, q, tau, head, c_phi, c_amp, tsun=T_SUN):
    """Training targets from the 3.5PN and Newtonian waveforms (FP64)."""
    mc, q, tau = _f64(mc), _f64(q), _f64(tau)
    y = np.empty((mc.size, 2))
    if _load().orc_surrogate_targets(mc.size, _ptr(mc), _ptr(q), _ptr(tau), float(tsun), int(bool(head)),
                                     float(c_phi), float(c_amp), _ptr(y)) != 0:
        raise ValueError("tau must be positive")
    return y


# --------------------------------------------------------------------------- brute force
def td_product(d, h, dt):
    """dt * sum_j d_j h_j (Eq. td_product, discrete)."""
    d, h = _f64(d), _f64(h)
    return _load().orc_td_product(_ptr(d), _ptr(h), d.size, float(dt))


def fd_product(x, h, dt, S):
    """4 Re int x~* h~ / S df on the full series with the oracle's FFT (Eq. fd_product)."""
    x, h = _f64(x), _f64(h)
    S = _f64(np.broadcast_to(S, (x.size // 2 + 1,)))
    return _load().orc_fd_product(_ptr(x), _ptr(h), x.size, float(dt), _ptr(S))


def set_threads(n):
    """Threads of the oracle's OpenMP loops."""
    _load().orc_set_threads(int(n))


def get_threads():
    return int(_load().orc_get_threads())


def tsft_max(delta, fddot_max):
    """Eq. max_tsft."""
    return _load().orc_tsft_max(float(delta), float(fddot_max))
