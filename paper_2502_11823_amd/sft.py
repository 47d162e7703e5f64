"""Thin ctypes binding of libsft.so (C ABI in include/sft.h).

Argument marshalling only: every step of the SFT inner product runs in the HIP
kernels of libsft.so.  PyTorch provides device memory and streams.  If the
library has not been built, ``lib()`` raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsft.so")

SFT_OK = 0
STORAGE = {"f64": 0, "f32": 1, "bf16": 2}
KERNEL = {"dirichlet": 0, "fresnel": 1, "auto": 2}
PRECISION = {"fp64": 0, "fp32_kahan": 1, "fp32_naive": 2}
WAVEFORM = {"newton": 0, "pn35": 1, "surrogate": 2}
FLAG_OUT_OF_BAND, FLAG_TAU_NONPOSITIVE, FLAG_TAYLOR_INVALID, FLAG_NONFINITE, FLAG_EMPTY = 1, 2, 4, 8, 64
FLAG_SURROGATE_FALLBACK = 32
FLAG_FSTAT_DEGENERATE = 128
K_MAX = 64
T_SUN = 4.925490947641267e-6


class SFTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("libsft status %d: %s" % (status, msg))
        self.status = status


class DataDesc(ctypes.Structure):
    _fields_ = [("n_sft", ctypes.c_int32), ("n_samples", ctypes.c_int32), ("t_sft", ctypes.c_double),
                ("k_lo", ctypes.c_int32), ("n_bins", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("kernel", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("waveform", ctypes.c_int32), ("t_ref", ctypes.c_int32), ("beta_switch", ctypes.c_double),
                ("a_plus", ctypes.c_double),
                ("a_cross", ctypes.c_double), ("tsun", ctypes.c_double), ("delta_max", ctypes.c_double),
                ("surrogate", ctypes.c_void_p)]


class Bank(ctypes.Structure):
    _fields_ = [("mc", ctypes.c_void_p), ("q", ctypes.c_void_p), ("t_c", ctypes.c_void_p),
                ("phi_c", ctypes.c_void_p), ("a_first", ctypes.c_void_p), ("a_last", ctypes.c_void_p),
                ("sky", ctypes.c_void_p)]


class Out(ctypes.Structure):
    _fields_ = [("zp", ctypes.c_void_p), ("zx", ctypes.c_void_p), ("hhp", ctypes.c_void_p),
                ("hhx", ctypes.c_void_p), ("rho", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("mismatch", ctypes.c_void_p), ("hhpx", ctypes.c_void_p), ("twoF", ctypes.c_void_p),
                ("n_used", ctypes.c_void_p)]


class SurrogateDesc(ctypes.Structure):
    _fields_ = [("hidden", ctypes.c_int32), ("layers", ctypes.c_int32), ("head", ctypes.c_int32),
                ("inference", ctypes.c_int32), ("mc_lo", ctypes.c_double), ("mc_hi", ctypes.c_double),
                ("q_lo", ctypes.c_double), ("q_hi", ctypes.c_double), ("lt_lo", ctypes.c_double),
                ("lt_hi", ctypes.c_double), ("c_phi", ctypes.c_double), ("c_amp", ctypes.c_double),
                ("judge_tol", ctypes.c_double)]


ORDER = {"given": 0, "track": 1}


class Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("chunk_groups", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("order", ctypes.c_int32)]

    def as_dict(self):
        return {"block": self.block, "chunk_groups": self.chunk_groups, "persistent": self.persistent,
                "order": {v: k for k, v in ORDER.items()}.get(self.order, self.order)}


EXPORTS = ["sft_load_data", "sft_free_data", "sft_default_opts", "sft_template_bank_scan",
           "sft_inner_product", "sft_last_error", "sft_version", "sft_kernel_timing", "sft_kernel_times",
           "sft_get_tuning", "sft_set_tuning", "sft_autotune", "sft_plan_create", "sft_plan_launch",
           "sft_plan_destroy", "sft_surrogate_param_count", "sft_surrogate_create", "sft_surrogate_free",
           "sft_surrogate_get_params", "sft_surrogate_targets", "sft_surrogate_loss_grad", "sft_surrogate_adam",
           "sft_surrogate_train", "sft_surrogate_infer", "sft_template_bank_scan_noalloc",
           "sft_set_ephemeris", "sft_make_sfts", "sft_load_strain", "sft_waveform_series", "sft_td_product",
           "sft_probe_issue_rate"]
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024

_lib = None


def lib():
    """Load libsft.so (raises if it is missing: build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsft.so not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    L.sft_load_data.argtypes = [ctypes.POINTER(DataDesc), P, P, P, P, P, P, ctypes.POINTER(P)]
    L.sft_load_data.restype = ctypes.c_int32
    L.sft_free_data.argtypes = [P]
    L.sft_free_data.restype = None
    L.sft_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.sft_default_opts.restype = None
    L.sft_template_bank_scan.argtypes = [P, ctypes.POINTER(Bank), ctypes.c_int64, ctypes.POINTER(Opts),
                                         ctypes.POINTER(Out), P]
    L.sft_template_bank_scan.restype = ctypes.c_int32
    L.sft_set_ephemeris.argtypes = [P, P, P]
    L.sft_make_sfts.argtypes = [P, P, P, P, P, P]
    L.sft_make_sfts.restype = ctypes.c_int32
    L.sft_load_strain.argtypes = [P, P, P, P, P, P, P]
    L.sft_load_strain.restype = ctypes.c_int32
    Dd = ctypes.c_double
    L.sft_waveform_series.argtypes = [ctypes.c_int32, Dd, Dd, Dd, Dd, Dd, Dd, Dd, ctypes.c_int64, P, P, Dd, Dd, P, P, P]
    L.sft_waveform_series.restype = ctypes.c_int32
    L.sft_td_product.argtypes = [P, P, ctypes.c_int64, Dd, Dd, P, P]
    L.sft_td_product.restype = ctypes.c_int32
    L.sft_set_ephemeris.restype = ctypes.c_int32
    L.sft_template_bank_scan_noalloc.argtypes = L.sft_template_bank_scan.argtypes
    L.sft_template_bank_scan_noalloc.restype = ctypes.c_int32
    D = ctypes.c_double
    L.sft_inner_product.argtypes = [P, D, D, D, D, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Opts),
                                    P, P, P, P, P, P]
    L.sft_inner_product.restype = ctypes.c_int32
    L.sft_last_error.argtypes = []
    L.sft_last_error.restype = ctypes.c_char_p
    L.sft_version.argtypes = []
    L.sft_version.restype = ctypes.c_char_p
    L.sft_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    L.sft_get_tuning.restype = ctypes.c_int32
    L.sft_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    L.sft_set_tuning.restype = ctypes.c_int32
    L.sft_autotune.argtypes = [P, ctypes.POINTER(Bank), ctypes.c_int64, ctypes.POINTER(Opts), ctypes.POINTER(Out),
                               P, ctypes.c_int32, ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_float)]
    L.sft_autotune.restype = ctypes.c_int32
    L.sft_plan_create.argtypes = [P, ctypes.POINTER(Bank), ctypes.c_int64, ctypes.POINTER(Opts),
                                  ctypes.POINTER(Out), ctypes.POINTER(P)]
    L.sft_plan_create.restype = ctypes.c_int32
    L.sft_plan_launch.argtypes = [P, P]
    L.sft_plan_launch.restype = ctypes.c_int32
    L.sft_plan_destroy.argtypes = [P]
    L.sft_plan_destroy.restype = None
    L.sft_kernel_timing.argtypes = [ctypes.c_int32]
    L.sft_kernel_timing.restype = ctypes.c_int32
    L.sft_kernel_times.argtypes = [P, ctypes.c_int32]
    L.sft_kernel_times.restype = ctypes.c_int32
    L.sft_probe_issue_rate.argtypes = [ctypes.c_int32, P, P]
    L.sft_probe_issue_rate.restype = ctypes.c_int32
    I32, I64, F32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.sft_surrogate_param_count.argtypes = [I32, I32]
    L.sft_surrogate_param_count.restype = I64
    L.sft_surrogate_create.argtypes = [ctypes.POINTER(SurrogateDesc), P, ctypes.POINTER(P)]
    L.sft_surrogate_create.restype = I32
    L.sft_surrogate_free.argtypes = [P]
    L.sft_surrogate_free.restype = None
    L.sft_surrogate_get_params.argtypes = [P, P]
    L.sft_surrogate_get_params.restype = I32
    L.sft_surrogate_targets.argtypes = [P, P, P, P, I64, D, P, P, P]
    L.sft_surrogate_targets.restype = I32
    L.sft_surrogate_loss_grad.argtypes = [P, P, P, I64, P, P, P]
    L.sft_surrogate_loss_grad.restype = I32
    L.sft_surrogate_adam.argtypes = [P, F32, P]
    L.sft_surrogate_adam.restype = I32
    L.sft_surrogate_train.argtypes = [P, P, P, I64, I32, I32, F32, F32, P, P]
    L.sft_surrogate_train.restype = I32
    L.sft_surrogate_infer.argtypes = [P, P, I64, P, P, P]
    L.sft_surrogate_infer.restype = I32
    _lib = L
    return L


def last_error() -> str:
    return lib().sft_last_error().decode()


def _check(status: int):
    if status != SFT_OK:
        raise SFTError(status, last_error())


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


T_REF = {"mid": 0, "start": 1}


def make_opts(K=8, kernel="auto", precision="fp32_kahan", waveform="newton", beta_switch=1e-7,
              a_plus=1.0, a_cross=0.0, tsun=T_SUN, delta_max=0.0, surrogate=None, t_ref="mid") -> Opts:
    o = Opts()
    lib().sft_default_opts(ctypes.byref(o))
    o.K = int(K)
    o.kernel = KERNEL[kernel] if isinstance(kernel, str) else int(kernel)
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.waveform = WAVEFORM[waveform] if isinstance(waveform, str) else int(waveform)
    o.t_ref = T_REF[t_ref] if isinstance(t_ref, str) else int(t_ref)
    o.beta_switch = float(beta_switch)
    o.a_plus = float(a_plus)
    o.a_cross = float(a_cross)
    o.tsun = float(tsun)
    o.delta_max = float(delta_max)
    if surrogate is not None:
        o.surrogate = surrogate.handle
        o._surrogate_ref = surrogate   # keep the network alive with the options
    return o


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class StrainDesc(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int32), ("n_samples", ctypes.c_int32), ("n_total", ctypes.c_int64),
                ("dt", ctypes.c_double), ("t0", ctypes.c_double), ("k_lo", ctypes.c_int32),
                ("n_bins", ctypes.c_int32), ("psd_w", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("s_white", ctypes.c_double)]


def _strain_desc(x_t, n, dt, t0, k_lo, n_bins, psd_w, storage="f32", s_white=0.0):
    if not x_t.is_cuda or not x_t.is_contiguous() or x_t.dim() != 2 or str(x_t.dtype) != "torch.float64":
        raise ValueError("strain must be a contiguous [n_det, n_total] float64 device tensor")
    return StrainDesc(int(x_t.shape[0]), int(n), int(x_t.shape[1]), float(dt), float(t0), int(k_lo), int(n_bins),
                      int(psd_w), STORAGE[storage], float(s_white))


def make_sfts(x_t, n, dt, k_lo, n_bins, psd_w, t0=0.0, stream=None, s_white=0.0):
    """SFT band bins, PSD estimates and keep flags of every segment of the strain series x_t
    [n_det, n_total] (device FP64): tensors [n_det, n_seg, n_bins] complex128, float64, int32."""
    import torch
    d = _strain_desc(x_t, n, dt, t0, k_lo, n_bins, psd_w, s_white=s_white)
    n_seg = d.n_total // int(n)
    bins = torch.empty((d.n_det, n_seg, int(n_bins), 2), dtype=torch.float64, device=x_t.device)
    psd = torch.empty((d.n_det, n_seg, int(n_bins)), dtype=torch.float64, device=x_t.device)
    keep = torch.empty((d.n_det, n_seg), dtype=torch.int32, device=x_t.device)
    _check(lib().sft_make_sfts(ctypes.byref(d), _tp(x_t), _tp(bins), _tp(psd), _tp(keep), _stream_ptr(stream)))
    return torch.view_as_complex(bins), psd, keep


def waveform_series(mc, t_c, t0, dt, n, waveform="newton", q=1.0, phi_c=0.0, fplus=None, fcross=None,
                    a_plus=1.0, a_cross=0.0, quantities=False, tsun=T_SUN, device="cuda", stream=None):
    """Strain h [n] of one template at t_j = t0 + j dt on the device (and the waveform
    quantities [n, 5] A, phi, f, fdot, fddot when asked)."""
    import torch
    h = torch.empty(int(n), dtype=torch.float64, device=device)
    qv = torch.empty((int(n), 5), dtype=torch.float64, device=device) if quantities else None
    for a in (fplus, fcross):
        if a is not None and (not a.is_cuda or not a.is_contiguous() or a.numel() != int(n)):
            raise ValueError("antenna patterns must be contiguous device tensors of n samples")
    _check(lib().sft_waveform_series(WAVEFORM[waveform], float(mc), float(q), float(t_c), float(phi_c), float(tsun),
                                     float(t0), float(dt), int(n), _tp(fplus), _tp(fcross), float(a_plus),
                                     float(a_cross), _tp(h), _tp(qv), _stream_ptr(stream)))
    return (h, qv) if quantities else h


def td_product(x_t, y_t, dt, psd, stream=None):
    """(2 / S) dt sum_j x_j y_j on the device (white one-sided PSD S)."""
    if x_t.numel() != y_t.numel() or not x_t.is_contiguous() or not y_t.is_contiguous():
        raise ValueError("x and y must be contiguous and of one length")
    out = ctypes.c_double()
    _check(lib().sft_td_product(_tp(x_t), _tp(y_t), int(x_t.numel()), float(dt), float(psd), _stream_ptr(stream),
                                ctypes.byref(out)))
    return out.value


class SFTData:
    """Device-resident whitened SFTs (owns an sft_data handle)."""

    def __init__(self, t_start, n_samples, t_sft, k_lo, x_bins, psd, fplus=None, fcross=None,
                 storage="f32", stream=None):
        xb = np.asarray(x_bins)
        if np.iscomplexobj(xb):
            xb = np.stack([xb.real, xb.imag], axis=-1)
        xb = np.ascontiguousarray(xb, dtype=np.float64)
        n_sft, n_bins = xb.shape[0], xb.shape[1]
        psd = np.ascontiguousarray(np.broadcast_to(psd, (n_sft, n_bins)), dtype=np.float64)
        self._keep = (_f64(t_start), xb, psd, _f64(fplus), _f64(fcross))
        desc = DataDesc(n_sft, int(n_samples), float(t_sft), int(k_lo), n_bins, STORAGE[storage], 0)
        h = ctypes.c_void_p()
        st = _stream_ptr(stream) if stream is not None else None
        _check(lib().sft_load_data(ctypes.byref(desc), _p(self._keep[0]), _p(xb), _p(psd),
                                   _p(self._keep[3]), _p(self._keep[4]), st, ctypes.byref(h)))
        self.handle = h
        self.n_sft, self.n_bins, self.storage = n_sft, n_bins, storage
        self.t_sft, self.n_samples, self.k_lo = float(t_sft), int(n_samples), int(k_lo)
        self._keep = None

    @classmethod
    def from_strain(cls, x_t, n, dt, k_lo, n_bins, psd_w, t0=0.0, fplus=None, fcross=None, storage="f32",
                    stream=None, s_white=0.0):
        """SFTs made on the device from the strain series x_t [n_det, n_total] (device FP64),
        whitened by their own PSD estimates; gaps (segments with a non-finite sample) dropped.
        fplus, fcross: [n_det, n_seg] per segment, or None."""
        d = _strain_desc(x_t, n, dt, t0, k_lo, n_bins, psd_w, storage, s_white)
        fp = None if fplus is None else np.ascontiguousarray(fplus, dtype=np.float64).ravel()
        fx = None if fcross is None else np.ascontiguousarray(fcross, dtype=np.float64).ravel()
        h = ctypes.c_void_p()
        nr = ctypes.c_int32()
        _check(lib().sft_load_strain(ctypes.byref(d), _tp(x_t), _p(fp), _p(fx), _stream_ptr(stream),
                                     ctypes.byref(h), ctypes.byref(nr)))
        self = cls.__new__(cls)
        self.handle = h
        self.n_sft, self.n_bins, self.storage = int(nr.value), int(n_bins), storage
        self.t_sft, self.n_samples, self.k_lo = float(dt) * int(n), int(n), int(k_lo)
        self._keep = None
        return self

    @classmethod
    def from_workload(cls, w, storage="f32", stream=None):
        return cls(w.t_start, w.n_samples, w.t_sft, w.k_lo, w.x_bins, w.psd, w.fplus, w.fcross,
                   storage=storage, stream=stream)

    def set_ephemeris(self, eph, stream=None):
        """Detector r/c, v/c, a/c per SFT row at its midpoint, [n_sft, 9] (Doppler form)."""
        e = np.ascontiguousarray(np.reshape(eph, (self.n_sft, 9)), dtype=np.float64)
        _check(lib().sft_set_ephemeris(self.handle, e.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream)))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().sft_free_data(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bank_to_device(bank: Dict[str, np.ndarray], device="cuda"):
    import torch
    out = {}
    for k in ("mc", "q", "t_c", "phi_c", "sky"):
        if k in bank and bank[k] is not None:
            out[k] = torch.as_tensor(np.ascontiguousarray(bank[k], dtype=np.float64), device=device)
    for k in ("a_first", "a_last"):
        if k in bank and bank[k] is not None:
            out[k] = torch.as_tensor(np.ascontiguousarray(bank[k], dtype=np.int32), device=device)
    return out


def alloc_out(n: int, device="cuda", mismatch=False, fstat=False):
    import torch
    out = {"zp": torch.empty((n, 2), dtype=torch.float64, device=device),
           "zx": torch.empty((n, 2), dtype=torch.float64, device=device),
           "hhp": torch.empty(n, dtype=torch.float64, device=device),
           "hhx": torch.empty(n, dtype=torch.float64, device=device),
           "rho": torch.empty(n, dtype=torch.float64, device=device),
           "flags": torch.empty(n, dtype=torch.int32, device=device),
           "n_used": torch.empty(n, dtype=torch.int32, device=device)}
    if mismatch:
        out["mismatch"] = torch.zeros(n, dtype=torch.float64, device=device)
    if fstat:
        out["hhpx"] = torch.empty(n, dtype=torch.float64, device=device)
        out["twoF"] = torch.empty(n, dtype=torch.float64, device=device)
    return out


def _tp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _bank_struct(bank_t):
    for k, t in bank_t.items():
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("bank array %s must be a contiguous device tensor" % k)
    sky = bank_t.get("sky")
    if sky is not None and tuple(sky.shape) != (int(bank_t["mc"].numel()), 3):
        raise ValueError("bank sky must be [n, 3]")
    return Bank(_tp(bank_t.get("mc")), _tp(bank_t.get("q")), _tp(bank_t.get("t_c")),
                _tp(bank_t.get("phi_c")), _tp(bank_t.get("a_first")), _tp(bank_t.get("a_last")), _tp(sky))


def _out_struct(out):
    return Out(_tp(out["zp"]), _tp(out["zx"]), _tp(out["hhp"]), _tp(out["hhx"]), _tp(out["rho"]),
               _tp(out["flags"]), _tp(out.get("mismatch")), _tp(out.get("hhpx")), _tp(out.get("twoF")),
               _tp(out.get("n_used")))


def template_bank_scan(data: SFTData, bank_t, opts: Opts, out=None, stream=None, n=None):
    """Asynchronous bank scan on ``stream`` (default: torch's current stream)."""
    n = int(bank_t["mc"].numel()) if n is None else int(n)
    if out is None:
        out = alloc_out(n, device=bank_t["mc"].device)
    b = _bank_struct(bank_t)
    o = _out_struct(out)
    _check(lib().sft_template_bank_scan(data.handle, ctypes.byref(b), n, ctypes.byref(opts),
                                        ctypes.byref(o), _stream_ptr(stream)))
    return out


def template_bank_scan_noalloc(data: SFTData, bank_t, opts: Opts, out, stream=None, n=None):
    """Asynchronous bank scan whose workspace is the library's own device array (no device
    allocation by the library; ``out`` must be given)."""
    n = int(bank_t["mc"].numel()) if n is None else int(n)
    b = _bank_struct(bank_t)
    o = _out_struct(out)
    _check(lib().sft_template_bank_scan_noalloc(data.handle, ctypes.byref(b), n, ctypes.byref(opts),
                                                ctypes.byref(o), _stream_ptr(stream)))
    return out


def inner_product(data: SFTData, mc, t_c, phi_c=0.0, q=1.0, a_first=0, a_last=None, opts: Opts = None):
    """One template, host in / host out (synchronous)."""
    opts = make_opts() if opts is None else opts
    a_last = data.n_sft - 1 if a_last is None else a_last
    zp = (ctypes.c_double * 2)()
    zx = (ctypes.c_double * 2)()
    hhp, hhx, rho = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    fl = ctypes.c_uint32()
    _check(lib().sft_inner_product(data.handle, float(mc), float(q), float(t_c), float(phi_c),
                                   int(a_first), int(a_last), ctypes.byref(opts),
                                   ctypes.cast(zp, ctypes.c_void_p), ctypes.cast(zx, ctypes.c_void_p),
                                   ctypes.cast(ctypes.pointer(hhp), ctypes.c_void_p),
                                   ctypes.cast(ctypes.pointer(hhx), ctypes.c_void_p),
                                   ctypes.cast(ctypes.pointer(rho), ctypes.c_void_p),
                                   ctypes.cast(ctypes.pointer(fl), ctypes.c_void_p)))
    return {"zp": zp[0] + 1j * zp[1], "zx": zx[0] + 1j * zx[1], "hhp": hhp.value, "hhx": hhx.value,
            "rho": rho.value, "flags": fl.value}


def kernel_timing(n: int):
    """Record HIP events around the scan kernel of the next n bank scans (0 stops)."""
    _check(lib().sft_kernel_timing(int(n)))


def kernel_times(max_records: int = 4096):
    """Elapsed milliseconds of the recorded scan kernels (waits for them)."""
    buf = (ctypes.c_float * max_records)()
    n = lib().sft_kernel_times(ctypes.cast(buf, ctypes.c_void_p), max_records)
    return [buf[i] for i in range(min(n, max_records))]


PROBE = {"v_fma_f32": 0, "v_rcp_f32": 1, "v_fma_f64": 2, "v_fma_f32+int32": 3}


def probe_issue_rate(op: str, stream=None) -> float:
    """VALU wave-instructions per second that one instruction sustains on the device (probe
    of 16 independent chains per lane; see sft_probe_issue_rate)."""
    r = ctypes.c_double()
    _check(lib().sft_probe_issue_rate(PROBE[op], ctypes.cast(ctypes.byref(r), ctypes.c_void_p), _stream_ptr(stream)))
    return r.value


def get_tuning(data: SFTData) -> Tuning:
    t = Tuning()
    _check(lib().sft_get_tuning(data.handle, ctypes.byref(t)))
    return t


def set_tuning(data: SFTData, block=0, chunk_groups=0, persistent=0, order="given"):
    """Launch shape and bank order ("given" or "track": sorted on the device) of the handle."""
    t = Tuning(int(block), int(chunk_groups), int(persistent), ORDER[order] if isinstance(order, str) else int(order))
    _check(lib().sft_set_tuning(data.handle, ctypes.byref(t)))


def autotune(data: SFTData, bank_t, opts: Opts, out=None, stream=None, reps=2):
    """Time candidate launch shapes on this bank; the best is kept by the handle."""
    n = int(bank_t["mc"].numel())
    out = alloc_out(n, device=bank_t["mc"].device) if out is None else out
    b, o = _bank_struct(bank_t), _out_struct(out)
    t = Tuning()
    ms = ctypes.c_float()
    _check(lib().sft_autotune(data.handle, ctypes.byref(b), n, ctypes.byref(opts), ctypes.byref(o),
                              _stream_ptr(stream), int(reps), ctypes.byref(t), ctypes.byref(ms)))
    return t, ms.value


class Plan:
    """A bank scan captured into a HIP graph (fixed bank/output pointers)."""

    def __init__(self, data: SFTData, bank_t, opts: Opts, out=None):
        n = int(bank_t["mc"].numel())
        self.out = alloc_out(n, device=bank_t["mc"].device) if out is None else out
        self._bank_t, self._data = bank_t, data
        b, o = _bank_struct(bank_t), _out_struct(self.out)
        h = ctypes.c_void_p()
        _check(lib().sft_plan_create(data.handle, ctypes.byref(b), n, ctypes.byref(opts), ctypes.byref(o),
                                     ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(lib().sft_plan_launch(self.handle, _stream_ptr(stream)))
        return self.out

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().sft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------------- surrogate
def surrogate_param_count(hidden: int, layers: int) -> int:
    return int(lib().sft_surrogate_param_count(int(hidden), int(layers)))


INFERENCE = {"fp64": 0, "fp64_bf16w": 1, "bf16x3": 2, "bf16": 3}


class Surrogate:
    """The learned-surrogate network (owns an sft_surrogate handle on the current device).

    params: FP32 values (any float array) packed layer by layer, W [n_in][n_out] then b.
    Ranges: mc, q and ln(tau) of the input normalisation; c_phi, c_amp output scales;
    head = 1 adds the analytic 1PN + 1.5PN phase; judge_tol the mismatch tolerance.
    inference: "fp64", "fp64_bf16w" (FP64 evaluation of BF16-rounded weights), "bf16x3"
    (BF16 matrix cores with split operands) or "bf16"; weights_bf16 = 1 is "fp64_bf16w"."""

    def __init__(self, params, hidden=128, layers=4, head=1, weights_bf16=0, mc=(1.19, 1.21), q=(1.0, 2.0),
                 ln_tau=(6.39, 9.74), c_phi=1.0, c_amp=1.0, judge_tol=1e-4, inference=None):
        mode = INFERENCE[inference] if inference is not None else (1 if weights_bf16 else 0)
        self.desc = SurrogateDesc(int(hidden), int(layers), int(head), mode, float(mc[0]),
                                  float(mc[1]), float(q[0]), float(q[1]), float(ln_tau[0]), float(ln_tau[1]),
                                  float(c_phi), float(c_amp), float(judge_tol))
        self.P = surrogate_param_count(hidden, layers)
        par = np.ascontiguousarray(params, dtype=np.float32)
        if par.size != self.P:
            raise ValueError("expected %d parameters, got %d" % (self.P, par.size))
        h = ctypes.c_void_p()
        _check(lib().sft_surrogate_create(ctypes.byref(self.desc), _p(par), ctypes.byref(h)))
        self.handle = h

    def get_params(self) -> np.ndarray:
        out = np.empty(self.P, dtype=np.float32)
        _check(lib().sft_surrogate_get_params(self.handle, _p(out)))
        return out

    def targets(self, mc_t, q_t, tau_t, tsun=T_SUN, stream=None):
        """Device FP64 mc, q, tau -> device FP32 inputs u [n][3] and targets y [n][2]."""
        import torch
        n = int(mc_t.numel())
        u = torch.empty((n, 3), dtype=torch.float32, device=mc_t.device)
        y = torch.empty((n, 2), dtype=torch.float32, device=mc_t.device)
        _check(lib().sft_surrogate_targets(self.handle, _tp(mc_t), _tp(q_t), _tp(tau_t), n, float(tsun), _tp(u),
                                           _tp(y), _stream_ptr(stream)))
        return u, y

    def loss_grad(self, u, y, stream=None):
        """FP32 loss (mean over rows of the squared residual norm) and gradient [P] (device)."""
        import torch
        n = int(u.shape[0])
        loss = torch.empty(1, dtype=torch.float32, device=u.device)
        grad = torch.empty(self.P, dtype=torch.float32, device=u.device)
        _check(lib().sft_surrogate_loss_grad(self.handle, _tp(u), _tp(y), n, _tp(loss), _tp(grad),
                                             _stream_ptr(stream)))
        return loss, grad

    def adam(self, lr, stream=None):
        _check(lib().sft_surrogate_adam(self.handle, float(lr), _stream_ptr(stream)))

    def train(self, u, y, batch=4096, epochs=1, lr=1e-3, lr_min=1e-5, stream=None) -> np.ndarray:
        """Mini-batch Adam over device (u, y) in row order; returns the mean loss per epoch."""
        buf = np.zeros(int(epochs), dtype=np.float32)
        _check(lib().sft_surrogate_train(self.handle, _tp(u), _tp(y), int(u.shape[0]), int(batch), int(epochs),
                                         float(lr), float(lr_min), _stream_ptr(stream), _p(buf)))
        return buf

    def infer(self, u64, stream=None):
        """The scan's network evaluation (in the handle's inference mode): u [n][3] -> y [n][2],
        dy/du_tau [n][2] (device, FP64)."""
        import torch
        n = int(u64.shape[0])
        y = torch.empty((n, 2), dtype=torch.float64, device=u64.device)
        dy = torch.empty((n, 2), dtype=torch.float64, device=u64.device)
        _check(lib().sft_surrogate_infer(self.handle, _tp(u64), n, _tp(y), _tp(dy), _stream_ptr(stream)))
        return y, dy

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().sft_surrogate_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
