"""Shared helpers of the GPU parity tests: run the HIP scan and the FP64 oracle on the
same inputs and compare them element by element (the metric is described in
test_gpu_parity.py)."""
import numpy as np

import oracle
from paper_2502_11823_amd import sft

KERN = {"dirichlet": oracle.K_DIRICHLET, "fresnel": oracle.K_FRESNEL, "auto": oracle.K_AUTO}


def gpu_scan(data, bank, mismatch=False, fstat=False, **kw):
    import torch
    opts = sft.make_opts(**kw)
    bt = sft.bank_to_device(bank)
    res = sft.template_bank_scan(data, bt, opts, out=sft.alloc_out(len(bank["mc"]), mismatch=mismatch,
                                                                    fstat=fstat))
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in res.items()}
    out["zp"] = out["zp"][:, 0] + 1j * out["zp"][:, 1]
    out["zx"] = out["zx"][:, 0] + 1j * out["zx"][:, 1]
    out["flags"] = out["flags"].astype(np.uint32)
    return out


def orc_scan(w, bank, x_bins=None, psd=None, **kw):
    od = oracle.SFTData(w.t_start, w.n_samples, w.t_sft, w.k_lo, w.x_bins if x_bins is None else x_bins,
                        w.psd if psd is None else psd, w.fplus, w.fcross)
    kw = dict(kw)
    kw.pop("precision", None)
    kw["kernel"] = KERN[kw.get("kernel", "auto")]
    kw.pop("surrogate", None)
    kw["wf"] = {"newton": oracle.WF_NEWTON, "pn35": oracle.WF_PN35,
                "surrogate": oracle.WF_SURROGATE}[kw.pop("waveform", "newton")]
    kw["t_ref"] = {"mid": oracle.REF_MID, "start": oracle.REF_START}[kw.pop("t_ref", "mid")]
    return oracle.scan(od, bank["mc"], bank["t_c"], phi_c=bank["phi_c"], q=bank.get("q"),
                       a_first=bank["a_first"], a_last=bank["a_last"], **kw)


def compare(g, o, idx=None, tol_z=1e-6, tol_rho=1e-5, tol_hh=1e-6, label="", noise_scale=None):
    """noise_scale: optional (hh+, hhx) of the template's full SFT set, used in place of the
    reported norm when the stored band cut some of its norm bins (OUT_OF_BAND)."""
    if idx is not None:
        g = {k: v[idx] for k, v in g.items()}
    ok = o["tie"] > 1e-9
    n_tie = int(np.sum(~ok))
    assert n_tie <= max(1, len(ok) // 1000), "too many rounding ties: %d" % n_tie
    hh = np.maximum(o["hhp"], 1e-300)
    hx = np.maximum(o["hhx"], 1e-300)
    if noise_scale is not None:
        hh = np.maximum(hh, noise_scale[0])
        hx = np.maximum(hx, noise_scale[1])
    ep = np.abs(g["zp"] - o["zp"]) / np.maximum(np.abs(o["zp"]), np.sqrt(hh))
    ex = np.where(o["hhx"] > 0, np.abs(g["zx"] - o["zx"]) / np.maximum(np.abs(o["zx"]), np.sqrt(hx)), 0.0)
    eh = np.abs(g["hhp"] - o["hhp"]) / np.maximum(o["hhp"], 1e-300)
    er = np.abs(g["rho"] - o["rho"]) / np.maximum(o["rho"], 1.0)
    print("%s: n=%d max e(z+)=%.3e e(zx)=%.3e e(hh)=%.3e e(rho)=%.3e ties=%d"
          % (label, len(ok), ep[ok].max(), ex[ok].max(), eh[ok].max(), er[ok].max(), n_tie))
    w = int(np.argmax(np.where(ok, np.maximum(ep, er), -1.0)))
    if max(ep[w], er[w]) > tol_z:
        print("  worst template %d: flags gpu %d orc %d, z+ gpu %r orc %r, hh+ gpu %r orc %r, rho gpu %r orc %r"
              % (w, g["flags"][w], o["flags"][w], g["zp"][w], o["zp"][w], g["hhp"][w], o["hhp"][w],
                 g["rho"][w], o["rho"][w]))
    assert np.array_equal(g["flags"][ok], o["flags"][ok]), (g["flags"][ok], o["flags"][ok])
    if "n_used" in g and "n_used" in o:
        assert np.array_equal(g["n_used"], o["n_used"]), "SFT rows used differ"
    assert ep[ok].max() <= tol_z
    assert ex[ok].max() <= tol_z
    assert eh[ok].max() <= tol_hh
    assert er[ok].max() <= tol_rho
    return ep[ok].max()


def compare_fstat(g, o, tol_f=2e-5, tol_hh=1e-6, label=""):
    """F-statistic outputs: the cross norm relative to sqrt(hh+ hhx) (<= 1e-6, as the other
    norms) and 2F in noise units, |d2F| / max(2F, 4) (<= 2e-5: 2F is a squared SNR, whose bar
    is twice rho's 1e-5; 4 is the mean of 2F in noise).  The degenerate flag is compared with
    the other flags by compare(); templates whose det N / (hh+ hhx) lies within 1e-6 of the
    threshold 1e-2 could be decided differently by rounding and are left out."""
    d = (o["hhp"] * o["hhx"] - o["hhpx"]**2) / np.maximum(o["hhp"] * o["hhx"], 1e-300)
    ok = (np.abs(d - 1e-2) > 1e-6) & (o["tie"] > 1e-9)
    sc = np.sqrt(np.maximum(o["hhp"] * o["hhx"], 1e-300))
    ec = np.abs(g["hhpx"] - o["hhpx"]) / sc
    ef = np.abs(g["twoF"] - o["twoF"]) / np.maximum(o["twoF"], 4.0)
    print("%s: n=%d max e(hh+x)=%.3e e(2F)=%.3e degenerate %d, near threshold %d"
          % (label, int(ok.sum()), ec[ok].max(), ef[ok].max(),
             int(np.sum((o["flags"] & oracle.F_FSTAT_DEGENERATE) != 0)), int(np.sum(~ok))))
    assert np.array_equal(g["flags"][ok], o["flags"][ok])
    assert ec[ok].max() <= tol_hh
    assert ef[ok].max() <= tol_f
    return ef[ok].max()
