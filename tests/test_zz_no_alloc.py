"""The allocation-free bank scan (sft_template_bank_scan_noalloc) against the allocating one.

Both are called through the C ABI on the same data and banks; the no-alloc scan keeps its
workspace in the library's own device array, so its launch may use fewer chunks and its
FP64 combination of partial sums runs in another order: the two agree to the parity bar
of the other GPU tests (e <= 1e-6 in noise units on z, 1e-5 on rho, 1e-6 on hh, flags
bit-exact), not bitwise.  Two calls in a row, the second with a smaller bank, check that the
shared array's previous contents do not leak into a result.
"""
import ctypes

import numpy as np
import pytest

from paper_2502_11823_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_11823_amd import sft  # noqa: E402

from parity_helpers import compare, orc_scan  # noqa: E402


def _host(out):
    o = {k: v.cpu().numpy() for k, v in out.items()}
    o["zp"] = o["zp"][:, 0] + 1j * o["zp"][:, 1]
    o["zx"] = o["zx"][:, 0] + 1j * o["zx"][:, 1]
    o["flags"] = o["flags"].astype(np.uint32)
    return o


def _as_reference(g):
    """The allocating scan's result in the oracle's dictionary form (no rounding ties)."""
    r = dict(g)
    r["tie"] = np.ones(len(g["rho"]))
    return r


def _pair(data, bank, opts):
    bt = sft.bank_to_device(bank)
    n = len(bank["mc"])
    ref = sft.template_bank_scan(data, bt, opts, out=sft.alloc_out(n))
    # poison the outputs so that a missing write shows
    out = sft.alloc_out(n)
    for v in out.values():
        v.fill_(-7)
    sft.template_bank_scan_noalloc(data, bt, opts, out)
    torch.cuda.synchronize()
    return _host(ref), _host(out)


def test_noalloc_matches_allocating_scan_twice():
    w = synth.ground(seed=11, n_templates=200_000, n_slots=64, n_det=2, k_lo=40, k_hi=470,
                     t_end_pad=300.0)
    data = sft.SFTData.from_workload(w, storage="f32")
    opts = sft.make_opts(K=8, kernel="auto", precision="fp32_kahan", a_plus=1.0, a_cross=1.0)
    # one timestamp group per chunk: the allocating scan's 64 chunks of partial sums
    # (666 MB for 2e5 templates) do not fit the scratch, so the no-alloc scan merges chunks
    sft.set_tuning(data, block=128, chunk_groups=1, persistent=0)
    ref, got = _pair(data, w.bank, opts)
    print("first call: 200000 templates, %d SFT rows" % w.n_sft, flush=True)
    compare(got, _as_reference(ref), label="noalloc vs scan (2e5)")
    # and a sample against the oracle
    idx = np.arange(0, 200_000, 997)
    o = orc_scan(w, w.subset(idx), K=8, kernel="auto", a_plus=1.0, a_cross=1.0)
    compare({k: v[idx] for k, v in got.items()}, o, label="noalloc vs oracle")

    # second call, smaller bank and another launch shape, into the same scratch
    w2 = synth.ground(seed=12, n_templates=3000, n_slots=48, n_det=3, k_lo=40, k_hi=470,
                      t_end_pad=300.0)
    data2 = sft.SFTData.from_workload(w2, storage="f32")
    ref2, got2 = _pair(data2, w2.bank, opts)
    print("second call: 3000 templates, %d SFT rows" % w2.n_sft, flush=True)
    compare(got2, _as_reference(ref2), label="noalloc vs scan (3000)")
    o2 = orc_scan(w2, w2.bank, K=8, kernel="auto", a_plus=1.0, a_cross=1.0)
    compare(got2, o2, label="noalloc vs oracle (3000)")
    data.close()
    data2.close()


def test_noalloc_rejects_oversized_bank_and_surrogate():
    w = synth.ground(seed=13, n_templates=64, n_slots=16, n_det=1, k_lo=40, k_hi=470, t_end_pad=300.0)
    data = sft.SFTData.from_workload(w, storage="f32")
    opts = sft.make_opts(K=8)
    n = sft.NOALLOC_SCRATCH_BYTES // 52 + 1        # one chunk of partial sums no longer fits
    bt = {"mc": torch.full((n,), 1.2, dtype=torch.float64, device="cuda"),
          "t_c": torch.full((n,), 1e6, dtype=torch.float64, device="cuda")}
    out = sft.alloc_out(n)
    with pytest.raises(sft.SFTError) as ei:
        sft.template_bank_scan_noalloc(data, bt, opts, out)
    assert ei.value.status == -4 and "scratch" in str(ei.value)
    o = sft.make_opts(K=4, kernel="dirichlet", precision="fp32_kahan")
    o.waveform = 2                      # surrogate: rejected before the network is looked at
    b, ou = sft._bank_struct(bt), sft._out_struct(out)
    st = sft.lib().sft_template_bank_scan_noalloc(data.handle, ctypes.byref(b), 64, ctypes.byref(o),
                                                  ctypes.byref(ou), None)
    assert st in (-1, -5)
    data.close()
