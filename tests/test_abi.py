"""The C ABI: every symbol declared in include/sft.h is exported by libsft.so, and the
host-side validation returns the documented codes (no GPU needed: these paths fail
before any device call)."""
import ctypes
import os
import re

import pytest

from paper_2502_11823_amd import sft

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sft_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L = sft.lib()
    names = _declared()
    assert set(names) == set(sft.EXPORTS)
    for name in names:
        assert hasattr(L, name), name


def test_version_and_defaults():
    assert b"gfx950" in sft.lib().sft_version()
    o = sft.Opts()
    sft.lib().sft_default_opts(ctypes.byref(o))
    assert (o.K, o.kernel, o.precision, o.waveform, o.t_ref) == (8, 2, 1, 0, 0)
    assert o.beta_switch == 1e-7 and o.a_plus == 1.0 and o.a_cross == 0.0
    assert abs(o.tsun - 4.925490947641267e-6) < 1e-20
    assert o.surrogate is None
    assert ctypes.sizeof(sft.DataDesc) == 32 and ctypes.sizeof(sft.Opts) == 72
    assert ctypes.sizeof(sft.Out) == 80 and ctypes.sizeof(sft.SurrogateDesc) == 88
    assert ctypes.sizeof(sft.Tuning) == 16


def test_load_data_rejects_bad_descriptors():
    L = sft.lib()
    h = ctypes.c_void_p()
    one = (ctypes.c_double * 8)()
    assert L.sft_load_data(None, one, one, one, None, None, None, ctypes.byref(h)) == -1
    for desc in [sft.DataDesc(0, 64, 32.0, 0, 33, 1, 0),      # no SFTs
                 sft.DataDesc(2, 63, 32.0, 0, 32, 1, 0),      # odd n
                 sft.DataDesc(2, 64, 32.0, 10, 30, 1, 0),     # band beyond n/2
                 sft.DataDesc(2, 64, -1.0, 0, 33, 1, 0),      # bad T
                 sft.DataDesc(2, 64, 32.0, 0, 33, 7, 0)]:     # bad storage
        st = L.sft_load_data(ctypes.byref(desc), one, one, one, None, None, None, ctypes.byref(h))
        assert st == -1, (desc.n_sft, desc.n_samples, desc.k_lo, desc.storage)
        assert sft.last_error().startswith("sft_load_data")


def test_scan_rejects_bad_options():
    L = sft.lib()
    b, o = sft.Bank(), sft.Out()
    opts = sft.make_opts()
    assert L.sft_template_bank_scan(None, ctypes.byref(b), 1, ctypes.byref(opts), ctypes.byref(o), None) == -1
    z = (ctypes.c_double * 2)()
    assert L.sft_inner_product(None, 1.2, 1.0, 100.0, 0.0, 0, 0, ctypes.byref(opts), z, z, None, None, None, None) == -1


def test_issue_probe_host_validation():
    L = sft.lib()
    r = ctypes.c_double()
    assert L.sft_probe_issue_rate(0, None, None) == -1
    assert L.sft_probe_issue_rate(4, ctypes.cast(ctypes.byref(r), ctypes.c_void_p), None) == -1
    assert L.sft_probe_issue_rate(-1, ctypes.cast(ctypes.byref(r), ctypes.c_void_p), None) == -1
    assert sft.last_error().startswith("sft_probe_issue_rate")
    assert sorted(sft.PROBE.values()) == [0, 1, 2, 3]


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(sft, "_lib", None)
    monkeypatch.setattr(sft, "LIB_PATH", "/nonexistent/libsft.so")
    with pytest.raises(RuntimeError):
        sft.lib()


def test_surrogate_host_validation(orc):
    L = sft.lib()
    assert sft.surrogate_param_count(128, 4) == 50306 == orc.mlp_param_count(128, 4)
    assert sft.surrogate_param_count(32, 2) == orc.mlp_param_count(32, 2)
    assert sft.surrogate_param_count(0, 4) == 0
    h = ctypes.c_void_p()
    par = (ctypes.c_float * 16)()
    good = dict(hidden=32, layers=2, head=1, inference=0, mc_lo=1.0, mc_hi=2.0, q_lo=1.0, q_hi=2.0,
                lt_lo=6.0, lt_hi=9.0, c_phi=1.0, c_amp=0.01, judge_tol=1e-4)
    for bad, code in [(dict(hidden=4), -4), (dict(layers=9), -4), (dict(mc_hi=1.0), -1),
                      (dict(lt_hi=5.0), -1), (dict(c_phi=0.0), -1), (dict(judge_tol=-1.0), -1),
                      (dict(inference=7), -1), (dict(inference=2, hidden=48), -5), (dict(inference=3, hidden=256), -5)]:
        d = sft.SurrogateDesc(**dict(good, **bad))
        assert L.sft_surrogate_create(ctypes.byref(d), par, ctypes.byref(h)) == code, bad
        assert sft.last_error().startswith("sft_surrogate_create")
    assert L.sft_surrogate_create(None, par, ctypes.byref(h)) == -1
    assert L.sft_surrogate_targets(None, None, None, None, 1, 1.0, None, None, None) == -1
    assert L.sft_surrogate_infer(None, None, 1, None, None, None) == -1
    assert L.sft_surrogate_loss_grad(None, None, None, 1, None, None, None) == -1
    assert L.sft_surrogate_train(None, None, None, 1, 16, 1, 1e-3, 1e-5, None, None) == -1
    assert L.sft_surrogate_adam(None, 1e-3, None) == -1
    # a surrogate scan without a network is rejected before any device work
    opts = sft.make_opts(waveform="surrogate")
    b, o = sft.Bank(), sft.Out()
    fake = ctypes.c_void_p(1)
    assert L.sft_template_bank_scan(fake, ctypes.byref(b), 1, ctypes.byref(opts), ctypes.byref(o), None) == -1
    assert "surrogate" in sft.last_error()
