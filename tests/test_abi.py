"""The C ABI without a GPU: the library builds and loads, exports every
entry point declared in include/nll.h, and argument errors are reported
without touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "nll.h")).read()
    return sorted(set(re.findall(r"^(?:nll_status|void|const char\*)\s+(nll_\w+)\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2003_12875_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_2003_12875_amd import build
        build.build()
    return _native.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 14
    from paper_2003_12875_amd import _native
    assert set(names) == set(_native.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, -9):
        assert L.nll_status_string(code)
    assert L.nll_status_string(0) == b"ok"


def test_argument_errors_without_device(L):
    from paper_2003_12875_amd import _native
    h = ctypes.c_void_p()
    assert L.nll_create_model(None, ctypes.byref(h)) == -1
    assert L.nll_eval(None, None, None) == -1
    assert L.nll_eval_grad(None, None, None, None) == -1
    assert L.nll_eval_batched_noalloc(None, 1, None, None, None, None, None) == -1
    assert L.nll_sync(None, None) == -1
    assert L.nll_set_schedule(None, None) == -1
    assert L.nll_get_info(None, None) == -1
    assert L.nll_set_weights(None, None) == -1
    assert L.nll_hf_create(None, ctypes.byref(h)) == -1
    assert L.nll_hf_set_data(None, None, None, None, None) == -1
    assert L.nll_hf_eval(None, None, None, None) == -1
    assert L.nll_hf_sync(None, None) == -1
    L.nll_destroy_model(None)  # no-op
    L.nll_hf_destroy(None)  # no-op


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2003_12875_amd import _native
    monkeypatch.setattr(_native, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _native.lib()


def test_binned_descriptor_errors_without_device(L):
    """Descriptor validation happens before any device call."""
    from paper_2003_12875_amd import _native
    lo = (ctypes.c_double * 2)(0.0, -5.0)
    hi = (ctypes.c_double * 2)(10.0, 5.0)
    mods = (_native.HFModifier * 2)()
    mods[0].type, mods[0].sample, mods[0].param = 1, 0, 0
    mods[1].type, mods[1].sample, mods[1].param, mods[1].hi, mods[1].lo = 2, 0, 1, 1.1, 0.9
    d = _native.HFDesc()
    d.n_bins, d.n_samples, d.n_param = 100, 1, 2
    d.param_lo, d.param_hi = lo, hi
    d.n_modifiers, d.modifiers = 2, mods
    h = ctypes.c_void_p()
    for field, bad, code in (("n_samples", 0, -1), ("n_samples", 9, -2), ("n_param", 0, -1), ("n_param", 33, -2)):
        keep = getattr(d, field)
        setattr(d, field, bad)
        assert L.nll_hf_create(ctypes.byref(d), ctypes.byref(h)) == code, field
        setattr(d, field, keep)
    mods[1].lo = 0.0  # a normsys factor must be positive
    assert L.nll_hf_create(ctypes.byref(d), ctypes.byref(h)) == -1
    mods[1].lo = 0.9
    mods[1].sample = 3  # no such sample
    assert L.nll_hf_create(ctypes.byref(d), ctypes.byref(h)) == -1
    mods[1].sample = 0
    mods[1].type = 7
    assert L.nll_hf_create(ctypes.byref(d), ctypes.byref(h)) == -1
