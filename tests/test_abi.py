"""CPU-side checks of the C-ABI boundary: the built library loads, exports every
function declared in include/afq.h with the binding's signature table, and
rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_2003_01831_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "afq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(afq_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libafq.so is not built; run `python -m paper_2003_01831_amd.build`")
    return _lib.load()


def test_header_and_binding_agree():
    assert _declared() == sorted(_lib.SIGNATURES)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_version(lib):
    assert lib.afq_version() >> 16 == 1


def test_null_arguments_are_rejected(lib):
    h = C.c_void_p()
    assert lib.afq_system_create(None, 8, 2, 2, 4, None, None, None, 0.0, 0, None, 0) == -1
    assert b"out" in lib.afq_last_error()
    assert lib.afq_system_create(C.byref(h), 0, 2, 2, 4, None, None, None, 0.0, 0, None, 0) == -1
    assert lib.afq_system_create(C.byref(h), 8, 0, 2, 4, None, None, None, 0.0, 0, None, 0) == -1
    assert lib.afq_system_create(C.byref(h), 8, 2, 2, 0, None, None, None, 0.0, 0, None, 0) == -1
    assert lib.afq_system_create(C.byref(h), 300, 200, 2, 4, None, None, None, 0.0, 0, None, 0) == -6
    assert lib.afq_system_create(C.byref(h), 8, 2, 2, 4, None, None, None, 0.0, 0, None, 0) == -1
    assert lib.afq_walkers_create(C.byref(h), None, 4, None, None) == -1
    assert lib.afq_step(None, None, 1, 0.01, None, 0, 5, 0.0, 6, None, None, None, None) == -1
    assert lib.afq_energy(None, None, None, None, None, None) == -1
    assert lib.afq_energy_backward(None, None, 1.0, None, None, None) == -1
    assert lib.afq_walkers_get(None, None, None, None, None, None) == -1
    assert lib.afq_walkers_stats(None, None, None) == -1
    assert lib.afq_fields_generate(0, 0, 0, -1, 1, 1, None, None) == -1
    # destroy is NULL-safe
    assert lib.afq_system_destroy(None) == 0
    assert lib.afq_walkers_destroy(None) == 0
    assert lib.afq_batch_destroy(None) == 0


def test_python_binding_fails_loudly_without_library(tmp_path):
    saved = _lib._lib
    try:
        _lib._lib = None
        with pytest.raises(RuntimeError, match="not found"):
            _lib.load(str(tmp_path / "missing.so"))
    finally:
        _lib._lib = saved
