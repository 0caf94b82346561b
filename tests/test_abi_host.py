"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid parameters without touching a device."""

import ctypes
import os
import re

import pytest

import paper_1708_07515_amd as pkg
from paper_1708_07515_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "fdkod.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdkod_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = pkg.load_library()
    names = header_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.EXPORTS, f"binding does not declare {name}"


def test_version_and_status_strings():
    lib = pkg.load_library()
    assert lib.fdkod_version() >= 100
    for code in range(7):
        assert lib.fdkod_status_str(code)
    assert lib.fdkod_status_str(99) == b"unknown status"


@pytest.mark.parametrize("args,code", [
    (dict(n=1, p=90, r=512.0), "E_ARG"),
    (dict(n=5000, p=90, r=1e5), "E_ARG"),
    (dict(n=64, p=0, r=512.0), "E_ARG"),
    (dict(n=64, p=90, r=512.0, store=7), "E_ARG"),
    (dict(n=64, p=90, r=44.0), "E_GEOMETRY"),            # R <= (N-1)/sqrt(2)
    (dict(n=64, p=90, r=float("nan")), "E_GEOMETRY"),
    (dict(n=64, p=90, r=512.0, s=7), "E_GEOMETRY"),      # 2^s > N
    (dict(n=64, p=90, r=512.0, s=2, skip=3), "E_GEOMETRY"),
    (dict(n=64, p=7, r=512.0, s=2), "E_GEOMETRY"),       # P < 2 D
    (dict(n=64, p=90, r=512.0, nz=-1), "E_ARG"),
    (dict(n=64, p=90, r=512.0, s=2, decim=2), "E_ARG"),
    (dict(n=64, p=90, r=512.0, s=2, decim="sinc", taps=3), "E_ARG"),
    (dict(n=64, p=90, r=512.0, s=2, decim="sinc", taps=8), "E_ARG"),
    (dict(n=64, p=90, r=512.0, s=2, taps=4), "E_ARG"),                  # the triangle has 2
    (dict(n=64, p=90, r=512.0, s=2, rows=2), "E_ARG"),
    (dict(n=64, p=90, r=512.0, s=2, interp=2), "E_ARG"),
    (dict(n=64, p=23, r=512.0, s=2, decim="sinc", taps=6), "E_GEOMETRY"),  # P < taps D
])
def test_validation_codes(args, code):
    with pytest.raises(pkg.FdkodError) as ei:
        pkg.validate(**args)
    assert ei.value.code == code


@pytest.mark.parametrize("args", [dict(n=64, p=90, r=512.0, s=2), dict(n=2000, p=720, r=8000.0, s=4),
                                  dict(n=64, p=8, r=45.0, s=2, skip=0), dict(n=3, p=1, r=2.0),
                                  dict(n=64, p=90, r=512.0, s=2, rows="cone"),
                                  dict(n=64, p=90, r=512.0, s=0, rows="cone"),
                                  dict(n=64, p=90, r=512.0, s=2, decim="sinc", taps=6, interp="cubic"),
                                  dict(n=64, p=24, r=512.0, s=2, decim="sinc", taps=6)])
def test_validation_accepts(args):
    pkg.validate(**args)


def test_null_arguments_are_rejected():
    lib = pkg.load_library()
    assert lib.fdkod_validate(None) == 1
    assert lib.fdkod_plan_create(None, 0, None) == 1
    assert lib.fdkod_plan_info(None, None) == 1
    assert lib.fdkod_filter(None, None, None, None) == 1
    assert lib.fdkod_backproject(None, None, None, None, None) == 1
    assert lib.fdkod_plan_destroy(None) == 0
    assert lib.fdkod_last_error()


def test_plan_create_reports_invalid_before_device():
    lib = pkg.load_library()
    prm = _lib.Params(64, 0, 90, 10.0, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    assert lib.fdkod_plan_create(ctypes.byref(prm), 0, ctypes.byref(h)) == 2
    assert h.value is None


def test_batch_validation_before_device():
    lib = pkg.load_library()
    good = _lib.Params(32, 0, 45, 128.0, 1, 0, 0, 0)
    bad = _lib.Params(32, 0, 45, 10.0, 1, 0, 0, 0)          # R too small
    mixed = _lib.Params(32, 0, 45, 128.0, 1, 0, 2, 0)       # another store type
    h = ctypes.c_void_p()
    arr = (_lib.Params * 2)(good, bad)
    assert lib.fdkod_batch_create(arr, 2, 0, ctypes.byref(h)) == 2
    arr = (_lib.Params * 2)(good, mixed)
    assert lib.fdkod_batch_create(arr, 2, 0, ctypes.byref(h)) == 1
    for knob in (_lib.Params(32, 0, 45, 128.0, 1, 0, 0, 0, 0, 1, 0),     # cone-corrected rows
                 _lib.Params(32, 0, 45, 128.0, 1, 0, 0, 1, 4, 0, 0),     # windowed sinc
                 _lib.Params(32, 0, 45, 128.0, 1, 0, 0, 0, 0, 0, 1)):    # cubic shift
        arr = (_lib.Params * 2)(good, knob)
        assert lib.fdkod_batch_create(arr, 2, 0, ctypes.byref(h)) == 3
    assert lib.fdkod_batch_create(arr, 0, 0, ctypes.byref(h)) == 1
    assert h.value is None
    assert lib.fdkod_batch_run(None, None) == 1
    assert lib.fdkod_batch_replay(None, None) == 1
    assert lib.fdkod_batch_destroy(None) == 0
    assert lib.fdkod_get_tuning(None, None) == 1
    assert lib.fdkod_tune(None, None, None, None, None, None) == 1
