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


def test_check_counts_on_unchecked_build():
    # the ordinary library is not a checked build: the counters are refused
    # (before any device call), and bad arguments are reported first
    if os.environ.get("FDKOD_LIB"):
        pytest.skip("another library is loaded")
    lib = pkg.load_library()
    arr = (ctypes.c_int64 * 4)()
    assert lib.fdkod_check_counts(arr, 4, 1) == 3
    assert lib.fdkod_check_counts(None, 4, 1) == 1
    assert lib.fdkod_check_counts(arr, 5, 1) == 1


@pytest.mark.parametrize("args", [dict(n=64, p=90, r=512.0, s=2), dict(n=37, p=50, r=150.0, s=3, skip=1),
                                  dict(n=512, p=360, r=2048.0, s=3), dict(n=300, p=96, r=1200.0, s=2, skip=1),
                                  dict(n=48, p=60, r=192.0, s=0, nz=20)])
def test_cost_counts_match_the_oracle(args):
    """The library's host count of the two cost terms of Sec. 2.2 (eq. (6),
    eq. (7)) equals the oracle's, which counts them from its own plan."""
    from oracle import fdkod as ofdkod
    cropped, updates = pkg.cost_counts(**args)
    n, p, r = args["n"], args["p"], args["r"]
    want_c, want_u = ofdkod.cost_counts(n, args.get("nz") or n, p, r, args.get("s", 0), args.get("skip", 0))
    if args.get("s", 0) == 0:
        want_c, want_u = 0, n * n * (args.get("nz") or n) * p
    assert (cropped, updates) == (want_c, want_u)


def test_choose_s_minimises_the_predicted_time():
    c1, c2 = 3.7e-10, 6e-10
    for n, p in [(256, 360), (512, 360), (1024, 720), (2000, 720)]:
        s, ms = pkg.choose_s(n, p, 4.0 * n, s_max=6, costs=(c1, c2))
        times = {}
        for cand in range(0, 7):
            if (1 << cand) > n:
                continue
            c, u = pkg.cost_counts(n, p, 4.0 * n, s=cand)
            times[cand] = c1 * u + c2 * c
        assert s == min(times, key=times.get) and ms == pytest.approx(times[s])
        # eq. (8): the optimum grows with N (2^s = sqrt(C1 N / C2) up to the
        # squares' margins)
    s_small, _ = pkg.choose_s(256, 360, 1024.0, costs=(c1, c2))
    s_large, _ = pkg.choose_s(2000, 720, 8000.0, costs=(c1, c2))
    assert s_large > s_small


def test_batch_workloads_are_valid_plans():
    """The benchmark's batched workloads (32 volumes of N = 128..512, 256 of
    N = 32..64): every volume, with s from the cost model, passes the
    library's validation, and the sizes follow the workload's seed."""
    import bench
    from synth import configs
    for bw in (configs.C4, configs.C4S):
        vols = bench.batch_volumes(bw, pkg)
        assert len(vols) == bw.count
        assert {v["n"] for v in vols} <= set(bw.sizes)
        for v in vols:
            assert v["p"] == round(bw.p_per_n * v["n"]) and v["r"] == bw.r_per_n * v["n"]
            pkg.validate(**v)
        assert vols == bench.batch_volumes(bw, pkg)
