"""The checked build of the library (FDKOD_CHECKS: kernels count the events
the host's planning should rule out) on the small parity cases, in a process
of its own that loads libfdkod_checked.so: every counter stays zero and every
case still matches the FP64 oracle."""

import json
import os
import subprocess
import sys

import pytest

from gpu_common import log, require_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CHECKED = os.path.join(ROOT, "paper_1708_07515_amd", "libfdkod_checked.so")


def test_checked_build_counts_no_events():
    require_gpu()
    assert os.path.exists(CHECKED), "libfdkod_checked.so is missing: build with __graft_entry__.build()"
    env = dict(os.environ, FDKOD_LIB=CHECKED)
    out = subprocess.run([sys.executable, "-u", os.path.join(HERE, "checked_cases.py")], env=env,
                         stdout=subprocess.PIPE, stderr=subprocess.PIPE, timeout=240, text=True)
    log(out.stdout)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = [json.loads(x) for x in out.stdout.splitlines() if x.startswith("{")]
    assert len(lines) == 8
    for rec in lines:
        tol = 1e-4 if rec["case"][5] == "f32" else 2e-3
        assert rec["counts"] == [0, 0, 0, 0], rec
        assert rec["rel_rmse"] <= tol, rec


def test_unchecked_build_refuses_counts():
    require_gpu()
    import paper_1708_07515_amd as pkg
    if os.environ.get("FDKOD_LIB"):
        pytest.skip("another library is loaded")
    with pytest.raises(pkg.FdkodError) as ei:
        pkg.check_counts()
    assert ei.value.code == "E_UNSUPPORTED"
