"""Build libfdkod.so (gfx950) in-tree with hipcc.

    python -m paper_1708_07515_amd.build

Compiles every .hip file of csrc/ into one shared library next to this file.
Packed FP32 instructions are disabled for the device code (-packed-fp32-ops).
"""

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfdkod.so")
# the checked build: the same sources with FDKOD_CHECKS defined (kernels count
# the events the host's planning should rule out; see fdkod_check_counts)
LIB_CHECKED = os.path.join(HERE, "libfdkod_checked.so")

# Per-file options.  The learned convolutions keep their MFMA accumulators in
# ordinary VGPRs (no AGPR copies), which lowers their register count to five
# waves per SIMD.
FILE_FLAGS = {"k_learned.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose=False, jobs=8, checked=False):
    """Compile every .hip file of csrc/ and link libfdkod.so (checked=True:
    libfdkod_checked.so with FDKOD_CHECKS defined); returns its path."""
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    objdir = os.path.join(HERE, "_build_checked" if checked else "_build")
    os.makedirs(objdir, exist_ok=True)
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument",
             "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    if checked:
        flags.append("-DFDKOD_CHECKS")
    procs, objs = [], []
    for src in srcs:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [hipcc()] + flags + FILE_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs)
            procs = []
    _wait(procs)
    lib = LIB_CHECKED if checked else LIB
    tmp = lib + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if out.returncode != 0:
        raise RuntimeError("link failed:\n" + out.stdout.decode())
    os.replace(tmp, lib)
    return lib


def _wait(procs):
    errs = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode()
        if p.returncode != 0:
            errs.append(f"{src}:\n{text}")
        elif text.strip() and "warning" in text and "packed-fp32-ops" not in text:
            sys.stderr.write(text)
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, checked="--checked" in sys.argv))
