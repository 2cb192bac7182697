"""Build libgcb.so (HIP for gfx950) in-tree with hipcc.

Each translation unit is compiled separately (in parallel) and linked into
paper_2007_14401_amd/libgcb.so.  The binary64 push and adjoint units are
compiled with -ffp-contract=off so that their arithmetic is evaluated exactly
as written (no fused multiply-add: the parity build, GCB_ARITH_EXACT); the
contracted binary64 push (GCB_ARITH_FAST, the production build) is the same
source compiled with -ffp-contract=fast; the mixed-precision units may
contract and use the hardware's binary32 reciprocal and square root.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.environ.get("GCB_LIB_OUT", os.path.join(HERE, "libgcb.so"))
BUILD = os.environ.get("GCB_BUILD_DIR", BUILD)

ARCH = os.environ.get("GCB_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          *os.environ.get("GCB_HIPCC_FLAGS", "").split()]
# The precision form's binary32 division and square root need not be
# correctly rounded (its error is measured against the binary64 oracle and its
# switch decisions near the thresholds are re-taken in binary64).
FAST_F32 = ["-fno-hip-fp32-correctly-rounded-divide-sqrt"]
UNITS = {
    "gcb_host.hip": ["-ffp-contract=off"],
    "gcb_push_f64.hip": ["-ffp-contract=off"],
    "gcb_push_f64_fast.hip": ["-ffp-contract=fast"],
    "gcb_adjoint.hip": ["-ffp-contract=off"],
    "gcb_adjoint3.hip": ["-ffp-contract=off"],
    "gcb_push_mixed.hip": FAST_F32,
    "gcb_sort.hip": ["-ffp-contract=off"],
    "gcb_util.hip": ["-ffp-contract=off"],
    "gcb_gr.hip": ["-ffp-contract=off"],
    "gcb_gr_fast.hip": ["-ffp-contract=fast"],
    "gcb_gr_mixed.hip": FAST_F32,
    "gcb_push3_f64.hip": ["-ffp-contract=off"],
    "gcb_push3_f64_fast.hip": ["-ffp-contract=fast"],
    "gcb_push3_mixed.hip": FAST_F32,
}


def hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return h


def _compile(src: str, flags) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [hipcc(), *COMMON, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(UNITS), os.cpu_count() or 4)) as ex:
        futs = {ex.submit(_compile, s, f): s for s, f in UNITS.items()}
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp"
    # every symbol must resolve at link time (a missing definition would
    # otherwise surface only when the library is loaded)
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", "-Wl,--no-undefined", *objs,
           "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
