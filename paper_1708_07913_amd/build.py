"""Build libsq.so (HIP kernels for gfx950 + the C ABI host code) in-tree.

The host code is plain C++ compiled by g++ against the HIP runtime API.

    python -m paper_1708_07913_amd.build

The kernels are compiled with packed FP32 instructions disabled; the host file
is compiled without floating-point contraction (the projector sphere test
r^2 <= r_c^2 must be evaluated exactly as written).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsq.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DEVICE_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics",
                # the plane loops of the recurrence kernels must unroll fully
                # (register-resident columns are indexed by plane)
                "-mllvm", "-pragma-unroll-threshold=1000000"]
# optional extra -D definitions for the kernels (tuning knobs, e.g.
# "SQ_MOMENTS_AHEAD=3 SQ_LANCZOS_AHEAD=3")
DEVICE_FLAGS += ["-D" + d for d in os.environ.get("SQ_DEVICE_DEFINES", "").split()]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
              "-I/opt/rocm/include"]
CXX = os.environ.get("CXX", "g++")

# recurrence kernels are split into several translation units by cube size so
# that the build parallelises
CUBE_GROUPS = [[3, 5, 7, 9, 11, 13], [15, 17, 19], [21], [23], [25], [27], [29], [31], [33], [35], [37]]
# the two-row shapes of the 21-27-point cubes: a second build of the same
# source (SQ_TWO_ROWS=1, kernels in namespace sq::two_rows)
TWO_ROW_GROUPS = [[21], [23], [25], [27]]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    cmds = []
    objs = []
    src_k = os.path.join(CSRC, "sq_kernels.hip")
    parts = [(g, 0) for g in CUBE_GROUPS] + [(g, 1) for g in TWO_ROW_GROUPS]
    for i, (group, two) in enumerate(parts):
        cubes = " ".join(f"X({c})" for c in group)
        obj = os.path.join(BUILD, f"sq_kernels_{i}.o")
        defs = [f"-DSQ_CUBES={cubes}", "-DSQ_PART=%d" % i, "-DSQ_TWO_ROWS=%d" % two]
        cmds.append([HIPCC, *DEVICE_FLAGS, *defs, "-c", src_k, "-o", obj])
        objs.append(obj)
    obj = os.path.join(BUILD, "sq_common.o")
    cmds.append([HIPCC, *DEVICE_FLAGS, "-DSQ_COMMON_ONLY", "-c", src_k, "-o", obj])
    objs.append(obj)
    obj = os.path.join(BUILD, "sq_api.o")
    cmds.append([CXX, *HOST_FLAGS, "-c", os.path.join(CSRC, "sq_api.cpp"), "-o", obj])
    objs.append(obj)
    with ThreadPoolExecutor(jobs) as ex:
        for r in ex.map(_run, cmds):
            if verbose and r.stderr:
                sys.stderr.write(r.stderr)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
