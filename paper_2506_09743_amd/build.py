"""Builds libqmc.so (HIP, gfx950) in-tree with hipcc.

Each source compiles to an object in its own hipcc process (in parallel),
then one hipcc call links the shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqmc.so")
# longest compiles first
SOURCES = ["qmc_form_bf16.hip", "qmc_form_bf16_x1.hip", "qmc_form_fp32.hip", "qmc_form_backflow.hip",
           "qmc_form_backflow_max.hip", "qmc_form_fp64.hip", "qmc_grad.hip", "qmc_api.hip", "qmc_kernels.hip"]
ARCH = os.environ.get("QMC_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # no packed FP32 instructions in device code.  The feature exists only
    # for the device target, but the driver cannot forward an option pair
    # such as "-Xclang -target-feature" through -Xarch_device, so the host
    # pass sees it too and prints that it ignores it (HOST_NOTE below).
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
HOST_NOTE = "'-packed-fp32-ops' is not a recognized feature for this target (ignoring feature)"


def _quiet(text: str) -> str:
    return "".join(l for l in text.splitlines(True) if l.strip() != HOST_NOTE)


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _jobs() -> int:
    try:
        n = int(os.environ.get("MAX_JOBS", "0"))
    except ValueError:
        n = 0
    return max(1, min(n or (os.cpu_count() or 1), len(SOURCES), 16))


def build(extra=(), out: str = LIB, verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [hipcc(), *FLAGS, *extra, "-c", "-o", obj, os.path.join(CSRC, src)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, r

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = [(s, r) for s, _, r in results if r.returncode != 0]
    for s, _, r in results:
        if verbose or r.returncode != 0:
            sys.stderr.write(_quiet(r.stdout + r.stderr))
    if failed:
        raise RuntimeError("hipcc failed on " + ", ".join(s for s, _ in failed) + ":\n" +
                           _quiet(failed[0][1].stderr)[-4000:])
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + [o for _, o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if verbose or r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
    if r.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(extra=sys.argv[1:], verbose=True)
    print(LIB)
