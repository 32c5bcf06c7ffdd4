"""Build the HIP library for gfx950: ``python paper_2308_00497_amd/build.py``.

Compiles every source under ``csrc/`` with hipcc (in parallel) into
``_build/`` at the repository root and links ``lib/libfft_mi355x.so`` inside
the package, where the Python binding looks for it.  Always rebuilds from
scratch: this is also the "does it build" check.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libfft_mi355x.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Sources of the library, in link order.
SOURCES = [
    "k_single.hip",
    "k_pass.hip",
    "k_single64.hip",
    "k_pass64.hip",
    "k_real.hip",
    "k_real64.hip",
    "k_ops.hip",
    "k_nd.hip",
    "k_misc.hip",
    "ragged.hip",
    "noalloc.hip",
    "plan.cpp",
    "autotune.cpp",
    "capi.cpp",
]

COMMON = [
    "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off: ordinary float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


# per-kernel register and scratch use, as reported by the compiler
RESOURCES = os.path.join(BUILD, "kernel_resources.json")


def _resources(remarks: list[str]) -> list[dict]:
    """Kernel entries (name, VGPRs, spills, scratch bytes per lane) from the
    compiler's kernel-resource-usage remarks."""
    out, cur = [], None
    for line in remarks:
        msg = line.split("remark:", 1)[-1].strip()
        if msg.startswith("Function Name:"):
            cur = {"name": msg.split(":", 1)[1].split("[")[0].strip()}
            out.append(cur)
        elif cur is not None and ":" in msg:
            key, val = msg.split(":", 1)
            val = val.split("[")[0].strip()
            if key in ("VGPRs", "AGPRs", "VGPRs Spill", "SGPRs Spill", "ScratchSize [bytes/lane]",
                       "Occupancy [waves/SIMD]", "LDS Size [bytes/block]"):
                try:
                    cur[key] = int(val)
                except ValueError:
                    pass
    return out


def _compile(src: str) -> tuple[str, str, list[dict]]:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    r = subprocess.run(cmd, capture_output=True, text=True)
    lines = r.stderr.splitlines()
    remarks = [l for l in lines if "kernel-resource-usage" in l]
    # the host pass does not know the packed-fp32 feature; drop that notice
    err = "\n".join(l for l in lines if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    return obj, err, _resources(remarks)


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    objs, kernels = [], []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, err, res in ex.map(_compile, SOURCES):
            objs.append(obj)
            kernels += res
            if verbose and err.strip():
                print(err, file=sys.stderr)
    with open(RESOURCES, "w") as f:
        json.dump({"arch": ARCH, "kernels": kernels}, f, indent=0)
    tmp = LIB + ".tmp%d" % os.getpid()
    # -z defs: an unresolved symbol fails the build instead of the first load
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Wl,-z,defs", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
