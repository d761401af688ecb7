"""Build libmixgraph.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2509_15948_amd.build

Every source under csrc/ is compiled to an object in csrc/_build/ (in
parallel) and linked into paper_2509_15948_amd/libmixgraph.so.  The packed
FP32 instructions are disabled for all device code.

The build fails if a kernel needs more private (scratch) memory than
SCRATCH_ALLOWED grants it (none for any kernel not listed): the runtime
allocates scratch for a queue when a kernel that uses it is first dispatched
there, and that allocation fails, aborting the queue, when the process's
device memory is full, so scratch users are kept few and small.  The
compiler's resource remarks name every kernel and its scratch bytes per lane.
"""
from __future__ import annotations

import concurrent.futures
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmixgraph.so")
BUILD = os.path.join(CSRC, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MG_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-Wno-unknown-warning-option", "-Wno-unused-value"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


_REMARK = "-Rpass-analysis=kernel-resource-usage"

# kernel (mangled-name stem) -> scratch bytes per lane it may use: the EQ
# window kernels spill a few registers at the 64-register cap that gives two
# blocks per CU
SCRATCH_ALLOWED = {"_ZN2mg8k_eq_bwd": 32}


def _allowed(kernel: str) -> int:
    return max([b for k, b in SCRATCH_ALLOWED.items() if kernel.startswith(k)] + [0])


def scratch_kernels(remarks: str) -> list:
    """(kernel, bytes per lane) of every kernel whose remarks report scratch."""
    out, name = [], None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name is not None and int(m.group(1)) > 0:
            out.append((name, int(m.group(1))))
    return out


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + [_REMARK, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + FLAGS + [_REMARK, "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    bad = [(k, b) for k, b in scratch_kernels(r.stderr) if b > _allowed(k)]
    if bad:
        raise RuntimeError(f"{os.path.basename(src)}: kernels using more scratch memory than allowed: {bad}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    build()
    sys.exit(0)
