"""Build libmsc.so (host C++ + HIP kernels for gfx950) in-tree.

Every source is compiled by hipcc for --offload-arch=gfx950 with packed
FP32 instructions disabled, then linked into
paper_2609_19116_amd/libmsc.so.  Run ``python -m paper_2609_19116_amd.build``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
OUT = PKG / "libmsc.so"
BUILD = ROOT / "_build"

SOURCES = [
    CSRC / "host" / "circuit.cpp",
    CSRC / "host" / "prescreen_compile.cpp",
    CSRC / "host" / "sampler.cpp",
    CSRC / "host" / "stats.cpp",
    CSRC / "host" / "order.cpp",
    CSRC / "host" / "camps.cpp",
    CSRC / "host" / "capi.cpp",
    CSRC / "kernels" / "mps.hip",
    CSRC / "kernels" / "prescreen.hip",
    CSRC / "kernels" / "sampler.hip",
    CSRC / "kernels" / "batch.hip",
    CSRC / "kernels" / "camps.hip",
    CSRC / "kernels" / "twosite.hip",
    CSRC / "kernels" / "lx.hip",
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          f"-I{ROOT / 'include'}", f"-I{CSRC}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops"]


def _compile(src: Path) -> Path:
    obj = BUILD / (src.stem + (".hip.o" if src.suffix == ".hip" else ".o"))
    if src.suffix == ".hip":
        cmd = [HIPCC, "-x", "hip", *DEVICE, *COMMON, "-c", str(src), "-o", str(obj)]
    else:
        # host-only sources still include the HIP runtime headers
        cmd = [HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *COMMON, "-c", str(src),
               "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        warn = [ln for ln in r.stderr.splitlines()
                if "packed-fp32-ops" not in ln and ln.strip()]
        if warn:
            sys.stderr.write("\n".join(warn) + "\n")
    return obj


def build(verbose: bool = True) -> Path:
    if shutil.which(HIPCC) is None and not Path(HIPCC).exists():
        raise RuntimeError("hipcc not found")
    BUILD.mkdir(exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT.with_suffix(".so.tmp")
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", str(tmp), *map(str, objs),
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build()
