"""Builds the HIP transport library (libmcv.so) for gfx950, in-tree, and the
primitive cost probe (libmcv_probe.so, measurement only)."""

from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmcv.so")
SOURCES = ["mcv_transport.hip", "mcv_api.cpp"]
PROBE_LIB = os.path.join(HERE, "libmcv_probe.so")
PROBE_SOURCES = ["mcv_probe.hip"]
ARCH = os.environ.get("MCV_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libmcv.so")
    return exe


def build(verbose: bool = False, out: str = LIB, extra=(), sources=None) -> str:
    """Compile every source for gfx950 and link libmcv.so next to this file
    (or to `out`, with extra compiler flags, for variants)."""
    objs = []
    sources = SOURCES if sources is None else sources
    bdir = os.path.join(HERE, "_build") if out == LIB else out + ".build"
    os.makedirs(bdir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
              # packed FP32 instructions are kept out of generated code
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              # binary32 division and square root to ~2.5 ulp instead of
              # correctly rounded: far inside the 1e-5 parity bars, and the
              # correctly rounded sequences are ~10 instructions each
              "-fno-hip-fp32-correctly-rounded-divide-sqrt",
              "-I", os.path.join(HERE, "..", "include"), "-Wall"] + list(extra)
    for src in sources:
        obj = os.path.join(bdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else ["-x", "hip"]
        cmd = [hipcc()] + common + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr)
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


def build_probe(verbose: bool = False) -> str:
    """The cost probe: the library's sources plus the probe kernels."""
    return build(verbose, out=PROBE_LIB, sources=PROBE_SOURCES)


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_probe(verbose=True))
