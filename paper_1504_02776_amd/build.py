"""Builds the HIP transport library (libmcv.so) for gfx950, in-tree, and the
primitive cost probe (libmcv_probe.so, measurement only)."""

from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmcv.so")
SOURCES = ["mcv_transport.hip", "mcv_reduce.hip", "mcv_adjoint.hip", "mcv_determ.hip",
           "mcv_api.cpp"]
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
              # multiply-adds fused only within one source expression: every
              # kernel that inlines the same device code (plain, trace, event
              # and batched launches) then rounds it the same way
              "-ffp-contract=on",
              # binary32 denormals flushed: division and square root then
              # need no frexp/ldexp range scaling (identical results for
              # normal operands; nothing on the path is that small, and
              # histograms and tables are binary64, which keeps denormals)
              "-fgpu-flush-denormals-to-zero",
              "-I", os.path.join(HERE, "..", "include"), "-Wall"] + list(extra)
    cmds = []
    for src in sources:
        obj = os.path.join(bdir, src + ".o")
        cmds.append([hipcc()] + common + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # the translation units are independent: compile them side by side
    procs = [subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
             for c in cmds]
    for c, pr in zip(cmds, procs):
        so, err = pr.communicate()
        if pr.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(c)}\n{so}\n{err}")
        if verbose and err.strip():
            print(err)
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


def build_all(verbose: bool = False):
    """libmcv.so and libmcv_probe.so, built concurrently."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(2) as ex:
        a = ex.submit(build, verbose)
        b = ex.submit(build_probe, verbose)
        return a.result(), b.result()


if __name__ == "__main__":
    print(build_all(verbose=True))
