"""Build ``librx.so`` (the C-ABI receive library) for gfx950 with hipcc, in-tree.

Usage: ``python -m paper_1901_07499_amd.build`` (or ``build()`` from Python).
The library is written next to this file; the Python binding loads it from
there.  Every call recompiles.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librx.so")

ARCH = "gfx950"
# Packed FP32 instructions are kept out of generated code on purpose.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "include")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build librx.so)")


def build(verbose: bool = False, save_temps: str | None = None) -> str:
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="rxbuild_") as tmp:
        objs = []
        api_o = os.path.join(tmp, "rx_api.o")
        cmd = [cc, *COMMON, f"--offload-arch={ARCH}", "-c", os.path.join(CSRC, "rx_api.cpp"), "-o", api_o]
        _run(cmd, verbose)
        objs.append(api_o)
        for name in ("rx_batch", "rx_dn_api", "rx_sync_api"):
            o = os.path.join(tmp, name + ".o")
            _run([cc, *COMMON, f"--offload-arch={ARCH}", "-c", os.path.join(CSRC, name + ".cpp"), "-o", o], verbose)
            objs.append(o)
        for name in ("rx_denoise", "rx_sync", "rx_mfma_fft", "rx_noalloc"):
            o = os.path.join(tmp, name + ".o")
            _run([cc, *COMMON, f"--offload-arch={ARCH}", *DEVICE_FLAGS, "-x", "hip", "-c",
                  os.path.join(CSRC, name + ".hip"), "-o", o], verbose)
            objs.append(o)
        k_o = os.path.join(tmp, "rx_kernels.o")
        cmd = [cc, *COMMON, f"--offload-arch={ARCH}", *DEVICE_FLAGS, "-x", "hip", "-c",
               os.path.join(CSRC, "rx_kernels.hip"), "-o", k_o]
        if save_temps:
            os.makedirs(save_temps, exist_ok=True)
            cmd += ["-save-temps=obj", "-Rpass-analysis=kernel-resource-usage"]
            k_o_saved = os.path.join(save_temps, "rx_kernels.o")
            cmd[-1] = k_o_saved
            k_o = k_o_saved
        _run(cmd, verbose)
        objs.append(k_o)
        tmp_lib = os.path.join(tmp, "librx.so")
        _run([cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp_lib], verbose)
        shutil.copyfile(tmp_lib, LIB + ".tmp")
        os.replace(LIB + ".tmp", LIB)
    return LIB


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd)}")
    if verbose and (r.stdout or r.stderr):
        sys.stderr.write(r.stdout + r.stderr)


if __name__ == "__main__":
    print(build(verbose=True))
