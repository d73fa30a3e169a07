"""Build step of the HIP library (hipcc, gfx950).

The shared library libmeso.so is built in-tree next to this file from nine
translation units, compiled in parallel.  The FP64 kernels and the host code
are compiled with -ffp-contract=off (every operation rounds separately, so
the FP64 mode follows the arithmetic contract bit for bit); the FP32-bulk,
FP32 and fast-FP64 kernels with -ffp-contract=fast (fused multiply-adds).
The FP64, fast-FP64 and FP32 kernels take the ILP-maximising instruction
scheduler.  No fast-math anywhere, and packed FP32 instructions are disabled
(-packed-fp32-ops).
"""
from __future__ import annotations

import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmeso.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MESO_OFFLOAD_ARCH", "gfx950")

# (source, floating-point contraction, extra flags).  The FP64 kernels (IEEE
# and fast) are latency bound at 2 waves per SIMD; the backend's
# ILP-maximising scheduler runs them 1.5-4 % faster (same instructions,
# reordered).  The FP32-mode kernels
# keep the default scheduler, which holds their registers under the 3- and
# 4-wave occupancy limits.
UNITS = [("meso_kernels.hip", "off", ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]),
         ("meso_kernels_fast.hip", "fast", []),
         ("meso_kernels_fp32.hip", "fast", ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]),
         ("meso_kernels_react.hip", "off", []), ("meso_kernels_react_fast.hip", "fast", []),
         ("meso_kernels_fast64.hip", "fast", ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]),
         ("meso_stream.hip", "off", []),
         ("meso_api.hip", "off", []), ("meso_server.hip", "off", [])]

COMMON = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-fno-fast-math",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False) -> str:
    """Compile every HIP source (in parallel) and link libmeso.so (always
    recompiles)."""
    with tempfile.TemporaryDirectory(prefix="meso_build_") as tmp:
        jobs = []
        for src, contract, extra in UNITS:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            cmd = [HIPCC, *COMMON, f"-ffp-contract={contract}", *extra, "-c", "-o", obj,
                   os.path.join(CSRC, src)]
            if verbose:
                print(" ".join(cmd), flush=True)
            jobs.append((obj, subprocess.Popen(cmd)))
        failed = [obj for obj, p in jobs if p.wait() != 0]
        if failed:
            raise RuntimeError("hipcc failed for " + ", ".join(os.path.basename(f) for f in failed))
        objs = [obj for obj, _ in jobs]
        out = LIB + ".tmp"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
