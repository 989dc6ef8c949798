"""Build step of the HIP library (hipcc, gfx950) into paper_2508_08965_amd/lib/libcgks.so."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "lib", "libcgks.so")
RUNNER = os.path.join(HERE, "lib", "cgks_runner")

SOURCES = ["cgks_capi.hip", "cgks_kernels.hip", "cgks_recon_mfma.hip", "cgks_mlp.hip", "cgks_percell.hip",
           "cgks_consts.cpp"]
# compiled on its own, with the scheduler's register-pressure trackers (see the file's header)
FLUX_SOURCE = "cgks_flux.hip"
FLUX_FLAGS = ["-mllvm", "-amdgpu-use-amdgpu-trackers"]

FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
         # packed FP32 instructions are disabled for every HIP translation unit
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    tmp = OUT + ".tmp"
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    flux_obj = os.path.join(os.path.dirname(OUT), "cgks_flux.o")
    cmd = (["hipcc"] + [f for f in FLAGS if f != "-shared"] + FLUX_FLAGS + inc
           + ["-c", os.path.join(CSRC, FLUX_SOURCE), "-o", flux_obj])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed (flux):\n" + r.stderr)
    cmd = ["hipcc"] + FLAGS + inc + ["-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES] + ["-x", "none", flux_obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stderr)
    if verbose:
        print(r.stderr)
    os.remove(flux_obj)
    os.replace(tmp, OUT)
    # native runner (no PyTorch) used for hardware-counter profiles
    rflags = [f for f in FLAGS if f not in ("-shared", "-fPIC")]
    cmd = (["hipcc"] + rflags + ["-I", os.path.join(ROOT, "include"), "-o", RUNNER + ".tmp",
                                 os.path.join(CSRC, "cgks_runner.cpp"), "-L", os.path.dirname(OUT), "-lcgks",
                                 "-Wl,-rpath,$ORIGIN"])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed (runner):\n" + r.stderr)
    os.replace(RUNNER + ".tmp", RUNNER)
    return OUT


if __name__ == "__main__":
    print(build())
