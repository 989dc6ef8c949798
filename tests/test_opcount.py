"""The flux work figure used by bench.py's roofline equals the source-level operation count of
the flux (paper_2508_08965_amd/csrc/flux_opcount.cpp, a host build of the same template)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_flux_flops_per_gauss_point_matches_bench(tmp_path):
    exe = str(tmp_path / "flux_opcount")
    src = os.path.join(ROOT, "paper_2508_08965_amd", "csrc", "flux_opcount.cpp")
    r = subprocess.run(["hipcc", "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2508_08965_amd", "csrc"),
                        "-o", exe, src], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr)
    out = subprocess.run([exe, "1", "1", "1", "0"], capture_output=True, text=True, check=True).stdout.split()
    import bench
    assert int(out[0]) == bench.FLUX_FLOP_PER_GP
    assert int(out[7]) == bench.FLUX_FLOP_PER_GP_DERIV  # second stage: time derivatives only
