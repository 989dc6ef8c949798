"""The flux work figures used by bench.py's roofline equal the source-level operation count of
the flux (paper_2508_08965_amd/csrc/flux_opcount.cpp, a host build of the same template): the
method's work per Gauss point (work both lanes of a pair repeat counted once) and, for context,
what the lane pairs issue."""
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
    assert int(out[6]) == 0
    assert int(out[8]) == bench.FLUX_FLOP_PER_GP
    assert int(out[9]) == bench.FLUX_FLOP_PER_GP_DERIV  # second stage: time derivatives only
    assert int(out[0]) == bench.FLUX_ISSUED_PER_GP
    assert int(out[7]) == bench.FLUX_ISSUED_PER_GP_DERIV
    # the shared work is counted once, never dropped: between one lane's and both lanes' count
    assert int(out[0]) // 2 < int(out[8]) < int(out[0])
