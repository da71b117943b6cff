"""The stage kernels' wave-to-tile map (one or two band heights, four tile
orders) covers every cell of a domain exactly once: a host build of the
map's own functions from the device header, checked over ~75,000 shapes
(no GPU needed)."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1912_02457_amd", "csrc")
ROCM_INCLUDE = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INCLUDE),
                    reason="needs g++ and the HIP headers")
def test_tile_map_covers_every_cell_once(tmp_path):
    exe = str(tmp_path / "tiling_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM_INCLUDE}", f"-I{CSRC}",
                    os.path.join(HERE, "tiling_check.cpp"), "-o", exe], check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "bad 0" in r.stdout
