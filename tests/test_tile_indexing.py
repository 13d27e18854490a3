"""Host-side bounds check of every LDS and workspace index the tile march
and the staged streaming kernels form, for tile edges 4, 8 and 16 and both
candidate-flag layouts (tests/tile_index_check.cpp, built with the kernels'
own index header).  CPU only: it runs no kernel."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_tile_indices_in_bounds(tmp_path):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / "tile_index_check"
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O1",
                    "-I", os.path.join(ROOT, "paper_1502_07303_amd", "csrc"),
                    os.path.join(ROOT, "tests", "tile_index_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
