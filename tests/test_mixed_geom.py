"""Host check of the mixed-precision pair displacement: the FP32 form (cell
difference x edge + offset difference, minimum image on cell indices) must pick
the same periodic image as the FP64 half-open minimum image, including at a cell
difference of exactly half the axis, on axes of 4 to 1024 cells."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="needs hipcc")
def test_axis_disp_minimum_image(tmp_path):
    exe = str(tmp_path / "mixed_geom_check")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O2",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2005_02656_amd", "csrc"),
                    os.path.join(HERE, "mixed_geom_check.hip"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe, "4", "8", "16", "64", "512", "1024"], capture_output=True, text=True)
    rows = [list(map(float, ln.split())) for ln in r.stdout.split("\n") if ln.strip()]
    assert len(rows) == 6, r.stdout + r.stderr
    for nax, pairs, wrong, worst in rows:
        assert pairs > 300000
        assert wrong == 0, f"nax={nax:g}: {wrong:g} pairs took the wrong image"
        assert worst < 5e-7
    assert r.returncode == 0
