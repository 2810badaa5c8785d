"""Host check of the mixed-precision pair displacement: the FP32 form (32-bit
fixed-point coordinates, their integer difference modulo 2^32 on periodic axes,
converted and scaled) must pick the same periodic image as the FP64 half-open
minimum image and stay within a few FP32 roundings plus three units, on
periodic axes of several lengths and offsets (positions up to two periods
outside the box) and open axes of several extents (positions up to one extent
outside the bounding box, including an axis of zero extent)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="needs hipcc")
def test_fixed_point_displacement(tmp_path):
    exe = str(tmp_path / "mixed_geom_check")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O2",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2005_02656_amd", "csrc"),
                    os.path.join(HERE, "mixed_geom_check.hip"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    rows = [list(map(float, ln.split())) for ln in r.stdout.split("\n") if ln.strip()]
    assert len(rows) == 8, r.stdout + r.stderr
    for case, pairs, wrong, worst in rows:
        assert pairs > 300000
        assert wrong == 0, f"case {case:g}: {wrong:g} pairs outside the bound"
        assert worst <= 1.0
    assert r.returncode == 0
