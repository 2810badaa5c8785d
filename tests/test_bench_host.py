"""Host logic of bench.py (no GPU): the one-GPU contract, the algorithmic byte
and flop model, the choice of the binding roofline, and the committed counter
summary it reads the measured traffic from."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2005_02656_amd import profiling  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_byte_model_per_phase():
    """The algorithmic model of the step: 1,020 + 16 k_s bytes per particle
    under the weakly compressible EOS and 972 + 16 k_s with the ideal gas, split
    over the phases as the kernels of the method read and write them."""
    k_g, k_s, k_c = 91.7, 91.8, 121.5
    for wc, base in ((True, 1020), (False, 972)):
        tot = sum(bench.bytes_per_particle(ph, k_g, k_s, wc, k_c, 2)
                  for ph in bench.PHASE_KERNEL)
        assert tot == pytest.approx(base + 16 * k_s)
        unfused = sum(bench.bytes_per_particle(ph, k_g, k_s, wc, k_c, 2, fused=False)
                      for ph in bench.PHASE_KERNEL)
        assert unfused == pytest.approx(tot)
    bpp = lambda ph, **kw: bench.bytes_per_particle(ph, k_g, k_s, True, k_c, 2, **kw)
    # momentum: 12 FP64 fields and 6 C in, 4 out, the list read once
    assert bpp("momentum_energy") == pytest.approx(176 + 4 * k_s)
    # the implementation's record layout does not change what the method moves
    assert bpp("momentum_energy", urec=True) == bpp("momentum_energy")
    # Newton: x y z h per iteration and h out
    assert bpp("newton_h") == pytest.approx(72)
    # with the fused step the density is formed in the list filter
    assert bpp("density") == 0
    assert bpp("density", fused=False) == pytest.approx(96 + 4 * k_s)


def test_roofline_reports_the_binding_ceiling():
    n, k_g, k_s, k_c = 64_000_000, 91.7, 91.8, 121.5
    phases = {"build_cells": 17.0, "candidates": 53.0, "newton_h": 35.0, "lists": 36.0,
              "density": 0.0, "iad": 20.0, "momentum_energy": 69.0, "integrate": 2.5}
    r = bench.roofline(phases, n, k_g, k_s, True, 2, k_c, "no-such-workload", True)
    assert r["phase"] == "momentum_energy" and r["kernel"] == "k_momentum_energy"
    fl = bench.FLOPS_PER_PAIR["momentum_energy"] * k_s * n / 69e-3 / 1e12
    by = bench.bytes_per_particle("momentum_energy", k_g, k_s, True, k_c, 2) * n / 69e-3 / 1e9
    # the larger of the two fractions is the one reported, the other is `alt`
    assert r["bound"] == "alu" and r["achieved"] == pytest.approx(fl)
    assert r["frac"] == pytest.approx(fl / bench.FP64_VALU_PEAK_TFLOPS)
    assert r["alt"]["achieved"] == pytest.approx(by)
    assert r["frac"] >= r["alt"]["frac"]
    assert r["traffic"] is None                        # no summary for that workload
    # a phase without a flop model is priced against HBM alone
    r2 = bench.roofline({"build_cells": 50.0, "integrate": 1.0}, n, k_g, k_s, True, 2, k_c,
                        "c4", True)
    assert r2["bound"] == "hbm" and "alt" not in r2
    # the candidate walk has no algorithmic count: a longer walk is passed over
    r4 = bench.roofline({**phases, "candidates": 100.0}, n, k_g, k_s, True, 2, k_c,
                        "no-such-workload", True)
    assert r4["phase"] == "momentum_energy"
    # with equal masses and sound speeds the same kernel reads 112-byte records
    r3 = bench.roofline(phases, n, k_g, k_s, True, 2, k_c, "c4", True, urec=True)
    assert r3["kernel"] == "k_momentum_energy"
    assert r3["algorithmic_bytes"] == pytest.approx(
        bench.bytes_per_particle("momentum_energy", k_g, k_s, True, k_c, 2, True, True) * n)


def test_traffic_comes_from_a_summary_of_the_current_sources(tmp_path):
    # C4 has equal masses under the weakly compressible EOS: 112-byte records
    s = profiling.read_summary(os.path.join(ROOT, "profiles", "k_momentum_energy_c4.md"))
    assert s, "no committed summary for the C4 momentum kernel"
    t = bench.traffic_from_profile("k_momentum_energy", "c4")
    if s.get("source_digest") == profiling.source_digest():
        assert t == pytest.approx(float(s["fetch_bytes_per_launch"])
                                  + float(s["write_bytes_per_launch"]))
    else:
        assert t is None
    assert bench.traffic_from_profile("k_momentum_energy", "no-such-workload") is None
