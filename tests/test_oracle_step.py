"""Pins of the composed oracle step and of the square-patch initial conditions."""
import json
import os

import numpy as np
import pytest

from conftest import oracle_config
from paper_2005_02656_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_square_patch_pressure_solves_poisson():
    """eq. (8) with the reading (odd m, n; sin(n pi y / L)): P = 0 on the edge of the
    square and laplacian P = 2 rho omega^2 inside (incompressible rigid rotation)."""
    om = GOLD["square_patch_omega"]["value"]
    e = 1e-3
    pts = np.array([-0.3, -0.1, 0.0, 0.2, 0.35])
    xs = np.concatenate([pts - e, pts, pts + e])
    P = inputs.square_patch_pressure(xs, xs, omega=om)
    k = len(pts)
    c = P[k:2 * k, k:2 * k]
    lap = (P[:k, k:2 * k] + P[2 * k:, k:2 * k] + P[k:2 * k, :k] + P[k:2 * k, 2 * k:] - 4 * c) / e ** 2
    # the truncated sine series of a constant converges like 1/M pointwise
    assert np.allclose(lap, 2 * om ** 2, rtol=1e-2)
    edge = inputs.square_patch_pressure(np.array([-0.5, 0.5]), pts, omega=om)
    assert np.max(np.abs(edge)) < 1e-12
    centre = inputs.square_patch_pressure(np.array([0.0]), np.array([0.0]), omega=om)[0, 0]
    assert abs(centre + 3.6835676) < 2e-6


def test_square_patch_ic():
    w = inputs.square_patch(10)
    a = w.arrays
    om = GOLD["square_patch_omega"]["value"]
    assert np.allclose(a["vx"], om * a["y"]) and np.allclose(a["vy"], -om * a["x"])
    assert w.params["periodic"] == (0, 0, 1)
    # L_z(0) = -omega sum m (x^2 + y^2), which tends to -omega/6 for the unit square
    lz = (a["m"] * (a["x"] * a["vy"] - a["y"] * a["vx"])).sum()
    assert abs(lz - (-om * (a["m"] * (a["x"] ** 2 + a["y"] ** 2)).sum())) < 1e-14
    assert abs(lz + om / 6) < 0.01


def test_step_at_rest_stays_at_rest(ora):
    w = inputs.lattice(8, sigma_v=0.0)
    cfg = oracle_config(w.params)
    st = dict(w.arrays)
    st["h"] = ora.initial_h(cfg, st)
    st.update(vhx=st["vx"].copy(), vhy=st["vy"].copy(), vhz=st["vz"].copy(),
              du_m1=np.zeros(st["x"].size))
    new, g, f = ora.step(cfg, st, {"dt_m1": 0.0, "t": 0.0})
    assert np.max(np.abs(new["x"] - st["x"])) < 1e-15
    assert g["dt"] == pytest.approx(0.2 * np.min(f["h"] / f["c"]), rel=1e-15)


def _started(ora, w):
    cfg = oracle_config(w.params)
    st = dict(w.arrays)
    st["h"] = ora.initial_h(cfg, st)
    st.update(vhx=st["vx"].copy(), vhy=st["vy"].copy(), vhz=st["vz"].copy(),
              du_m1=np.zeros(st["x"].size))
    return cfg, st


def test_multistep_momentum_conservation(ora):
    """Random particles: violent, but the total momentum is conserved to roundoff by
    the pairwise antisymmetry whatever the step does."""
    cfg, st = _started(ora, inputs.random_periodic(250, seed=21, h_lo=0.11, h_hi=0.15,
                                                   sigma_v=0.2))
    gl = {"dt_m1": 0.0, "t": 0.0}
    s0 = ora.sums(st["m"], st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["u"])
    for _ in range(4):
        st, gl, f = ora.step(cfg, st, gl)
        assert np.max(np.abs(gl["mom"] - s0["mom"])) < 1e-14
        assert gl["mass"] == pytest.approx(s0["mass"], rel=1e-15)
    assert np.all((st["x"] >= 0) & (st["x"] < 1))


def test_multistep_energy_drift_lattice(ora):
    """A gently perturbed lattice: the second-order scheme keeps the total energy to
    a small drift (1e-4 relative bound over six steps)."""
    cfg, st = _started(ora, inputs.lattice(10, sigma_v=0.05))
    gl = {"dt_m1": 0.0, "t": 0.0}
    s0 = ora.sums(st["m"], st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["u"])
    e0 = s0["e_kin"] + s0["e_int"]
    for _ in range(6):
        st, gl, f = ora.step(cfg, st, gl)
    assert abs(gl["e_kin"] + gl["e_int"] - e0) < 1e-3 * e0
    assert gl["dt_m1"] == gl["dt"] and gl["t"] > 0
