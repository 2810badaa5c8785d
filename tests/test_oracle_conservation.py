"""Pins of the oracle's momentum/energy/AV pass (eqs. 2-5 with the readings in the
design notes) by exact identities and symmetries that hold for ANY input:

* pairwise antisymmetry -> total momentum rate sum_a m_a a_a = 0
* the energy identity sum_a m_a (v_a . a_a + du_a) = 0 (fails with the literal
  "+a^AV" sign of eq. 2 and with the garbled rho_a of eq. 3)
* the artificial viscosity only dissipates kinetic energy
* Galilean, translation, rotation/reflection and permutation invariance
* a uniform lattice at rest has a = 0 and du = 0
"""
import numpy as np
import pytest

from paper_2005_02656_amd import inputs
from conftest import oracle_config


def full_rates(ora, cfg, a, h=None):
    h = a["h"] if h is None else h
    x, y, z = a["x"], a["y"], a["z"]
    rho, om, p, c = ora.density(cfg, x, y, z, h, a["m"], a["u"])
    Cm, sing = ora.iad(cfg, x, y, z, h, a["m"], rho)
    assert not sing
    me = ora.momentum_energy(cfg, x, y, z, a["vx"], a["vy"], a["vz"], h, a["m"], rho, om, p, c, Cm)
    return me, (rho, om, p, c, Cm)


@pytest.fixture(scope="module")
def rnd(ora):
    w = inputs.random_periodic(1000, seed=11, h_lo=0.10, h_hi=0.14)
    cfg = oracle_config(w.params)
    me, f = full_rates(ora, cfg, w.arrays)
    return cfg, w.arrays, me, f


def test_momentum_conserved(rnd):
    cfg, a, me, _ = rnd
    for k in ("ax", "ay", "az"):
        tot = (a["m"] * me[k]).sum()
        scale = (a["m"] * me["scale_a"]).sum()
        assert abs(tot) < 1e-14 * scale, (k, tot, scale)


def test_energy_identity(rnd):
    cfg, a, me, _ = rnd
    rate = (a["m"] * (a["vx"] * me["ax"] + a["vy"] * me["ay"] + a["vz"] * me["az"] + me["du"])).sum()
    scale = (a["m"] * (np.abs(a["vx"] * me["ax"]) + np.abs(a["vy"] * me["ay"])
                       + np.abs(a["vz"] * me["az"]) + np.abs(me["du"]))).sum()
    assert abs(rate) < 1e-14 * scale


def test_av_is_dissipative(ora, rnd):
    cfg, a, me1, _ = rnd
    me0, _ = full_rates(ora, cfg.replace(alpha_av=0.0), a)
    dke = (a["m"] * (a["vx"] * (me1["ax"] - me0["ax"]) + a["vy"] * (me1["ay"] - me0["ay"])
                     + a["vz"] * (me1["az"] - me0["az"]))).sum()
    heat = (a["m"] * (me1["du"] - me0["du"])).sum()
    assert dke < 0.0
    # what the AV takes from the kinetic energy it returns as heat
    assert abs(dke + heat) < 1e-13 * abs(dke)


def test_galilean_invariance(ora, rnd):
    cfg, a, me, _ = rnd
    b = dict(a)
    V = np.array([0.7, -1.3, 0.4])
    b["vx"], b["vy"], b["vz"] = a["vx"] + V[0], a["vy"] + V[1], a["vz"] + V[2]
    me2, _ = full_rates(ora, cfg, b)
    for k, s in (("ax", "scale_a"), ("ay", "scale_a"), ("az", "scale_a"), ("du", "scale_du")):
        assert np.max(np.abs(me2[k] - me[k])) < 1e-12 * np.max(me[s])


def test_translation_invariance(ora, rnd):
    cfg, a, me, _ = rnd
    b = dict(a)
    for k, s in zip("xyz", (0.31, 0.77, 0.05)):
        b[k] = np.mod(a[k] + s, 1.0)
    me2, _ = full_rates(ora, cfg, b)
    for k, s in (("ax", "scale_a"), ("ay", "scale_a"), ("az", "scale_a"), ("du", "scale_du")):
        assert np.max(np.abs(me2[k] - me[k])) < 1e-11 * np.max(me[s])


def test_rotation_and_axis_permutation(ora, rnd):
    """A 90-degree rotation about z and a cyclic relabelling of the axes are symmetries
    of the periodic cube; accelerations must transform as vectors (catches
    transposed or mislabelled tensor components in C and A_ab)."""
    cfg, a, me, _ = rnd
    b = dict(a)
    # rotation: (x, y) -> (-y, x), velocities likewise
    b["x"], b["y"] = np.mod(-a["y"], 1.0), a["x"].copy()
    b["vx"], b["vy"] = -a["vy"], a["vx"].copy()
    me2, _ = full_rates(ora, cfg, b)
    sc = np.max(me["scale_a"])
    assert np.max(np.abs(me2["ax"] + me["ay"])) < 1e-11 * sc
    assert np.max(np.abs(me2["ay"] - me["ax"])) < 1e-11 * sc
    assert np.max(np.abs(me2["az"] - me["az"])) < 1e-11 * sc
    assert np.max(np.abs(me2["du"] - me["du"])) < 1e-11 * np.max(me["scale_du"])
    # cyclic permutation (x, y, z) -> (y, z, x)
    c = dict(a)
    c["x"], c["y"], c["z"] = a["y"], a["z"], a["x"]
    c["vx"], c["vy"], c["vz"] = a["vy"], a["vz"], a["vx"]
    me3, _ = full_rates(ora, cfg, c)
    assert np.max(np.abs(me3["ax"] - me["ay"])) < 1e-11 * sc
    assert np.max(np.abs(me3["ay"] - me["az"])) < 1e-11 * sc
    assert np.max(np.abs(me3["az"] - me["ax"])) < 1e-11 * sc


def test_permutation_invariance(ora, rnd):
    cfg, a, me, _ = rnd
    perm = np.random.default_rng(5).permutation(a["x"].size)
    b = {k: v[perm] for k, v in a.items()}
    me2, _ = full_rates(ora, cfg, b)
    for k, s in (("ax", "scale_a"), ("du", "scale_du")):
        assert np.max(np.abs(me2[k] - me[k][perm])) < 1e-13 * np.max(me[s])


def test_lattice_at_rest(ora):
    w = inputs.lattice(10, sigma_v=0.0)
    cfg = oracle_config(w.params)
    a = w.arrays
    h = ora.initial_h(cfg, a)
    me, _ = full_rates(ora, cfg, a, h)
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(me[k])) < 1e-13 * np.max(me["scale_a"])
    assert np.max(np.abs(me["du"])) == 0.0


def test_weakly_compressible_eos(ora):
    w = inputs.square_patch(8)
    cfg = oracle_config(w.params)
    a = w.arrays
    rho_ref = np.full(a["x"].size, 0.9)
    rho, om, p, c = ora.density(cfg, a["x"], a["y"], a["z"], a["h"], a["m"], a["u"],
                                a["p_ref"], rho_ref)
    assert np.allclose(p, a["p_ref"] + cfg.c0 ** 2 * (rho - rho_ref), rtol=0, atol=1e-12)
    assert np.all(c == cfg.c0)
