"""Edge cases and failure detection on the GPU, every condition forced from the
host on CPU-prepared inputs (the kernels flag it in the device error word and
finish normally): a single particle, ragged sizes around the wavefront and
workgroup widths, a list capacity below the true neighbour count, a NaN in the
internal energy, a smoothing length beyond the periodic cell bound, and a
coplanar (zero-extent axis) particle set whose IAD matrix is singular."""
import numpy as np
import pytest

import oracle
from paper_2005_02656_amd import inputs, sph
from gpu_support import Run, configs, rel_err

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _density_stages(cfg, r):
    sph.build_cells(cfg, r.parts, r.ws)
    sph.update_h(cfg, r.parts, r.ws)
    sph.find_neighbors(cfg, r.parts, r.ws)
    sph.density(cfg, r.parts, r.ws)


def test_single_particle():
    """n = 1: no neighbours, Newton has F' = 0 so h goes to kappa h0, rho is the
    self term B_n m / h^3, tau = 0 is flagged singular.  With the self term
    alone Omega = 1 - 3m/(3m) = 0, so P/(Omega rho^2) is infinite and du = inf*0
    is NaN (the oracle gives the same): flagged non-finite."""
    w = inputs.random_periodic(1, seed=2, h_lo=0.1, h_hi=0.1)
    cfg, ocfg = configs(w, ng_max=16)
    r = Run(w, cfg)
    sph.step(cfg, r.parts, r.g, r.ws)
    st, bits = r.status()
    assert bits == sph.ERRBIT_SINGULAR_TAU | sph.ERRBIT_NONFINITE, bits
    a = w.arrays
    h_o = oracle.update_h(ocfg, a["x"], a["y"], a["z"], a["h"])
    assert abs(r.by_id("h")[0] - h_o[0]) <= TOL * h_o[0]
    assert abs(r.by_id("h")[0] - cfg.h_ratio_max * a["h"][0]) <= TOL * h_o[0]
    rho_o = oracle.density(ocfg, a["x"], a["y"], a["z"], h_o, a["m"], a["u"])[0]
    assert abs(r.by_id("rho")[0] - rho_o[0]) <= TOL * rho_o[0]
    assert r.by_id("omega")[0] == 0.0
    assert r.by_id("ax")[0] == 0.0 and np.isnan(r.by_id("du")[0])


@pytest.mark.parametrize("n", [2, 63, 64, 65, 255, 257, 1000])
def test_ragged_sizes_density(n):
    """Sizes around the 64-lane wavefront and 256-thread workgroup: neighbour
    counts bit-exact and density within 1e-12 of the oracle."""
    # about 60 neighbours, and kappa h stays below a quarter of the box
    h = min(0.18, (60.0 / (33.5 * n)) ** (1.0 / 3.0))
    w = inputs.random_periodic(n, seed=n, h_lo=0.9 * h, h_hi=h)
    cfg, ocfg = configs(w, ng_max=1024)
    r = Run(w, cfg)
    _density_stages(cfg, r)
    assert r.status() == (0, 0)
    a = w.arrays
    h_o = oracle.update_h(ocfg, a["x"], a["y"], a["z"], a["h"])
    assert rel_err(r.by_id("h"), h_o) < TOL
    nc_o, ns_o, _, _ = oracle.neighbors(ocfg, a["x"], a["y"], a["z"], h_o, with_lists=False)
    _, nc, ns = r.neighbor_pairs()
    assert np.array_equal(nc, nc_o) and np.array_equal(ns, ns_o)
    rho_o = oracle.density(ocfg, a["x"], a["y"], a["z"], h_o, a["m"], a["u"])[0]
    assert rel_err(r.by_id("rho"), rho_o) < TOL


def test_neighbor_overflow_flag():
    """ng_max below the true count: the overflow bit is set, the counts stay the
    true counts (oracle), and the step's later passes run on the truncated lists."""
    w = inputs.lattice(8, seed=4, sigma_v=0.01)
    cfg, ocfg = configs(w, ng_max=24)
    r = Run(w, cfg)
    sph.step(cfg, r.parts, r.g, r.ws)
    st, bits = r.status()
    assert bits & sph.ERRBIT_NEIGHBOR_OVERFLOW, bits
    a = w.arrays
    # the stage path reports the true counts of the step's sets
    r2 = Run(w, cfg)
    _density_stages(cfg, r2)
    r2.status()
    h_o = oracle.update_h(ocfg, a["x"], a["y"], a["z"], a["h"])
    nc_o, ns_o, _, _ = oracle.neighbors(ocfg, a["x"], a["y"], a["z"], h_o, with_lists=False)
    nc, ns, _ = sph.neighbors_view(cfg, r2.ws)
    ids = r2.ids()
    assert np.array_equal(nc.cpu().numpy(), nc_o[ids]) and np.array_equal(ns.cpu().numpy(),
                                                                          ns_o[ids])
    assert nc_o.max() > cfg.ng_max


def test_nonfinite_flag():
    """A NaN internal energy makes P and c of that particle non-finite."""
    w = inputs.lattice(8, seed=5, sigma_v=0.01)
    a = dict(w.arrays)
    a["u"] = a["u"].copy()
    a["u"][17] = np.nan
    cfg, _ = configs(w, ng_max=400)
    r = Run(w, cfg, a)
    _density_stages(cfg, r)
    st, bits = r.status()
    assert bits & sph.ERRBIT_NONFINITE, bits
    assert st == 6
    rho = r.by_id("rho")
    assert np.all(np.isfinite(rho))
    p = r.by_id("p")
    assert np.isnan(p[17]) and np.sum(~np.isfinite(p)) == 1


def test_cell_range_flag():
    """4h beyond the periodic box length (64 particles, 100 target neighbours)."""
    w = inputs.lattice(4, seed=6, sigma_v=0.01)
    cfg, _ = configs(w, ng_max=400)
    r = Run(w, cfg)
    _density_stages(cfg, r)
    st, bits = r.status()
    assert bits & sph.ERRBIT_CELL_RANGE, bits


def test_coplanar_singular_tau():
    """Particles on one plane (a zero-extent open axis): cells, search and density
    still match the oracle; tau has no z-z component and is flagged singular,
    C = 0 (the reading for a singular matrix)."""
    n_side = 12
    g = (np.arange(n_side) + 0.5) / n_side
    X, Y = np.meshgrid(g, g, indexing="ij")
    n = n_side * n_side
    rng = np.random.default_rng(7)
    a = dict(x=X.ravel().copy(), y=Y.ravel().copy(), z=np.full(n, 0.25),
             vx=rng.normal(0, 0.01, n), vy=rng.normal(0, 0.01, n), vz=np.zeros(n),
             m=np.full(n, 1.0 / n), u=np.ones(n), h=np.full(n, 1.5 / n_side),
             id=np.arange(n, dtype=np.int64))
    params = inputs.base_params(periodic=(1, 1, 0), n_target=20.0)
    w = inputs.Workload("plane", a, params)
    cfg, ocfg = configs(w, ng_max=200)
    r = Run(w, cfg)
    _density_stages(cfg, r)
    assert r.status() == (0, 0)
    h_o = oracle.update_h(ocfg, a["x"], a["y"], a["z"], a["h"])
    assert rel_err(r.by_id("h"), h_o) < TOL
    rho_o = oracle.density(ocfg, a["x"], a["y"], a["z"], h_o, a["m"], a["u"])[0]
    assert rel_err(r.by_id("rho"), rho_o) < TOL
    sph.iad(cfg, r.parts, r.ws)
    st, bits = r.status()
    assert bits & sph.ERRBIT_SINGULAR_TAU, bits
    for k in ("c11", "c12", "c13", "c22", "c23", "c33"):
        assert np.all(r.by_id(k) == 0.0), k
    # the fused step on the flat axis: same h, the singular flag only
    r3 = Run(w, cfg)
    sph.step(cfg, r3.parts, r3.g, r3.ws)
    st, bits = r3.status()
    assert bits == sph.ERRBIT_SINGULAR_TAU, bits
    assert rel_err(r3.by_id("h"), h_o) < TOL
