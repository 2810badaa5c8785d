"""Step graphs (sph_step_graph_*): sph_step captured once as a HIP graph and
replayed.  Every replay must leave exactly the state that the same number of
sph_step calls leaves (the graph holds the same kernels with the same
arguments): checked bit for bit after each replay, with the program's own
eager work and synchronisations between replays, on a lattice (equal masses
and sound speeds, short-reach search) and on random particles with variable h
(unequal records, the full-reach refit), in FP64 and in mixed precision (whose
position records switch their spare lane from mass to volume within a step).
The eager steps themselves are held to the oracle by the parity tests."""
import numpy as np
import pytest
import torch

from paper_2005_02656_amd import inputs, sph
from gpu_support import Run, configs

pytestmark = pytest.mark.gpu

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "h", "u", "rho", "omega", "p", "c", "ax", "ay",
          "az", "du", "c11", "c23", "id")
CASES = {
    "lattice10": lambda: inputs.lattice(10, seed=1, sigma_v=0.01),
    "random": lambda: inputs.random_periodic(3001, seed=4, h_lo=0.06, h_hi=0.09),
}


def _state(r):
    torch.cuda.synchronize()
    out = {k: r.parts[k].cpu().numpy().copy() for k in FIELDS}
    out["g"] = r.g.t.cpu().numpy().copy()
    return out


def _same(a, b, where):
    for k in a:
        assert np.array_equal(a[k], b[k]), (where, k)


@pytest.mark.parametrize("precision", [sph.FP64, sph.MIXED])
@pytest.mark.parametrize("name", sorted(CASES))
def test_graph_replays_match_eager_steps(name, precision):
    w = CASES[name]()
    cfg, _ = configs(w, ng_max=400, precision=precision)
    eager = Run(w, cfg)
    sph.initialise(cfg, eager.parts, eager.ws, eager.g)
    ref = []
    for _ in range(5):
        sph.step(cfg, eager.parts, eager.g, eager.ws)
        assert eager.status() == (0, 0)
        ref.append(_state(eager))
    r = Run(w, cfg)
    sph.initialise(cfg, r.parts, r.ws, r.g)
    one = sph.StepGraph(cfg, r.parts, r.g, r.ws, steps=1)
    two = sph.StepGraph(cfg, r.parts, r.g, r.ws, steps=2)
    scratch = torch.zeros(1 << 16, device="cuda")
    for s in range(3):
        one.launch()
        assert r.status() == (0, 0)
        _same(_state(r), ref[s], f"one-step graph, replay {s}")
        scratch.add_(1.0)   # unrelated eager work between the replays
    two.launch()
    assert r.status() == (0, 0)
    _same(_state(r), ref[4], "two-step graph")
    one.close()
    two.close()
    with pytest.raises(RuntimeError):
        one.launch()
