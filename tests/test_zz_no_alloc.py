"""sph_step_static (the allocation-free step, scratch in the library's fixed
device array) against sph_step with a caller workspace, through the C ABI: two
calls in a row, the second with a smaller input, in FP64 and in mixed
precision, then a call whose lists overflow (error word set) and one after it
(word cleared again)."""
import numpy as np
import pytest
import torch

from paper_2005_02656_amd import inputs, sph
from gpu_support import Run, configs

pytestmark = pytest.mark.gpu

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "vhx", "vhy", "vhz", "h", "u", "du_m1", "id", "rho",
          "omega", "p", "c", "c11", "c12", "c13", "c22", "c23", "c33", "ax", "ay", "az", "du")


def _pair(w, **kw):
    """The same initialised state twice: one for sph_step, one for the static step."""
    cfg, _ = configs(w, **kw)
    a = Run(w, cfg)
    sph.initialise(cfg, a.parts, a.ws, a.g)
    b = sph.Particles({k: v.clone() for k, v in a.parts.t.items()})
    gb = sph.Globals()
    gb.t.copy_(a.g.t)
    return cfg, a, b, gb


def _compare(cfg, a, b, gb, err):
    sph.step(cfg, a.parts, a.g, a.ws)
    sph.step_static(cfg, b, gb, err)
    torch.cuda.synchronize()
    st, bits = sph.status_sync(a.ws)
    assert int(err.item()) == bits
    for k in FIELDS:
        x, y = a.parts[k], b[k]
        if x.dtype == torch.float64:
            # the same kernels on the same inputs: identical to the last bit
            assert torch.equal(x.view(torch.int64), y.view(torch.int64)), k
        else:
            assert torch.equal(x, y), k
    assert torch.equal(a.g.t.view(torch.int64), gb.t.view(torch.int64))
    return st, bits


@pytest.mark.parametrize("precision", [sph.FP64, sph.MIXED])
def test_static_step_matches_workspace_step(precision):
    err = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    # a 20^3 lattice (8,000 particles), then a smaller random set (3,001)
    for w in (inputs.c1_lattice(), inputs.random_periodic(3001, seed=4, h_lo=0.06, h_hi=0.09)):
        cfg, a, b, gb = _pair(w, ng_max=400, precision=precision)
        assert sph.lib().sph_workspace_bytes(__import__("ctypes").byref(cfg.c())) \
            <= sph.STATIC_SCRATCH_BYTES
        for _ in range(2):
            st, bits = _compare(cfg, a, b, gb, err)
            assert (st, bits) == (0, 0)
    # lists that overflow set the word in both; the next call starts from zero
    w = inputs.lattice(12, seed=1, sigma_v=0.01)
    cfg, a, b, gb = _pair(w, ng_max=40)
    st, bits = _compare(cfg, a, b, gb, err)
    assert bits & sph.ERRBIT_NEIGHBOR_OVERFLOW
    w = inputs.lattice(10, seed=1, sigma_v=0.01)
    cfg, a, b, gb = _pair(w, ng_max=160)
    assert _compare(cfg, a, b, gb, err) == (0, 0)


def test_static_step_rejects_oversized_config():
    w = inputs.lattice(32, seed=1, sigma_v=0.01)       # 32,768 particles: 79 MiB
    cfg, _ = configs(w)
    parts = sph.Particles.from_arrays(w.arrays, cfg)
    with pytest.raises(sph.SphError) as e:
        sph.step_static(cfg, parts, sph.Globals())
    assert e.value.status == 3
