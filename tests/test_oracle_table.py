"""Pins of the oracle's kernel lookup table (section 4.5: N precomputed kernel
values, linear interpolation in the relative distance v = r/h).  Linear
interpolation between exact node values is exact at the nodes, errs by
-(dv^2/8) S''(v) at the midpoints to leading order, and is bounded everywhere
by (dv^2/8) max|S''|; the bound shrinks as 1/N^2.  These are facts of the
interpolation itself, not of the oracle's code."""
import math

import numpy as np
import pytest

from paper_2005_02656_amd import inputs
from conftest import oracle_config

N_PAPER = 20000


def _cfg(N, n=6.0):
    import oracle
    return oracle.Config(sinc_n=n, kernel_table=N)


def _second_derivative_max(ora, fn, n=6.0, m=4001, h=1e-3):
    """max |f''| of f = S or dS/dv on [0, 2] by central differences of the exact
    function (S is even in v, so f(-v) = +-f(v) extends it past 0)."""
    vs = np.linspace(0.0, 2.0, m)
    best = 0.0
    for v in vs:
        a = max(v, h)   # the extension is smooth at 0; differences taken at v >= h
        b = min(a, 2.0 - h)
        d2 = (fn(b + h, n) - 2 * fn(b, n) + fn(b - h, n)) / (h * h)
        best = max(best, abs(d2))
    return best


def test_exact_at_the_nodes(ora):
    cfg = _cfg(N_PAPER)
    rng = np.random.default_rng(3)
    for i in rng.integers(0, N_PAPER - 1, 50):
        # v (N-1)/2 lands on i or one ulp below it, where f is 1 to rounding
        v = 2.0 * i / (N_PAPER - 1)
        assert ora.S_cfg(cfg, v) == pytest.approx(ora.S(v, 6.0), rel=0, abs=1e-15)
        assert ora.dSdv_cfg(cfg, v) == pytest.approx(ora.dSdv(v, 6.0), rel=0, abs=1e-14)
    assert ora.S_cfg(cfg, 0.0) == 1.0
    assert abs(ora.S_cfg(cfg, 2.0)) < 1e-30


def test_midpoint_error_is_the_interpolation_term(ora):
    """At a midpoint the chord exceeds the function by (dv^2/8) S''(v) + O(dv^4)."""
    N = 2000          # coarse enough that the leading term dominates rounding
    cfg = _cfg(N)
    dv = 2.0 / (N - 1)
    h = 1e-3
    for i in (0, 37, 400, 999, 1500, 1990):
        v = (i + 0.5) * dv
        err = ora.S_cfg(cfg, v) - ora.S(v, 6.0)
        vm = max(v, h)
        d2 = (ora.S(vm + h, 6.0) - 2 * ora.S(vm, 6.0) + ora.S(vm - h, 6.0)) / (h * h)
        pred = dv * dv / 8.0 * d2
        assert abs(err - pred) <= 2e-3 * dv * dv / 8.0 * 5.0 + 1e-15, (i, err, pred)


@pytest.mark.parametrize("deriv", [False, True])
def test_error_bound_and_its_order(ora, deriv):
    """max |error| over 20,000 random v stays below (dv^2/8) max|f''| and comes
    within a factor 2 of it; halving dv quarters it."""
    exact = ora.dSdv if deriv else ora.S
    table = ora.dSdv_cfg if deriv else ora.S_cfg
    f2max = _second_derivative_max(ora, exact, m=801)
    rng = np.random.default_rng(11 + deriv)
    vs = rng.uniform(0.0, 2.0, 20000)
    worst = {}
    for N in (N_PAPER // 2, N_PAPER):
        cfg = _cfg(N)
        dv = 2.0 / (N - 1)
        bound = dv * dv / 8.0 * f2max
        e = max(abs(table(cfg, v) - exact(v, 6.0)) for v in vs)
        assert e <= bound * (1 + 1e-3), (N, e, bound)
        assert e >= 0.5 * bound, (N, e, bound)
        worst[N] = e
    ratio = worst[N_PAPER // 2] / worst[N_PAPER]
    assert 3.5 < ratio < 4.5, ratio


def test_stated_bound_of_the_paper_table(ora):
    """The bound stated for N = 20,000 and n = 6: dv = 2/19999,
    (dv^2/8) max|S''| with max|S''| = |S''(0)| = n pi^2/12 (the curvature of
    sinc^n at 0)."""
    f2 = _second_derivative_max(ora, ora.S, m=801)
    assert f2 == pytest.approx(6.0 * math.pi ** 2 / 12.0, rel=1e-4)
    dv = 2.0 / (N_PAPER - 1)
    assert dv * dv / 8.0 * f2 == pytest.approx(6.17e-9, rel=1e-2)


def test_table_density_on_the_lattice(ora):
    """The table changes rho of the lattice by no more than the interpolation
    bound times the kernel sum with S replaced by 1, and does change it (the table
    is used); Omega and the Newton h move by a few times the bound."""
    w = inputs.lattice(10, seed=1, sigma_v=0.0)
    a = w.arrays
    direct = oracle_config(w.params)
    tab = direct.replace(kernel_table=N_PAPER)
    h = ora.initial_h(direct, a)
    r0, o0, _, _ = ora.density(direct, a["x"], a["y"], a["z"], h, a["m"], a["u"])
    r1, o1, _, _ = ora.density(tab, a["x"], a["y"], a["z"], h, a["m"], a["u"])
    dv = 2.0 / (N_PAPER - 1)
    eps = dv * dv / 8.0 * 6.0 * math.pi ** 2 / 12.0
    # |rho_table - rho| <= eps B/h^3 sum_{b in N(a) + a} m_b
    nc, _, _, _ = ora.neighbors(direct, a["x"], a["y"], a["z"], h, with_lists=False)
    bound = eps * ora.bn(6.0) / h ** 3 * a["m"] * (nc + 1)
    assert np.all(np.abs(r1 - r0) <= bound)
    assert np.max(np.abs(r1 - r0) / bound) > 0.01      # the table is used
    assert np.max(np.abs(o1 - o0)) <= 10 * eps
    # the Newton h moves by the table's error, no more
    h1 = ora.update_h(tab.replace(newton_iters=12, h_ratio_max=8.0), a["x"], a["y"], a["z"],
                      a["h"])
    h0 = ora.update_h(direct.replace(newton_iters=12, h_ratio_max=8.0), a["x"], a["y"], a["z"],
                      a["h"])
    assert np.max(np.abs(h1 - h0) / h0) < 10 * eps
