"""Pins of the oracle's integrator (section 4.1: second-order Press / kick-drift
leapfrog for x, v and second-order Adams-Bashforth for u) and time-step rule."""
import numpy as np
import pytest

from conftest import oracle_config
from paper_2005_02656_amd import inputs


def _state(n, x0, v0, u0):
    z = np.zeros(n)
    return dict(x=x0[0].copy(), y=x0[1].copy(), z=x0[2].copy(), vx=v0[0].copy(),
                vy=v0[1].copy(), vz=v0[2].copy(), vhx=v0[0].copy(), vhy=v0[1].copy(),
                vhz=v0[2].copy(), u=u0.copy(), du_m1=z.copy(), h=np.ones(n), m=np.ones(n))


OPEN = dict(box_lo=(-100.0,) * 3, box_hi=(100.0,) * 3, periodic=(0, 0, 0))


def test_constant_acceleration_exact(ora):
    cfg = oracle_config(inputs.base_params(**OPEN))
    rng = np.random.default_rng(0)
    n = 5
    x0, v0, g = rng.normal(size=(3, n)), rng.normal(size=(3, n)), rng.normal(size=(3, n))
    u0, du = rng.random(n), rng.normal(size=n)
    st = _state(n, x0, v0, u0)
    T, lam = 0.0, 0.0
    for dt in [0.1, 0.13, 0.07, 0.11, 0.05]:
        st = ora.integrate(cfg, st, g[0], g[1], g[2], du, dt, lam)
        T += dt
        lam = dt
    for k, c in enumerate("xyz"):
        assert np.allclose(st[c], x0[k] + v0[k] * T + 0.5 * g[k] * T * T, rtol=0, atol=1e-14)
        assert np.allclose(st["v" + c], v0[k] + g[k] * T, rtol=0, atol=1e-14)
    assert np.allclose(st["u"], u0 + du * T, atol=1e-14)


def test_ab2_exact_for_linear_rate(ora):
    """After the Euler start-up, each AB2 increment integrates du = alpha + beta t exactly."""
    cfg = oracle_config(inputs.base_params(**OPEN))
    n = 3
    alpha, beta = np.array([0.3, -1.0, 2.0]), np.array([1.5, 0.2, -0.7])
    st = _state(n, np.zeros((3, n)), np.zeros((3, n)), np.ones(n))
    t, lam = 0.0, 0.0
    for i, dt in enumerate([0.1, 0.2, 0.05, 0.15]):
        du = alpha + beta * t
        u_before = st["u"].copy()
        st = ora.integrate(cfg, st, np.zeros(n), np.zeros(n), np.zeros(n), du, dt, lam)
        if i > 0:
            exact = alpha * dt + beta * ((t + dt) ** 2 - t ** 2) / 2
            assert np.allclose(st["u"] - u_before, exact, rtol=1e-13, atol=1e-15)
        t += dt
        lam = dt


def test_second_order_convergence(ora):
    """Harmonic oscillator a = -x from x=1, v=0 to T=1 with a varying step pattern."""
    cfg = oracle_config(inputs.base_params(**OPEN))

    def run(k):
        st = _state(1, np.array([[1.0], [0.0], [0.0]]), np.zeros((3, 1)), np.zeros(1))
        pattern = np.array([1.0, 1.3, 0.7, 1.1, 0.9])
        dts = np.tile(pattern, k)
        dts *= 1.0 / dts.sum()
        lam = 0.0
        for dt in dts:
            st = ora.integrate(cfg, st, -st["x"], np.zeros(1), np.zeros(1), np.zeros(1), dt, lam)
            lam = dt
        return st["x"][0], st["vx"][0]

    errs = []
    for k in (8, 16, 32):
        x, v = run(k)
        errs.append(abs(x - np.cos(1.0)) + abs(v + np.sin(1.0)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.5 < r2 < 4.6, errs


def test_periodic_wrap(ora):
    cfg = oracle_config(inputs.base_params())
    st = _state(2, np.array([[0.99, 0.01], [0.5, 0.5], [0.5, 0.5]]),
                np.array([[1.0, -1.0], [0.0, 0.0], [0.0, 0.0]]), np.ones(2))
    z = np.zeros(2)
    st = ora.integrate(cfg, st, z, z, z, z, 0.02, 0.0)
    assert np.allclose(st["x"], [0.01, 0.99], atol=1e-15)
    assert np.all((st["x"] >= 0) & (st["x"] < 1))


def test_timestep_rule(ora):
    cfg = oracle_config(inputs.base_params(), acc_dt=0.0, energy_dt=0.0)
    h = np.array([0.1, 0.05, 0.2])
    c = np.array([1.0, 2.0, 0.5])
    z = np.zeros(3)
    u = np.ones(3)
    assert ora.timestep(cfg, h, c, u, z, z, z, z, 0.0) == pytest.approx(0.2 * 0.025, rel=1e-15)
    # growth limit 1.1 x previous
    assert ora.timestep(cfg, h, c, u, z, z, z, z, 0.001) == pytest.approx(0.0011, rel=1e-15)
    assert ora.timestep(cfg, h, c, u, z, z, z, z, 1.0) == pytest.approx(0.005, rel=1e-15)
    # acceleration criterion: |a| = 5 at h = 0.2 gives 0.2 sqrt(0.2/5) = 0.04 ...
    ca = cfg.replace(acc_dt=0.2)
    ax = np.array([0.0, 0.0, 3.0])
    ay = np.array([0.0, 0.0, 4.0])
    c2 = np.array([1e-3, 1e-3, 1e-3])    # slow sound: Courant would give 4.0+
    assert ora.timestep(ca, h, c2, u, ax, ay, z, z, 0.0) == pytest.approx(0.04, rel=1e-15)
    # ... and the energy criterion |u|/|du| = 1/50 gives 0.004
    ce = ca.replace(energy_dt=0.2)
    du = np.array([0.0, -50.0, 0.0])
    assert ora.timestep(ce, h, c2, u, ax, ay, z, du, 0.0) == pytest.approx(0.004, rel=1e-15)
