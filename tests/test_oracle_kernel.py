"""Pins of the oracle's interpolation kernel (eq. 6) against mathematics that does
not go through the oracle: numpy's own sinc, scipy's adaptive quadrature, a
Cartesian Riemann sum of the kernel, and finite differences."""
import math

import numpy as np
import pytest
from scipy import integrate


def np_S(v, n):
    # numpy's sinc is sin(pi t)/(pi t): S_n(pi v / 2) = sinc(v/2)^n
    return np.sinc(np.asarray(v) / 2.0) ** n


@pytest.mark.parametrize("n", [3, 4, 5, 6, 7, 8])
def test_bn_against_scipy_quad(ora, n):
    val, err = integrate.quad(lambda v: np_S(v, n) * v * v, 0.0, 2.0, epsabs=1e-300, epsrel=1e-13,
                              limit=200)
    ref = 1.0 / (4.0 * math.pi * val)
    assert abs(ora.bn(n) - ref) <= 1e-13 * ref


def test_bn6_value(ora):
    # value quoted from an independent numpy/scipy evaluation (two quadratures)
    assert abs(ora.bn(6) - 0.790449589432298) < 1e-14


@pytest.mark.parametrize("n", [3, 6, 8])
def test_S_matches_numpy_sinc(ora, n):
    for v in [0.0, 1e-9, 0.03, 0.5, 1.0, 1.37, 1.999]:
        assert abs(ora.S(v, n) - np_S(v, n)) <= 1e-15 * max(1.0, abs(np_S(v, n)))


@pytest.mark.parametrize("n", [3.0, 6.0, 5.5])
def test_dSdv_finite_difference(ora, n):
    for v in [0.001, 0.02, 0.0637, 0.07, 0.4, 1.1, 1.9]:
        eps = 1e-6
        fd = (ora.S(v + eps, n) - ora.S(v - eps, n)) / (2 * eps)
        assert abs(ora.dSdv(v, n) - fd) <= 1e-8, (v, ora.dSdv(v, n), fd)


def test_W_closed_forms(ora):
    n, h = 6.0, 0.37
    b = ora.bn(n)
    assert ora.W(0.0, h, n, b) == pytest.approx(b / h ** 3, rel=1e-15)
    assert ora.W((2 * h) * (2 * h), h, n, b) == 0.0          # v = 2 is outside (strict <)
    r = 2 * h * (1 - 1e-9)
    assert 0.0 < ora.W(r * r, h, n, b) < 1e-40                # S_6 ~ (2 - v)^6 at the edge
    # dW/dr -> 0 at the edge of the support
    e = 1e-5 * h
    r1 = 2 * h - e
    dwdr = (ora.W(r1 * r1, h, n, b) - ora.W((r1 - e) ** 2, h, n, b)) / e
    assert abs(dwdr) < 1e-20 * b / h ** 4


@pytest.mark.parametrize("h", [0.05, 0.2])
def test_W_normalised_riemann_sum(ora, h):
    """int W d^3x = 1 via a Cartesian midpoint sum (checks B_n and the 1/h^3 scaling)."""
    n = 6.0
    b = ora.bn(n)
    k = 28
    dx = 2 * h / k
    g = (np.arange(-k, k) + 0.5) * dx
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z).ravel()
    # evaluate W through numpy's sinc: same definition, independent evaluation
    ref = np.where(r < 2 * h, b / h ** 3 * np_S(r / h, n), 0.0).sum() * dx ** 3
    assert abs(ref - 1.0) < 1e-6
    # and the oracle's W at a sample of the same points agrees with numpy's
    idx = np.random.default_rng(0).integers(0, r.size, 500)
    for i in idx:
        expect = b / h ** 3 * np_S(r[i] / h, n) if r[i] < 2 * h else 0.0
        assert abs(ora.W(r[i] ** 2, h, n, b) - expect) <= 1e-14 * b / h ** 3


def test_dWdh_finite_difference(ora):
    n = 6.0
    b = ora.bn(n)
    for h in [0.1, 0.3]:
        for v in [0.0, 0.2, 0.9, 1.5, 1.95]:
            r2 = (v * h) ** 2
            e = 1e-6 * h
            fd = (ora.W(r2, h + e, n, b) - ora.W(r2, h - e, n, b)) / (2 * e)
            got = ora.dWdh(r2, h, n, b)
            assert abs(got - fd) <= 1e-7 * b / h ** 4, (h, v, got, fd)
