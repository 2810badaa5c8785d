"""Pins of the oracle's self-gravity (a multipole expansion on the particle
octree, section 4.1).  The direct sum is Newton's law with Plummer softening;
the expansion of two equal masses at +-a on the z axis is known in closed form
to second order along both axes; a single particle has no quadrupole, so its
expansion is its softened pair force; the tree with theta = 0 opens every node
and must equal the direct sum; and the tree's error shrinks with theta."""
import math

import numpy as np
import pytest


def _cluster(n=2000, seed=1):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 3)) * 0.3
    m = rng.uniform(0.5, 1.5, n) / n
    return X, m


def test_direct_pair_is_softened_newton(ora):
    G, eps = 2.5, 0.1
    x = np.array([0.0, 0.7]); y = np.array([0.0, -0.2]); z = np.array([0.0, 0.4])
    m = np.array([3.0, 5.0])
    gx, gy, gz, _ = ora.gravity_direct(x, y, z, m, G, eps)
    d = np.array([0.7, -0.2, 0.4])
    f = G / (d @ d + eps ** 2) ** 1.5
    assert np.allclose([gx[0], gy[0], gz[0]], f * m[1] * d, rtol=1e-15, atol=0)
    assert np.allclose([gx[1], gy[1], gz[1]], -f * m[0] * d, rtol=1e-15, atol=0)


def test_direct_sum_conserves_momentum(ora):
    X, m = _cluster(500)
    gx, gy, gz, sc = ora.gravity_direct(X[:, 0], X[:, 1], X[:, 2], m, 1.0, 0.01)
    tot = np.abs([np.sum(m * gx), np.sum(m * gy), np.sum(m * gz)]).max()
    assert tot <= 1e-15 * np.sum(m * sc)


@pytest.mark.parametrize("axis", [0, 2])
def test_quadrupole_of_two_masses_closed_form(ora, axis):
    """Masses m at (0, 0, +-a), target at distance d on the x or the z axis.
    Exact: g_x = -2Gm d/(d^2+a^2)^(3/2), g_z = -Gm(1/(d-a)^2 + 1/(d+a)^2); to
    second order -2Gm/d^2 + 3Gma^2/d^4 and -2Gm/d^2 - 6Gma^2/d^4.  The
    expansion matches the second-order terms, so its error against the exact
    field falls as (a/d)^4: 16x when a halves."""
    G, m, d = 1.3, 0.7, 1.0
    errs = []
    for a in (0.02, 0.01):
        x = np.zeros(2); y = np.zeros(2); z = np.array([a, -a])
        mo = ora.moments([0, 1], x, y, z, np.full(2, m))
        assert mo[0] == 2 * m and np.allclose(mo[1:4], 0.0)
        assert mo[4] + mo[7] + mo[9] == pytest.approx(0.0, abs=1e-18)    # traceless
        pos = np.zeros(3)
        pos[axis] = d
        g = ora.multipole_accel(mo, pos, G, 0.0)
        if axis == 0:
            exact = -2 * G * m * d / (d * d + a * a) ** 1.5
            second = -2 * G * m / d ** 2 + 3 * G * m * a * a / d ** 4
        else:
            exact = -G * m * (1 / (d - a) ** 2 + 1 / (d + a) ** 2)
            second = -2 * G * m / d ** 2 - 6 * G * m * a * a / d ** 4
        assert g[axis] == pytest.approx(second, rel=1e-14)
        assert np.allclose(np.delete(g, axis), 0.0, atol=1e-18)
        errs.append(abs(g[axis] - exact))
    assert 14.0 < errs[0] / errs[1] < 18.0


def test_single_particle_expansion_is_its_softened_pair_force(ora):
    G, eps = 0.9, 0.05
    x, y, z, m = np.array([0.3]), np.array([-0.1]), np.array([0.2]), np.array([2.0])
    mo = ora.moments([0], x, y, z, m)
    assert np.allclose(mo[4:], 0.0)
    pos = np.array([1.0, 0.5, -0.4])
    g = ora.multipole_accel(mo, pos, G, eps)
    d = pos - np.array([0.3, -0.1, 0.2])
    want = -G * 2.0 * d / (d @ d + eps ** 2) ** 1.5
    assert np.allclose(g, want, rtol=1e-14, atol=0)


def test_moments_shift_invariance(ora):
    X, m = _cluster(200)
    idx = np.arange(200)
    a = ora.moments(idx, X[:, 0], X[:, 1], X[:, 2], m)
    s = np.array([0.3, -1.1, 2.0])
    b = ora.moments(idx, X[:, 0] + s[0], X[:, 1] + s[1], X[:, 2] + s[2], m)
    assert np.allclose(b[1:4], a[1:4] + s, rtol=0, atol=1e-14)
    assert np.allclose(b[4:], a[4:], rtol=0, atol=1e-13 * np.abs(a[4:]).max())


def test_tree_with_theta_zero_is_the_direct_sum(ora):
    X, m = _cluster(3000)
    lo, hi = X.min(0), X.max(0)
    L = ora.gravity_leaf_level(X.shape[0])
    gd = ora.gravity_direct(X[:, 0], X[:, 1], X[:, 2], m, 1.0, 0.01)
    gt = ora.gravity_tree(X[:, 0], X[:, 1], X[:, 2], m, lo, hi, L, 1.0, 0.01, 0.0)
    err = max(np.max(np.abs(gt[k] - gd[k])) for k in range(3)) / np.max(gd[3])
    assert err < 1e-13


def test_tree_error_shrinks_with_theta(ora):
    """Max error against the direct sum, scaled by the largest per-particle sum
    of |terms|: decreasing in theta, and below 1e-3 at theta = 0.5; the
    quadrupole makes the error fall faster than theta^2 (a monopole-only
    expansion falls as theta^2)."""
    X, m = _cluster(4000, seed=7)
    lo, hi = X.min(0), X.max(0)
    L = ora.gravity_leaf_level(X.shape[0])
    gd = ora.gravity_direct(X[:, 0], X[:, 1], X[:, 2], m, 1.0, 0.01)
    errs = {}
    for th in (0.2, 0.4, 0.6, 0.8):
        gt = ora.gravity_tree(X[:, 0], X[:, 1], X[:, 2], m, lo, hi, L, 1.0, 0.01, th)
        errs[th] = max(np.max(np.abs(gt[k] - gd[k])) for k in range(3)) / np.max(gd[3])
    e = [errs[t] for t in sorted(errs)]
    assert all(a < b for a, b in zip(e, e[1:])), errs
    assert errs[0.4] < 1e-3
    assert errs[0.8] / errs[0.4] > 4.0, errs


def test_tree_momentum_balance(ora):
    """The expansion breaks pairwise antisymmetry only at its own error."""
    X, m = _cluster(3000, seed=3)
    lo, hi = X.min(0), X.max(0)
    L = ora.gravity_leaf_level(X.shape[0])
    gx, gy, gz, sc = ora.gravity_tree(X[:, 0], X[:, 1], X[:, 2], m, lo, hi, L, 1.0, 0.01, 0.5)
    tot = np.abs([np.sum(m * gx), np.sum(m * gy), np.sum(m * gz)]).max()
    assert tot <= 1e-3 * np.sum(m * sc)


def test_leaf_level_rule(ora):
    assert ora.gravity_leaf_level(1) == 0
    assert ora.gravity_leaf_level(7) == 0
    assert ora.gravity_leaf_level(8) == 1
    assert ora.gravity_leaf_level(511) == 2
    assert ora.gravity_leaf_level(512) == 3
    assert ora.gravity_leaf_level(10 ** 9) == 9


def _octant_config(pair_at, target_at, extra=(), pair_mass=1.0):
    """8 particles in the unit cube [0, 1]^3 (the key domain, fixed by two
    corner particles): two levels (L = 1, eight octant nodes of size 1/2).
    A tight pair sits at pair_at, the target (index 2) at target_at."""
    pts = [(0.0, 0.0, 0.0), (1.0, 1.0, 1.0)]          # the corners fix the domain
    pts = [tuple(np.add(pair_at, (0, 0, 0.01))), tuple(np.add(pair_at, (0, 0, -0.01))),
           target_at] + list(extra) + pts
    X = np.array(pts, dtype=float)
    m = np.ones(len(pts))
    m[-2:] = 1e-30                                    # the corners carry no mass
    m[:2] = pair_mass
    return X, m


def test_opening_rule_is_size_over_distance(ora):
    """The pair's octant (size 1/2) seen from the target in the opposite octant is
    expanded exactly when 1/2 < theta d (d: the distance to its centre of mass):
    just above theta = 1/(2d) the target gets the expansion, just below the
    direct pair sum."""
    X, m = _octant_config((0.2, 0.2, 0.2), (0.8, 0.8, 0.8),
                          extra=[(0.3, 0.8, 0.2), (0.8, 0.3, 0.2), (0.2, 0.3, 0.8)])
    lo, hi = np.zeros(3), np.ones(3)
    assert ora.gravity_leaf_level(X.shape[0]) == 1
    d = np.linalg.norm(X[2] - 0.5 * (X[0] + X[1]))
    th_c = 0.5 / d
    gd = ora.gravity_direct(X[:, 0], X[:, 1], X[:, 2], m, 1.0, 0.0, targets=[2])
    mo = ora.moments([0, 1], X[:, 0], X[:, 1], X[:, 2], m)
    gm = ora.multipole_accel(mo, X[2], 1.0, 0.0)
    assert abs(gm[2] - (gd[2][2] - 0.0)) > 1e-9          # the expansion differs visibly
    for th, expanded in ((th_c * 1.001, True), (th_c * 0.999, False)):
        gt = ora.gravity_tree(X[:, 0], X[:, 1], X[:, 2], m, lo, hi, 1, 1.0, 0.0, th,
                              targets=[2])
        got = np.array([gt[0][2], gt[1][2], gt[2][2]])
        want = np.array([gd[0][2], gd[1][2], gd[2][2]])
        if expanded:
            # the pair's node contributes its expansion, the single particles
            # their exact forces
            others = ora.gravity_direct(X[2:, 0], X[2:, 1], X[2:, 2], m[2:], 1.0, 0.0,
                                        targets=[0])
            want = gm + np.array([others[0][0], others[1][0], others[2][0]])
        assert np.allclose(got, want, rtol=1e-13, atol=0), (th, got, want)


def test_the_targets_own_node_is_always_opened(ora):
    """With theta = 0.9 the target's own octant would pass the size test (its
    mass sits in the far corner of the octant), but a node holding the target is
    opened: the target gets the direct sum of its octant-mates, never an
    expansion that includes itself."""
    X, m = _octant_config((0.45, 0.45, 0.44), (0.02, 0.02, 0.02), pair_mass=100.0)
    lo, hi = np.zeros(3), np.ones(3)
    mo = ora.moments(np.arange(X.shape[0] - 1), X[:, 0], X[:, 1], X[:, 2], m)
    assert 0.5 < 0.9 * np.linalg.norm(X[2] - mo[1:4])   # the size test alone would expand
    gt = ora.gravity_tree(X[:, 0], X[:, 1], X[:, 2], m, lo, hi, 1, 1.0, 0.0, 0.9, targets=[2])
    gd = ora.gravity_direct(X[:, 0], X[:, 1], X[:, 2], m, 1.0, 0.0, targets=[2])
    assert np.allclose([gt[k][2] for k in range(3)], [gd[k][2] for k in range(3)],
                       rtol=1e-14, atol=0)
