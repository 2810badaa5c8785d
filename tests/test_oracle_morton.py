"""Pins of the oracle's depth-first (Morton-like) key and its stable ordering
(section 4.3), by hand-computed keys."""
import numpy as np

LO = np.array([-0.5, -0.5, 0.0])
HI = np.array([0.5, 0.5, 2.0])
Q = 2 ** 21


def pos(qx, qy, qz):
    D = HI - LO
    return [LO[k] + (q + 0.5) * D[k] / Q for k, q in enumerate((qx, qy, qz))]


def test_hand_keys(ora):
    cases = {(0, 0, 0): 0, (1, 0, 0): 4, (0, 1, 0): 2, (0, 0, 1): 1, (1, 1, 1): 7,
             (2, 0, 0): 32, (3, 5, 6): 238, (Q - 1, Q - 1, Q - 1): 2 ** 63 - 1,
             (Q // 2, 0, 0): 1 << 62, (0, Q // 2, 0): 1 << 61, (0, 0, Q // 2): 1 << 60}
    P = np.array([pos(*q) for q in cases])
    keys = ora.morton_keys(P[:, 0], P[:, 1], P[:, 2], LO, HI)
    assert [int(k) for k in keys] == list(cases.values())


def test_clamping_and_degenerate_axis(ora):
    x = np.array([-0.5, 0.5, 0.7, -0.9])     # lo maps to 0, hi and beyond clamp to 2^21-1
    y = np.zeros(4)
    z = np.zeros(4)
    keys = ora.morton_keys(x, y, z, LO, HI)
    qx = [0, Q - 1, Q - 1, 0]
    # y = 0 sits at the middle of [-0.5, 0.5]: q_y = 2^20
    for k, q in zip(keys, qx):
        assert (int(k) >> 61) & 1 == 1
        got = 0
        for i in range(21):
            got |= ((int(k) >> (3 * i + 2)) & 1) << i
        assert got == q
    # zero extent: q = 0
    k0 = ora.morton_keys(np.array([3.0]), np.array([3.0]), np.array([3.0]),
                         np.array([3.0, 3.0, 3.0]), np.array([3.0, 3.0, 3.0]))
    assert int(k0[0]) == 0


def test_stable_sort(ora):
    keys = np.array([5, 3, 5, 1, 3, 5, 0], dtype=np.uint64)
    perm = ora.sort_keys(keys)
    assert list(perm) == [6, 3, 1, 4, 0, 2, 5]


def test_level_order_is_a_stable_prefix_sort(ora):
    """The particle order of the cell build: a stable sort by the keys' prefix of
    L levels (numpy's stable argsort of key >> 3(21 - L)); at L = 21 it is the
    full-key order, and inside one finest cell the input order survives."""
    rng = np.random.default_rng(4)
    keys = rng.integers(0, 1 << 63, 5000, dtype=np.uint64)
    keys[1000:1100] = keys[50]          # ties
    for L in (0, 1, 3, 7, 8, 9, 21):
        want = np.argsort(keys >> np.uint64(3 * (21 - L)), kind="stable")
        assert np.array_equal(ora.sort_keys(keys, level=L), want), L
    assert np.array_equal(ora.sort_keys(keys, level=21), ora.sort_keys(keys))
