"""Pins of the oracle's learned-correction network: closed forms of the
activation and of a hand-set network, zero-output fallback, symmetry."""
import itertools
import math

import numpy as np

from oracle import mlp


def test_silu_closed_form():
    for z in (-3.0, -0.5, 0.0, 0.7, 4.0):
        assert abs(mlp.silu(np.array(z)) - z / (1 + math.exp(-z))) < 1e-15


def test_zero_output_layer_is_the_plain_table():
    rng = np.random.default_rng(0)
    th = rng.standard_normal(mlp.N_PARAMS)
    th[mlp.O_W3:] = 0.0
    tab = rng.standard_normal((9, 9, 9))
    np.testing.assert_array_equal(mlp.corrected_table(tab, 2, 3, th), tab)


def test_hand_set_network():
    # one path: h1_0 = silu(x0), h2_0 = silu(2 h1_0 - 1), out = 3 h2_0 + 0.5
    th = np.zeros(mlp.N_PARAMS)
    th[mlp.O_W1 + 0 * mlp.N_IN + 0] = 1.0   # W1[0][0]
    th[mlp.O_W2 + 0 * 64 + 0] = 2.0         # W2[0][0]
    th[mlp.O_B2 + 0] = -1.0                 # b2[0]
    th[mlp.O_W3 + 0] = 3.0                  # W3[0]
    th[mlp.O_B3] = 0.5                      # b3
    assert mlp.N_PARAMS == 8 * 64 + 64 + 64 * 64 + 64 + 64 + 1
    for x0 in (0.0, 0.3, 0.9):
        x = np.array([x0, 0.2, 0.1, 0.5, 0.0, 0.25, 0.25, 0.6])
        s = lambda z: z / (1 + math.exp(-z))
        expect = 3 * s(2 * s(x0) - 1) + 0.5
        assert abs(mlp.forward(th, x) - expect) < 1e-14


def test_features_cube_symmetry():
    rng = np.random.default_rng(1)
    j = rng.integers(-23, 24, (50, 3))
    f = mlp.features(j, 3, 6)
    for perm in itertools.permutations(range(3)):
        for sg in itertools.product((1, -1), repeat=3):
            np.testing.assert_array_equal(mlp.features(j[:, perm] * np.array(sg), 3, 6), f)
    assert np.all(f[:, 0] >= f[:, 1]) and np.all(f[:, 1] >= f[:, 2])
    np.testing.assert_allclose(f[:, 6:], [[3 / 8, 0.6]] * 50)


def test_features_carry_the_in_gridlet_residue():
    # j = a - a' - p d (Eq. 6): along an axis with d_i = 0 the residue is
    # |a_i - a'_i| itself; with d_i = 1 and a_i - a'_i = r >= 0 it is p - r
    # for 0 < r < p
    p = 6
    for r in range(0, p):
        f0 = mlp.features(np.array([r, 0, 0]), 2, p)
        assert f0[0] == r / (4 * p) and f0[3] == r / p
    for r in range(1, p):
        f1 = mlp.features(np.array([r - p, 0, 0]), 2, p)
        assert f1[0] == (p - r) / (4 * p) and f1[3] == (p - r) / p
    f = mlp.features(np.array([[13, -7, 2]]), 3, 6)[0]
    np.testing.assert_array_equal(f[:6], [13 / 24, 7 / 24, 2 / 24, 1 / 6, 1 / 6, 2 / 6])
