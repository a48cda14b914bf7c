"""Pins of the oracle's isolated (non-periodic) twin (Sec. 3, Eq. 3): the
free-space convolution and the FMM with no periodic images.

* ``conv.isolated`` (zero-padded FFT) equals the pairwise sum of G_0 from its
  formula (brute force, 8^3), and a unit point mass gives -1/(4 pi r) exactly.
* ``fmm(..., periodic=False)`` with two levels and gridlet = leaf (s = p)
  equals the direct isolated sum, as in the periodic case (Sec. 3: identical
  by construction).
* The isolated FMM operator is symmetric (reciprocity: the potential at cell a
  from a unit mass at b equals that at b from a unit mass at a) and commutes
  with the reflections of the box; its error falls with p.
"""
import numpy as np

from oracle import conv, fmm as ofmm
from oracle import green as ogreen


def test_isolated_fft_equals_brute_force():
    rho = np.random.default_rng(11).standard_normal((8, 8, 8)) + 0.3  # nonzero mean: no images
    a = conv.isolated(rho)
    b = conv.isolated_brute(rho)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_isolated_point_mass_is_newtonian():
    N = 16
    h = 1.0 / N
    rho = np.zeros((N, N, N))
    src = (3, 11, 6)
    rho[src] = 1.0 / h ** 3                       # unit mass
    phi = conv.isolated(rho)
    for c in [(0, 0, 0), (15, 15, 15), (3, 11, 7), (12, 2, 9)]:
        r = h * np.linalg.norm(np.subtract(c, src))
        assert abs(phi[c] - (-1.0 / (4 * np.pi * r))) <= 1e-12 * abs(phi[c])
    assert abs(phi[src] - ogreen.self_value(h)) <= 1e-12 * abs(phi[src])


def test_isolated_two_levels_gridlet_equals_leaf_is_direct():
    rho = np.random.default_rng(12).standard_normal((16, 16, 16))
    a = ofmm.fmm(rho, 2, 4, periodic=False)
    b = conv.isolated(rho)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    tg = np.array([[0, 0, 0], [15, 3, 7], [8, 8, 8], [1, 14, 2]])
    t = ofmm.fmm(rho, 2, 4, periodic=False, targets=tg)
    assert np.max(np.abs(t - a[tg[:, 0], tg[:, 1], tg[:, 2]])) <= 1e-13 * np.max(np.abs(a))


def test_isolated_fmm_is_symmetric_and_reflection_covariant():
    N, L, p = 16, 3, 4
    a, b = (1, 2, 14), (13, 9, 3)
    ea = np.zeros((N, N, N))
    ea[a] = 1.0
    eb = np.zeros((N, N, N))
    eb[b] = 1.0
    pa = ofmm.fmm(ea, L, p, periodic=False)
    pb = ofmm.fmm(eb, L, p, periodic=False)
    assert abs(pa[b] - pb[a]) <= 1e-12 * abs(pa[b])
    rho = np.random.default_rng(13).standard_normal((N, N, N))
    ref = ofmm.fmm(rho, L, p, periodic=False)
    for ax in range(3):
        got = ofmm.fmm(np.flip(rho, axis=ax), L, p, periodic=False)
        assert np.max(np.abs(got - np.flip(ref, axis=ax))) <= 1e-12 * np.max(np.abs(ref))


def test_isolated_fmm_error_falls_with_p():
    rho = np.random.default_rng(14).standard_normal((32, 32, 32))
    exact = conv.isolated(rho)
    errs = [np.max(np.abs(ofmm.fmm(rho, 3, p, periodic=False) - exact)) for p in (3, 4, 6)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-4 * np.max(np.abs(exact))
