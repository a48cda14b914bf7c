"""Pins of the oracle's Eq. 3 machinery (Sec. 3): FMM accelerations from the
expansion, PM accelerations of point sources, the twin's translation, the
norms and the downhill simplex.

* The interpolant-gradient weights equal a central difference of the
  interpolation weights themselves (built by the Vandermonde solve at shifted
  points, not by the derivative formula).
* With all mass in one leaf of a two-level tree, every target in that leaf's
  27-leaf neighbourhood has no far field, so the FMM acceleration from the
  expansion must equal PM's differenced potential exactly (periodic and twin).
* PM accelerations of point sources equal the 4th-order difference of the FFT
  convolution with the lattice G (an independent route), and, for the
  free-space twin, of the zero-padded convolution away from the faces; far
  from a source they approach the Newtonian -m x / (4 pi r^3).
* The expansion accelerations of a smooth field converge to PM's as p grows.
* The simplex finds known minima.
* The exact periodic force of a point mass (Ewald summation) does not depend
  on the splitting radius, tends to the Newtonian force plus the background's
  +x/3 near the source, and is translation and reflection covariant.
"""
import numpy as np

from oracle import conv, fd, fit, metric
from oracle import fmm as ofmm
from oracle import green as og


def test_interpolant_gradient_weights_are_the_derivative():
    for p, s in [(4, 16), (6, 16), (8, 16), (5, 8)]:
        v = (np.arange(s) + 0.5 - 0.5 * s) * (p / s)
        D = ofmm.interpolant_derivative_weights(p, v)
        d = 1e-5
        num = (ofmm.moment_matching_weights(p, v + d) - ofmm.moment_matching_weights(p, v - d)) / (2 * d)
        assert np.max(np.abs(D - num)) < 1e-6 * max(1.0, np.max(np.abs(D)))


def _one_leaf_mass(N, L, leaf, seed):
    s = N >> L
    rho = np.zeros((N, N, N))
    r = np.random.default_rng(seed).standard_normal((s, s, s))
    b = np.asarray(leaf) * s
    rho[b[0]:b[0] + s, b[1]:b[1] + s, b[2]:b[2] + s] = r
    return rho


def _neighbourhood_mask(N, L, leaf, periodic):
    s = N >> L
    nL = 1 << L
    idx = np.arange(N) // s
    m = np.ones((N, N, N), bool)
    for ax in range(3):
        d = idx - leaf[ax]
        if periodic:
            d = (d + nL // 2) % nL - nL // 2
        sel = np.abs(d) <= 1
        shape = [1, 1, 1]
        shape[ax] = N
        m &= sel.reshape(shape)
    return m


def test_expansion_accel_is_exact_where_the_far_field_vanishes():
    N, L, p = 16, 2, 4
    h = 1.0 / N
    for periodic, leaf in [(True, (0, 3, 1)), (False, (1, 2, 1))]:
        rho = _one_leaf_mass(N, L, leaf, seed=21)
        g, _ = ofmm.fmm_accel(rho, L, p, "S1", periodic=periodic)
        cells = np.argwhere(rho != 0)
        masses = rho[rho != 0] * h ** 3
        ref = metric.point_sources_accel(N, cells, masses, "S1", periodic=periodic)
        m = _neighbourhood_mask(N, L, leaf, periodic)
        err = np.max(np.abs(g[:, m] - ref[:, m]))
        assert err <= 1e-12 * np.max(np.abs(ref[:, m])), (periodic, err)
        # and the far field is what makes up the rest
        assert np.max(np.abs(g[:, ~m] - ref[:, ~m])) > 1e-9 * np.max(np.abs(ref))


def test_point_source_pm_accel_matches_fft_route():
    N = 16
    h = 1.0 / N
    rng = np.random.default_rng(22)
    cells = rng.integers(0, N, size=(3, 3))
    masses = rng.uniform(0.5, 2.0, size=3)
    for kind, a in [("S1", (-0.125,)), ("S", (-0.13,)), ("X", None)]:
        rho = np.zeros((N, N, N))
        for c, mm in zip(cells, masses):
            rho[tuple(c)] += mm / h ** 3
        ref = fd.accel_fd4(conv.pm(rho, kind, a) if a else conv.pm(rho, kind))
        got = metric.point_sources_accel(N, cells, masses, kind, a if a else (-0.125,))
        assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref)), kind
        sh = metric.point_sources_accel(N, cells, masses, kind, a if a else (-0.125,), shift=5)
        assert np.max(np.abs(sh - np.roll(got, (5, 5, 5), axis=(1, 2, 3)))) <= 1e-12 * np.max(np.abs(got))


def test_point_source_twin_accel():
    N = 16
    h = 1.0 / N
    cells = np.array([[3, 9, 7], [10, 4, 12]])
    masses = np.array([1.0, 0.7])
    rho = np.zeros((N, N, N))
    for c, mm in zip(cells, masses):
        rho[tuple(c)] = mm / h ** 3
    got = metric.point_sources_accel(N, cells, masses, periodic=False)
    # interior cells: the difference stencil stays inside the box
    ref = fd.accel_fd4(conv.isolated(rho))[:, 2:-2, 2:-2, 2:-2]
    assert np.max(np.abs(got[:, 2:-2, 2:-2, 2:-2] - ref)) <= 1e-11 * np.max(np.abs(ref))
    # far from a single source: Newtonian within the stencil's truncation
    one = metric.point_sources_accel(64, [[0, 0, 0]], [1.0], periodic=False)
    x = np.array([40, 30, 20]) / 64.0
    newton = -x / (4 * np.pi * np.linalg.norm(x) ** 3)
    assert np.max(np.abs(one[:, 40, 30, 20] - newton)) < 1e-6 * np.linalg.norm(newton)


def test_expansion_accel_converges_with_p():
    N, L = 32, 3
    rho = np.random.default_rng(23).standard_normal((N, N, N))
    ref = fd.accel_fd4(conv.pm(rho, "S1"))
    errs = []
    for p in (3, 5):
        g, _ = ofmm.fmm_accel(rho, L, p, "S1")
        errs.append(np.max(np.abs(g - ref)) / np.max(np.abs(ref)))
    assert errs[1] < 0.2 * errs[0] and errs[1] < 1e-3, errs


def test_norms_and_delta_g():
    e = np.random.default_rng(24).standard_normal((3, 4, 4, 4))
    assert np.all(metric.delta_g(e, e) == 0)
    dg = metric.delta_g(e, 0 * e)
    assert np.allclose(dg, np.linalg.norm(e, axis=0))
    l2, lmax = metric.norms(dg)
    assert np.isclose(l2, np.sqrt(np.mean(np.sum(e * e, axis=0)))) and lmax == dg.max()
    assert np.array_equal(metric.untranslate(np.roll(e, 2, axis=(1, 2, 3)), 2), e)
    assert metric.twin_shift(128) == 64


def test_nelder_mead_finds_known_minima():
    x, fx, nev = fit.nelder_mead(lambda v: (v[0] - 0.3) ** 2 + 1.0, [0.0], 0.1, xtol=1e-9)
    assert abs(x[0] - 0.3) < 1e-8 and abs(fx - 1.0) < 1e-15
    assert nev < 100  # stops on the simplex size, well before the iteration cap

    def rosen(v):
        return (1 - v[0]) ** 2 + 100 * (v[1] - v[0] ** 2) ** 2
    x, fx, _ = fit.nelder_mead(rosen, [-1.2, 1.0], 0.5, xtol=1e-8, maxiter=2000)
    assert np.max(np.abs(x - 1.0)) < 1e-6 and fx < 1e-12
    # a non-smooth (L_MAX-like) objective
    x, _, _ = fit.nelder_mead(lambda v: max(abs(v[0] - 0.2), abs(v[1] + 0.4)), [0, 0], 0.3,
                              xtol=1e-9, maxiter=2000)
    assert np.max(np.abs(x - [0.2, -0.4])) < 1e-7


def test_exact_periodic_force_of_a_point_mass():
    N = 32
    h = 1.0 / N
    g1 = metric.periodic_point_accel(N, (0, 0, 0), alpha=0.08)
    g2 = metric.periodic_point_accel(N, (0, 0, 0), alpha=0.12)
    # Ewald's split does not depend on the splitting radius
    assert np.nanmax(np.abs(g1 - g2)) < 1e-8 * np.nanmax(np.abs(g1))
    # near the source: Newtonian plus the background's +x/3 (the images' linear
    # tidal terms cancel by cubic symmetry)
    for c in [(2, 0, 0), (2, 2, 1), (1, 1, 1)]:
        x = np.array(c) * h
        r = np.linalg.norm(x)
        rest = g1[:, c[0], c[1], c[2]] + x / (4 * np.pi * r ** 3)
        assert np.max(np.abs(rest - x / 3)) < 0.05 * np.linalg.norm(x / 3)
    # translation
    g3 = metric.periodic_point_accel(N, (5, 7, 9), alpha=0.1)
    g0 = metric.periodic_point_accel(N, (0, 0, 0), alpha=0.1)
    assert np.nanmax(np.abs(np.roll(g0, (5, 7, 9), axis=(1, 2, 3)) - g3)) < 1e-12 * np.nanmax(np.abs(g0))
    # point reflection through the source: g(-x) = -g(x)
    flip = -np.roll(np.flip(g0, axis=(1, 2, 3)), 1, axis=(1, 2, 3))
    m = np.isfinite(g0)
    assert np.max(np.abs(flip[m] - g0[m])) < 1e-12 * np.nanmax(np.abs(g0))
