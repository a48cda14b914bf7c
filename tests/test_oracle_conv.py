"""Pins of the oracle's exact periodic convolution ("PM with G", Eq. 4) and of
PM with G_K (Eq. 1): brute force, closed-form single modes, invariants."""
import numpy as np
import pytest

from oracle import conv, fd, green
from paper_2011_07099_amd import fields

KINDS = ("X", "S1", "K")


def _rho(N, seed):
    r = np.random.default_rng(seed).standard_normal((N, N, N))
    return r - r.mean()


@pytest.mark.parametrize("kind", KINDS)
def test_direct_equals_fft(kind):
    N = 8
    rho = _rho(N, 3)
    g = conv.lattice_table(kind, N)
    a = conv.direct(rho, g)
    b = conv.fft(rho, g)
    np.testing.assert_allclose(a, b, atol=1e-12 * np.abs(a).max())


@pytest.mark.parametrize("kind", KINDS)
def test_brute_force_8cubed(kind):
    # every pair evaluated from the closed form (no table, no FFT)
    N = 8
    rho = _rho(N, 4)
    a = conv.brute(rho, kind)
    b = conv.fft(rho, conv.lattice_table(kind, N))
    np.testing.assert_allclose(a, b, atol=1e-12 * np.abs(b).max())


def test_pm_gk_equals_direct_with_gk():
    N = 16
    rho = _rho(N, 5)
    a = conv.pm_gk(rho)
    b = conv.direct(rho, conv.lattice_table("K", N), targets=[(0, 0, 0), (3, 7, 11), (15, 15, 0)])
    np.testing.assert_allclose(a[[0, 3, 15], [0, 7, 15], [0, 11, 0]], b, atol=1e-12 * np.abs(a).max())


def test_pm_gk_single_mode_closed_form():
    # rho = cos(2 pi n.x) is an eigenfunction: Phi = -rho / (2 pi |n|)^2
    N = 16
    x = (np.arange(N) + 0.5) / N
    for n in [(1, 0, 0), (2, 3, 1), (0, 0, 8)]:
        ph = 2 * np.pi * (n[0] * x[:, None, None] + n[1] * x[None, :, None] + n[2] * x[None, None, :])
        rho = np.cos(ph)
        k2 = (2 * np.pi) ** 2 * sum(v * v for v in n)
        np.testing.assert_allclose(conv.pm_gk(rho), -rho / k2, atol=1e-14)


@pytest.mark.parametrize("kind", KINDS)
def test_translation_invariance(kind):
    N = 8
    rho = _rho(N, 6)
    g = conv.lattice_table(kind, N)
    phi = conv.direct(rho, g)
    sh = (3, -2, 5)
    phi2 = conv.direct(np.roll(rho, sh, (0, 1, 2)), g)
    np.testing.assert_allclose(phi2, np.roll(phi, sh, (0, 1, 2)), atol=1e-12 * np.abs(phi).max())


@pytest.mark.parametrize("kind", KINDS)
def test_zero_mean_potential_and_zero_net_force(kind):
    N = 16
    rho = fields.lognormal(N, 2.0, 1.0, seed=9)
    phi = conv.pm(rho, kind)
    assert abs(phi.mean()) < 1e-12 * np.abs(phi).max()
    acc = fd.accel_fd4(phi)
    net = np.array([np.sum(rho * acc[i]) for i in range(3)])
    assert np.all(np.abs(net) < 1e-10 * np.sum(np.abs(rho)) * np.abs(acc).max())


def test_point_mass_is_newtonian_for_gx():
    # a unit point mass: Phi at distance r (inside half the box) is the mean-free
    # -1/(4 pi r) + const; differences remove the constant
    N = 32
    rho = fields.point_sources(N, [(5, 5, 5)])
    phi = conv.pm(rho, "X")
    for (i, j) in [((5, 5, 9), (5, 5, 13)), ((8, 5, 5), (5, 14, 5))]:
        r1 = np.linalg.norm(np.subtract(i, (5, 5, 5))) / N
        r2 = np.linalg.norm(np.subtract(j, (5, 5, 5))) / N
        assert abs((phi[i] - phi[j]) - (-1 / (4 * np.pi * r1) + 1 / (4 * np.pi * r2))) < 1e-12


def test_fd4_single_mode_closed_form():
    # 4th-order stencil on exp(i theta j): derivative factor (8 sin t - sin 2t)/(6h)
    N = 16
    h = 1 / N
    x = (np.arange(N) + 0.5) / N
    for n in (1, 3, 7):
        phi = np.cos(2 * np.pi * n * x)[:, None, None] * np.ones((1, N, N))
        th = 2 * np.pi * n * h
        fac = (8 * np.sin(th) - np.sin(2 * th)) / (6 * h)
        a = fd.accel_fd4(phi)
        np.testing.assert_allclose(a[0], fac * np.sin(2 * np.pi * n * x)[:, None, None] * np.ones((1, N, N)),
                                   atol=1e-10 * fac)
        assert np.abs(a[1]).max() < 1e-10 and np.abs(a[2]).max() < 1e-10
