"""Pins of the oracle's Ewald Green's function G_E (Sec. 1).

Ewald's identity: the real-space part on all images plus the damped Fourier
part is the zero-mean periodic Green's function minus r_S^2/4 (the integral of
-erfc(r/r_S)/(4 pi r) over space is -r_S^2/4), for every r_S.  With r_S << L
the images beyond the nearest are negligible, and with r_S >> h the mesh
truncation of the Fourier sum is, so G_E for two values of r_S differs by the
constant -(r_1^2 - r_2^2)/4 + 1/(2 pi^(3/2)) (1/r_1 - 1/r_2) at every lattice
separation, the zero separation included.  A wrong erfc argument, damping
exponent, sign or constant breaks this.
"""
import numpy as np

from oracle import conv
from oracle import green as og


def test_ewald_identity_between_two_splitting_radii():
    N = 64
    r1, r2 = 0.06, 0.09
    g1 = conv.lattice_table("E", N, (r1,))
    g2 = conv.lattice_table("E", N, (r2,))
    want = -(r1 ** 2 - r2 ** 2) / 4.0 + og.ewald_constant(r1) - og.ewald_constant(r2)
    d = g1 - g2
    assert np.max(np.abs(d - want)) < 1e-11 * np.max(np.abs(g1))
    assert abs(want) > 0.1  # the constant itself is checked, not only that d is flat


def test_ewald_near_field_is_newtonian_plus_smooth():
    # G_E + 1/(4 pi r) is smooth: its second differences along an axis at small
    # r are of order h^2 / r_S^3, far below those of -1/(4 pi r)
    N, rs = 64, 0.1
    h = 1.0 / N
    x = h * np.arange(1, 6)
    ge = og.green_product_grid("E", N, x, [0.0], [0.0], a=(rs,), h_self=h)[:, 0, 0]
    smooth = ge + 1.0 / (4 * np.pi * x)
    d2s = np.abs(np.diff(smooth, 2))
    d2n = np.abs(np.diff(-1.0 / (4 * np.pi * x), 2))
    assert np.all(d2s < 1e-2 * d2n)
