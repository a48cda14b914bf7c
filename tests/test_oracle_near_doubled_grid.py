"""Pin of the doubled-grid reading of the near zone (Sec. 2: a leaf's near zone
by a PM solver with non-periodic boundaries; Sec. 3: grid doubling), which
the FFT near zone of the library implements.

For a target leaf b and a neighbour b + e, the near-zone contribution is a
linear convolution of the neighbour's s^3 cells with G(h (m - s e)), m the
in-leaf separation, |m_i| <= s - 1.  On a cyclic grid of 2s points every such
m has its own residue, so the cyclic convolution of the zero-padded leaf,
restricted to the target cells, is the linear sum exactly, and the 27
neighbours add in Fourier space.  Checked here in plain NumPy FFTs against
the oracle's direct near-zone sum, periodic and isolated, for leaf edges
1 .. 8 and three G; and a counter-example: on a cyclic grid of 2s - 2 points
two separations share a residue and the identity fails.
"""
import numpy as np
import pytest

from oracle import fmm as ofmm


def _doubled_grid_near(rho, s, tab, J, periodic, M=None):
    """Near zone of every cell by cyclic convolutions on M = 2s points per axis
    (per leaf pair), added per frequency over the 27 neighbours."""
    N = rho.shape[0]
    nb = N // s
    M = 2 * s if M is None else M
    h3 = 1.0 / N ** 3
    blocks = rho.reshape(nb, s, nb, s, nb, s).transpose(0, 2, 4, 1, 3, 5) * h3
    pad = np.zeros((nb, nb, nb, M, M, M))
    pad[:, :, :, :s, :s, :s] = blocks
    spec = np.fft.fftn(pad, axes=(3, 4, 5))
    w = np.arange(M)
    w = np.where(w < M // 2, w, w - M)                 # signed cyclic separation
    out = np.zeros_like(spec)
    for e in ofmm.near_offsets():
        K = np.zeros((M, M, M))
        jx, jy, jz = (w - s * e[0], w - s * e[1], w - s * e[2])
        okx, oky, okz = (np.abs(w) < s,) * 3
        sel = np.ix_(okx, oky, okz)
        K[sel] = tab[np.ix_(jx[okx] + J, jy[oky] + J, jz[okz] + J)]
        Kh = np.fft.fftn(K)
        src = np.zeros_like(spec)
        for bx in range(nb):
            for by in range(nb):
                for bz in range(nb):
                    t = np.array([bx, by, bz]) + np.asarray(e)
                    if periodic:
                        t %= nb
                    elif np.any(t < 0) or np.any(t >= nb):
                        continue
                    src[bx, by, bz] = spec[tuple(t)]
        out += Kh * src
    y = np.real(np.fft.ifftn(out, axes=(3, 4, 5)))[:, :, :, :s, :s, :s]
    return y


def _direct(rho, s, tab, J, periodic):
    N = rho.shape[0]
    nb = N // s
    mb = rho.reshape(nb, s, nb, s, nb, s).transpose(0, 2, 4, 1, 3, 5) / N ** 3
    return ofmm._near_sum(tab, J, mb, periodic)


@pytest.mark.parametrize("N,s,kind,periodic", [
    (8, 2, "S1", True), (16, 4, "S1", True), (16, 4, "N", False), (8, 1, "X", True),
    (16, 8, "K", True), (16, 2, "N", False),
])
def test_cyclic_convolution_on_2s_points_is_the_near_zone(N, s, kind, periodic):
    rho = np.random.default_rng(N + s).standard_normal((N, N, N))
    tab, J = ofmm.near_table(kind, N, s)
    got = _doubled_grid_near(rho, s, tab, J, periodic)
    ref = _direct(rho, s, tab, J, periodic)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_fewer_than_2s_points_alias():
    N, s = 16, 4
    rho = np.random.default_rng(5).standard_normal((N, N, N))
    tab, J = ofmm.near_table("S1", N, s)
    ref = _direct(rho, s, tab, J, True)
    short = _doubled_grid_near(rho, s, tab, J, True, M=2 * s - 2)
    assert np.max(np.abs(short - ref)) > 1e-3 * np.max(np.abs(ref))
