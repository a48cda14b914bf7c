"""The paper's error metric for the Green's function (Sec. 3, Eq. 3) (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Eq. 3 measures the error due to the choice of G as the absolute difference of
two acceleration errors: FMM minus PM in the periodic box, less FMM minus PM in
the non-periodic twin (the latter estimates the multipole-expansion error).
PM accelerations are 4th-order central differences of the PM potential.
Norms: L2 = root mean square of |Delta g| over the cells, L_MAX = its maximum
(absolute errors, unit box, G M = 1; Sec. 3).

Reading adopted for the twin of a periodic test with point sources (the paper
does not say where the twin's sources sit): the twin holds the same sources
translated by half the box along every axis (so that no source touches a face
and every target sees its nearest source through the same leaves and zones as
in the periodic run: N/2 is a multiple of every node width at levels >= 2), and
its error field is translated back by the same amount before it is subtracted.
With the sources left at the same cells instead, targets next to a periodic
image of a source have no counterpart in the twin, their expansion error stays
in Delta g, and Delta g of the corner source comes out an order of magnitude
above the values the paper tabulates.
"""
import itertools

import numpy as np

from . import green as _g


def point_sources_accel(N, cells, masses, kind="S1", a=(-0.125,), periodic=True, shift=0):
    """PM accelerations of point masses: g = -D4 Phi, Phi = sum_k m_k G(x - x_k),
    D4 the 4th-order central difference (Sec. 3).  Differencing a sum of
    shifted G is the sum of the differenced G, so each source contributes
        -(8 (G(r + h e_i) - G(r - h e_i)) - (G(r + 2h e_i) - G(r - 2h e_i))) / (12 h)
    with r the lattice separation (periodically wrapped for the periodic
    kinds; G_0 of the free-space twin with ``periodic=False``, evaluated past
    the box faces as the free-space potential).  The self cell takes the
    self-cell value of G.  ``shift`` translates every source by that many
    cells along each axis (wrapped into the box).  Returns (3, N, N, N)."""
    h = 1.0 / N
    cells = (np.asarray(cells, np.int64).reshape(-1, 3) + shift) % N
    out = np.zeros((3, N, N, N))
    for c, m in zip(cells, np.asarray(masses, np.float64).reshape(-1)):
        coords = []
        for ax in range(3):
            j = np.arange(-2, N + 2) - c[ax]
            if periodic:
                j = (j + N // 2) % N - N // 2            # nearest image
            coords.append(h * j)
        G = _g.green_product_grid(kind if periodic else "N", N, coords[0], coords[1], coords[2],
                                  a=a, h_self=h)
        for ax in range(3):
            def sh(k):
                return tuple(slice(2 + k, 2 + k + N) if i == ax else slice(2, 2 + N)
                             for i in range(3))
            out[ax] -= m * (8.0 * (G[sh(1)] - G[sh(-1)]) - (G[sh(2)] - G[sh(-2)])) / (12.0 * h)
    return out


def twin_shift(N):
    """Translation (cells per axis) of the non-periodic twin's sources: N/2."""
    return N // 2


def delta_g(err_periodic, err_twin):
    """|Delta g| of Eq. 3 per cell from the two acceleration errors (3, N, N, N):
    err_periodic = g_FMM^P - g_PM^P, err_twin = g_FMM^NP - g_PM^NP, the latter
    already translated back onto the periodic run's cells."""
    d = np.asarray(err_periodic, np.float64) - np.asarray(err_twin, np.float64)
    return np.sqrt(np.sum(d * d, axis=0))


def untranslate(field, shift):
    """Translate a (3, N, N, N) field computed with sources moved by ``shift``
    back onto the original cells."""
    return np.roll(field, (-shift, -shift, -shift), axis=(1, 2, 3))


def norms(dg):
    """(L2, L_MAX) of a per-cell error magnitude: root mean square and maximum."""
    dg = np.asarray(dg, np.float64)
    return float(np.sqrt(np.mean(dg * dg))), float(np.max(dg))


def periodic_point_accel(N, cell=(0, 0, 0), alpha=0.1, images=1):
    """Exact acceleration of a unit point mass at the centre of ``cell`` in the
    periodic unit box, with the uniform background that makes the mean density
    zero (the periodic Poisson problem the FMM solves), at every cell centre:
    Ewald's split of -1/(4 pi r) summed over all images,
        g = -grad[ sum_n -erfc(|x + n|/alpha) / (4 pi |x + n|) ]
            - grad[ sum_{k != 0} -exp(-k^2 alpha^2 / 4) / k^2 cos(k . x) ],
    the real-space sum over the (2 images + 1)^3 nearest images (alpha << 1
    makes the rest negligible), the Fourier sum by an inverse FFT over the
    mesh frequencies (exp(-k^2 alpha^2 / 4) is negligible beyond them for
    alpha >> 1/N).  NaN at the source cell.  Returns (3, N, N, N).
    This is the Newtonian force of the periodic problem, the reference for the
    deviation of the FMM's force from the Newtonian form (Sec. 3, Fig. 6)."""
    from scipy.special import erfc
    h = 1.0 / N
    j = np.arange(N)
    out = np.zeros((3, N, N, N))
    X = [((j - c + N // 2) % N - N // 2) * h for c in cell]   # nearest-image displacement
    x3 = np.stack(np.meshgrid(*X, indexing="ij"))
    for n in itertools.product(range(-images, images + 1), repeat=3):
        y = x3 + np.asarray(n, np.float64)[:, None, None, None]
        r = np.sqrt(np.sum(y * y, axis=0))
        with np.errstate(divide="ignore", invalid="ignore"):
            dphi = erfc(r / alpha) / (4 * np.pi * r * r) \
                + np.exp(-(r / alpha) ** 2) / (2 * np.pi ** 1.5 * alpha * r)
            out -= dphi * y / r
    f = np.fft.fftfreq(N, d=1.0 / N)
    kx, ky, kz = np.meshgrid(2 * np.pi * f, 2 * np.pi * f, 2 * np.pi * f, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    c = np.zeros_like(k2)
    nz = k2 > 0
    c[nz] = -np.exp(-k2[nz] * alpha * alpha / 4.0) / k2[nz]
    phase = np.exp(-1j * 2 * np.pi * (f[:, None, None] * cell[0] + f[None, :, None] * cell[1]
                                      + f[None, None, :] * cell[2]) / N)
    for ax, k in enumerate((kx, ky, kz)):
        # -grad of sum c cos(k.(x - x_s)) = sum c k sin(k.(x - x_s)), as a DFT
        out[ax] += np.real(np.fft.ifftn(-1j * k * c * phase)) * N ** 3
    out[:, cell[0], cell[1], cell[2]] = np.nan
    return out
