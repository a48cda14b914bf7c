"""Periodic Green's functions of the natively periodic FMM (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Box of side ``Lbox`` (default 1).  Separation vectors ``x`` are arrays of shape
(..., 3).  Conventions: G_0 = -1/(4 pi r) so that lap(Phi) = rho (Sec. 1,
continuum Green's function); the potential of cell masses m_j is
Phi_i = sum_j G(x_i - x_j) m_j.
"""
import numpy as np

FOUR_PI = 4.0 * np.pi


def wrap(x, Lbox=1.0):
    """Periodic coordinate wrap x <> L = x - L nint(x/L)  (Sec. 1, after Eq. 2).

    The tie |x| = L/2 is irrelevant: every G below depends on |x <> L| only.
    """
    x = np.asarray(x, dtype=np.float64)
    return x - Lbox * np.rint(x / Lbox)


def self_cell_constant():
    """c0 = integral over the unit cube [-1/2,1/2]^3 of d^3u/|u|.

    The paper leaves G(0) undefined for the real-space forms G_X / G_S1.  Reading
    adopted: the self term of a cell is the potential at the centre of a uniform
    cube of side h, G(0) = -c0 / (4 pi h).  Closed form of the cube integral:
    c0 = 3 ln((sqrt3+1)/(sqrt3-1)) - pi/2.
    """
    r3 = np.sqrt(3.0)
    return 3.0 * np.log((r3 + 1.0) / (r3 - 1.0)) - np.pi / 2.0


def self_value(h):
    """G(0) for the real-space Green's functions on a mesh of spacing h."""
    return -self_cell_constant() / (FOUR_PI * h)


def green_x(x, Lbox=1.0):
    """"Exact-in-real-space" G_X(x) = -1/(4 pi |x <> L|)  (Eq. 2, 3D: g(r)=1/r).

    Undefined at x = 0 (callers substitute ``self_value``); returns -inf there.
    """
    w = wrap(x, Lbox)
    r = np.sqrt(np.sum(w * w, axis=-1))
    with np.errstate(divide="ignore"):
        return -1.0 / (FOUR_PI * r)


def xi(t, a=(-0.125,)):
    """Ansatz map xi_n(t) of Sec. 3 (the G_S approximation of G_*):

    xi_n(t) = sin(pi t)/pi + sum_k a_k ( sin((2k+1) pi t)/((2k+1) pi) - sin(pi t)/pi ).

    ``a`` holds a_1..a_n; the default a_1 = -1/8 is the G_S1 choice.
    """
    t = np.asarray(t, dtype=np.float64)
    base = np.sin(np.pi * t) / np.pi
    out = base.copy()
    for k, ak in enumerate(a, start=1):
        m = 2 * k + 1
        out = out + ak * (np.sin(m * np.pi * t) / (m * np.pi) - base)
    return out


def green_s(x, a=(-0.125,), Lbox=1.0):
    """Approximately optimal G_S(x) = -1/(4 pi |x_hat <> L|), x_hat = L xi_n(x/L)
    applied to each component (Sec. 3 ansatz).  With a = (-1/8,) this is G_S1."""
    x = np.asarray(x, dtype=np.float64)
    xh = Lbox * xi(x / Lbox, a)
    w = wrap(xh, Lbox)
    r = np.sqrt(np.sum(w * w, axis=-1))
    with np.errstate(divide="ignore"):
        return -1.0 / (FOUR_PI * r)


def green_s1(x, Lbox=1.0):
    """G_S1 in the closed form of Eq. 9:
    x_hat = (9L/(8 pi)) sin(pi x/L) - (L/(24 pi)) sin(3 pi x/L), per component."""
    x = np.asarray(x, dtype=np.float64)
    xh = (9.0 * Lbox / (8.0 * np.pi)) * np.sin(np.pi * x / Lbox) \
        - (Lbox / (24.0 * np.pi)) * np.sin(3.0 * np.pi * x / Lbox)
    w = wrap(xh, Lbox)
    r = np.sqrt(np.sum(w * w, axis=-1))
    with np.errstate(divide="ignore"):
        return -1.0 / (FOUR_PI * r)


def gk_fourier(N, Lbox=1.0):
    """Fourier-space G_K on the N^3 frequency grid in FFT order  (Eq. 1):
    G~_K(k) = -1/k^2 for k != 0, 0 at k = 0, with k = 2 pi n / L."""
    n = np.fft.fftfreq(N, d=1.0 / N)
    k2 = (2.0 * np.pi / Lbox) ** 2 * (n[:, None, None] ** 2 + n[None, :, None] ** 2
                                       + n[None, None, :] ** 2)
    g = np.zeros_like(k2)
    nz = k2 > 0
    g[nz] = -1.0 / k2[nz]
    return g


def gk_lattice(N, Lbox=1.0):
    """"Exact-in-Fourier-space" G_K at the lattice separations x = j L/N
    (Eq. 1 and the inverse transform below it):
    G_K(x_j) = (1/L^3) sum_k G~_K(k) exp(i k.x_j), returned as an N^3 array
    indexed by j mod N (FFT order).  Uses numpy's inverse FFT as the sum."""
    gt = gk_fourier(N, Lbox)
    return np.real(np.fft.ifftn(gt)) * N ** 3 / Lbox ** 3


def gk_series(N, cx, cy, cz, Lbox=1.0, rs=None):
    """G_K evaluated off the lattice on the product grid cx x cy x cz.

    The paper defines G_K only through its Fourier coefficients on the
    n_i in [-N/2+1, N/2] grid (Eq. 1).  Reading adopted for off-lattice points
    (needed when the gridlet spacing does not divide the cell grid): the real,
    even trigonometric interpolant that splits the Nyquist term equally between
    n_i = +N/2 and -N/2,
        G(x) = (1/L^3) sum_{n_i in [-N/2, N/2]} w(n) G~_K(n) prod_i cos(2 pi n_i x_i / L),
    w(n) = prod_i (1/2 if |n_i| = N/2 else 1).  At lattice points it equals the
    paper's sum.  The three 1D cosine factors are contracted one axis at a time.
    With ``rs`` the coefficients carry the Ewald damping exp(-k^2 rs^2 / 4)
    (the Fourier part of G_E).
    """
    n = np.arange(-(N // 2), N // 2 + 1)
    w1 = np.where(np.abs(n) == N // 2, 0.5, 1.0)
    k2 = (2.0 * np.pi / Lbox) ** 2 * (n[:, None, None] ** 2 + n[None, :, None] ** 2
                                       + n[None, None, :] ** 2)
    gt = np.zeros_like(k2)
    nz = k2 > 0
    gt[nz] = -1.0 / k2[nz]
    if rs is not None:
        gt *= np.exp(-k2 * rs * rs / 4.0)
    gt *= w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
    Cx = np.cos(2.0 * np.pi * np.outer(n, np.asarray(cx, np.float64)) / Lbox)
    Cy = np.cos(2.0 * np.pi * np.outer(n, np.asarray(cy, np.float64)) / Lbox)
    Cz = np.cos(2.0 * np.pi * np.outer(n, np.asarray(cz, np.float64)) / Lbox)
    t = np.tensordot(gt, Cz, axes=([2], [0]))          # [nx, ny, z]
    t = np.tensordot(t, Cy, axes=([1], [0]))           # [nx, z, y]
    t = np.tensordot(t, Cx, axes=([0], [0]))           # [z, y, x]
    return np.transpose(t, (2, 1, 0)) / Lbox ** 3


def ewald_constant(rs):
    """The constant 1/(2 pi^(3/2) r_S) of G_E."""
    return 1.0 / (2.0 * np.pi ** 1.5 * rs)


def green_e(N, cx, cy, cz, rs, h_self=None, Lbox=1.0):
    """Ewald G_E on the product grid cx x cy x cz (Sec. 1):
        G_E(x) = G_X(x) erfc(r / r_S) + 1/(2 pi^(3/2) r_S) + F^-1[G~_K(k) exp(-k^2 r_S^2 / 4)],
    with the Fourier part over the mesh frequencies as for G_K (Eq. 1; reading
    of ``gk_series`` between mesh points) and the real-space part on the
    nearest image (r_S << L: the other images are negligible).

    Zero separation (reading, as for the real-space kinds): the Newtonian
    -1/(4 pi r) inside G_X erfc is replaced by the self-cell value; what is
    left of G_X erfc there is its limit erf(r/r_S)/(4 pi r) -> 1/(2 pi^(3/2) r_S).
    NaN there when ``h_self`` is None."""
    from scipy.special import erfc
    cx = np.asarray(cx, np.float64)
    cy = np.asarray(cy, np.float64)
    cz = np.asarray(cz, np.float64)
    X = np.stack(np.meshgrid(cx, cy, cz, indexing="ij"), axis=-1)
    w = wrap(X, Lbox)
    r = np.sqrt(np.sum(w * w, axis=-1))
    c = ewald_constant(rs)
    zero = r == 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        real = -erfc(r / rs) / (FOUR_PI * r)
    real[zero] = (np.nan if h_self is None else self_value(h_self)) + c
    return real + c + gk_series(N, cx, cy, cz, Lbox, rs=rs)


GREEN_KINDS = ("X", "K", "S1", "S", "E")


def green_newton(x):
    """Free-space G_0(x) = -1/(4 pi |x|), no periodic images: the Green's
    function of the non-periodic twin used to separate the multipole-expansion
    error from the Green's-function error (Sec. 3, Eq. 3).  Undefined at 0."""
    x = np.asarray(x, dtype=np.float64)
    r = np.sqrt(np.sum(x * x, axis=-1))
    with np.errstate(divide="ignore"):
        return -1.0 / (FOUR_PI * r)


def green_product_grid(kind, N, cx, cy, cz, a=(-0.125,), h_self=None):
    """G of kind ``kind`` on the product grid of separation coordinates
    cx x cy x cz (box units, L = 1).  Points with x = 0 exactly get the self-cell
    value for the real-space kinds (``h_self`` = mesh spacing, required then);
    for G_K the zero separation is the series value itself (Eq. 1).  ``a``
    holds the kind's parameters: a_1.. for "S", (r_S,) for "E"."""
    cx = np.asarray(cx, np.float64)
    cy = np.asarray(cy, np.float64)
    cz = np.asarray(cz, np.float64)
    if kind == "K":
        return gk_series(N, cx, cy, cz)
    if kind == "E":
        return green_e(N, cx, cy, cz, a[0], h_self)
    X = np.stack(np.meshgrid(cx, cy, cz, indexing="ij"), axis=-1)
    if kind == "X":
        g = green_x(X)
    elif kind == "N":
        g = green_newton(X)
    elif kind == "S1":
        g = green_s1(X)
    elif kind == "S":
        g = green_s(X, a)
    else:
        raise ValueError(kind)
    zero = np.all(X == 0.0, axis=-1)
    if np.any(zero):
        # without a mesh spacing the zero separation has no value: NaN, so that
        # any use of it shows up in the result
        g[zero] = np.nan if h_self is None else self_value(h_self)
    return g
