"""The exact result the natively periodic FMM approximates (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Unit box, N^3 cells of side h = 1/N, cell centres x_i = (i + 1/2) h, cell masses
m_j = rho_j h^3.  "PM with G" (Eq. 4 and the definition of G_* in Sec. 3) is the
periodic convolution

    Phi_i = h^3 sum_j G((x_i - x_j) <> 1) rho_j ,

with one Green's function G used everywhere.  It is computed here three
independent ways: ``brute`` (G from its formula for every pair), ``direct``
(lattice table + explicit sum over sources) and ``fft`` (convolution theorem).
``pm_gk`` is the standard PM solve with G~_K (Sec. 1, Eq. 1).
"""
import numpy as np

from . import green as _g


def lattice_table(kind, N, a=(-0.125,)):
    """g[j] = G(h j <> 1) for j in [0, N)^3 (FFT order: index j stands for the
    separation j mod N), with the self value at j = 0 for real-space kinds
    (Eq. 2 / Eq. 9 with the cube self term; Eq. 1 for G_K)."""
    h = 1.0 / N
    if kind == "K":
        return _g.gk_lattice(N)
    j = np.arange(N)
    js = np.where(j < N // 2, j, j - N) * h  # representative in [-1/2, 1/2)
    return _g.green_product_grid(kind, N, js, js, js, a=a, h_self=h)


def direct(rho, g, targets=None):
    """Direct periodic convolution Phi_i = h^3 sum_j g[(i - j) mod N] rho_j
    (Eq. 4 written out as a sum over source cells).

    ``targets``: optional integer array (T, 3) of target cells; default = all.
    Cost O(T N^3).
    """
    rho = np.asarray(rho, np.float64)
    N = rho.shape[0]
    h3 = (1.0 / N) ** 3
    if targets is None:
        idx = np.indices((N, N, N)).reshape(3, -1).T
    else:
        idx = np.asarray(targets, dtype=np.int64).reshape(-1, 3)
    j = np.arange(N)
    out = np.empty(len(idx))
    for t, (ix, iy, iz) in enumerate(idx):
        # g[(i - j) mod N] over all sources j, as an N^3 array indexed by j
        sx = (ix - j) % N
        sy = (iy - j) % N
        sz = (iz - j) % N
        gij = g[sx[:, None, None], sy[None, :, None], sz[None, None, :]]
        out[t] = h3 * np.sum(gij * rho)
    if targets is None:
        return out.reshape(N, N, N)
    return out


def brute(rho, kind, a=(-0.125,)):
    """Pairwise brute force: for every (target, source) pair evaluate G from
    its closed form at the wrapped separation (Eqs. 1, 2, 9; G_K by its cosine
    series).  O(N^6) formula evaluations — tiny boxes only."""
    rho = np.asarray(rho, np.float64)
    N = rho.shape[0]
    h = 1.0 / N
    cells = (np.indices((N, N, N)).reshape(3, -1).T + 0.5) * h
    out = np.zeros(N ** 3)
    rflat = rho.reshape(-1)
    if kind == "K":
        n1 = np.arange(-N // 2 + 1, N // 2 + 1)
        nvec = np.stack(np.meshgrid(n1, n1, n1, indexing="ij"), -1).reshape(-1, 3)
        nvec = nvec[np.any(nvec != 0, axis=1)].astype(np.float64)
        coef = -1.0 / (4.0 * np.pi ** 2 * np.sum(nvec ** 2, axis=1))
    for t in range(N ** 3):
        sep = cells[t][None, :] - cells  # x_i - x_j
        if kind == "K":
            # G_K(x) = sum_{n != 0} -exp(2 pi i n.x)/(4 pi^2 |n|^2) over the
            # paper's n_i in [-N/2+1, N/2] (Eq. 1), summed for every pair
            vals = np.real(np.exp(2j * np.pi * (sep @ nvec.T)) @ coef)
        else:
            if kind == "X":
                vals = _g.green_x(sep)
            elif kind == "S1":
                vals = _g.green_s1(sep)
            else:
                vals = _g.green_s(sep, a)
            vals[t] = _g.self_value(h)
        out[t] = h ** 3 * np.dot(vals, rflat)
    return out.reshape(N, N, N)


def fft(rho, g):
    """Phi = h^3 IFFT(FFT(g) FFT(rho)) — the convolution theorem applied to the
    same periodic sum as ``direct`` (PM with G, Eq. 4)."""
    rho = np.asarray(rho, np.float64)
    N = rho.shape[0]
    return np.real(np.fft.ifftn(np.fft.fftn(g) * np.fft.fftn(rho))) / N ** 3


def pm_gk(rho):
    """Standard PM solve with the exact-in-Fourier-space G_K  (Sec. 1, Eq. 1):
    Phi = IFFT( G~_K(k) FFT(rho) ), G~_K(0) = 0."""
    rho = np.asarray(rho, np.float64)
    N = rho.shape[0]
    return np.real(np.fft.ifftn(_g.gk_fourier(N) * np.fft.fftn(rho)))


def pm(rho, kind, a=(-0.125,)):
    """PM with the chosen G (Eq. 4): FFT convolution with the lattice table."""
    return fft(rho, lattice_table(kind, rho.shape[0], a))


# ---------------------------------------------------------------------------
# the isolated (non-periodic) twin: Sec. 3, Eq. 3
# ---------------------------------------------------------------------------

def isolated(rho):
    """Non-periodic convolution with the free-space G_0 over the box only,
    Phi_i = h^3 sum_j G_0(x_i - x_j) rho_j (self value at i = j): the
    "non-periodic PM" of Eq. 3, by the convolution theorem on the zero-padded
    2N grid (separations -(N-1)..N-1 fit without wrap)."""
    rho = np.asarray(rho, np.float64)
    N = rho.shape[0]
    h = 1.0 / N
    j = np.arange(2 * N)
    js = np.where(j < N, j, j - 2 * N) * h
    g = _g.green_product_grid("N", N, js, js, js, h_self=h)
    g[N, :, :] = 0.0  # separation N never occurs; keep the table finite
    g[:, N, :] = 0.0
    g[:, :, N] = 0.0
    pad = np.zeros((2 * N,) * 3)
    pad[:N, :N, :N] = rho
    out = np.real(np.fft.ifftn(np.fft.fftn(g) * np.fft.fftn(pad)))[:N, :N, :N]
    return out * h ** 3


def isolated_brute(rho):
    """The same sum with G_0 evaluated from its formula for every pair (small
    boxes only)."""
    rho = np.asarray(rho, np.float64)
    N = rho.shape[0]
    h = 1.0 / N
    x = (np.indices((N, N, N)).reshape(3, -1).T + 0.5) * h
    d = x[:, None, :] - x[None, :, :]
    g = _g.green_newton(d)
    np.fill_diagonal(g, _g.self_value(h))
    return (h ** 3 * (g @ rho.ravel())).reshape(N, N, N)
