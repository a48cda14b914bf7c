"""Seeded synthetic density fields shaped like the paper's workloads.

This module holds input generators only (no FMM arithmetic).  It serves the
tests, the benchmark and the smoke check, which hand the same FP64 array to the
CPU oracle and (cast to FP32) to the GPU library.

Workloads (all on the unit periodic box, N^3 cells, C order, x slowest):

* ``blobs``     — Gaussian blobs of width sigma centred uniformly in the box,
  masses U(0.5, 1.5), sampled at cell centres with the nearest periodic image,
  mean subtracted.
* ``lognormal`` — rho = exp(delta) - mean, delta a Gaussian random field with
  power spectrum P(k) ~ k^-alpha normalised to standard deviation sigma_delta.
* ``point_sources`` — unit-mass sources in single cells (the paper's corner
  source and random-source tests, Sec. 3), mean subtracted.
"""
import numpy as np


def blobs(N, n_blobs=32, sigma=0.03, seed=1):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, (n_blobs, 3))
    masses = rng.uniform(0.5, 1.5, n_blobs)
    x = (np.arange(N) + 0.5) / N
    rho = np.zeros((N, N, N))
    norm = (2.0 * np.pi * sigma ** 2) ** -1.5
    for c, m in zip(centres, masses):
        d = [x - c[i] for i in range(3)]
        d = [di - np.rint(di) for di in d]  # nearest periodic image
        r2 = d[0][:, None, None] ** 2 + d[1][None, :, None] ** 2 + d[2][None, None, :] ** 2
        rho += m * norm * np.exp(-r2 / (2.0 * sigma ** 2))
    return rho - rho.mean()


def gaussian_random_field(N, alpha, seed):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((N, N, N))
    n = np.fft.fftfreq(N, d=1.0 / N)
    k = np.sqrt(n[:, None, None] ** 2 + n[None, :, None] ** 2 + n[None, None, :] ** 2)
    amp = np.zeros_like(k)
    nz = k > 0
    amp[nz] = k[nz] ** (-0.5 * alpha)
    delta = np.real(np.fft.ifftn(np.fft.fftn(w) * amp))
    return delta / delta.std()


def lognormal(N, alpha=2.0, sigma_delta=1.0, seed=2):
    delta = sigma_delta * gaussian_random_field(N, alpha, seed)
    rho = np.exp(delta)
    return rho - rho.mean()


def point_sources(N, cells, masses=None):
    """Unit (or given) masses in the listed cells: density m / h^3 there."""
    rho = np.zeros((N, N, N))
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
    if masses is None:
        masses = np.ones(len(cells))
    for c, m in zip(cells, masses):
        rho[tuple(c)] += m * N ** 3
    return rho - rho.mean()


def corner_source(N):
    return point_sources(N, [(0, 0, 0)])


def random_sources(N, n=10, seed=7):
    rng = np.random.default_rng(seed)
    return point_sources(N, rng.integers(0, N, (n, 3)))


def batch_specs(n_fields=128, seed=4):
    """Mixed batch: N from {32, 64, 128}, p from {4, 6, 8}, sigma_delta ~
    U(0.5, 2), alpha = 2, per-field seed 1000 + i."""
    rng = np.random.default_rng(seed)
    Ns = rng.choice([32, 64, 128], n_fields)
    ps = rng.choice([4, 6, 8], n_fields)
    sig = rng.uniform(0.5, 2.0, n_fields)
    return [dict(N=int(N), p=int(p), sigma_delta=float(s), alpha=2.0, seed=1000 + i)
            for i, (N, p, s) in enumerate(zip(Ns, ps, sig))]
