"""Pin of the spectral reading of the interaction zones (Eq. 6), which the
library's spectral stencils implement.

Node t receives from node t + d through K_d[a, a'] = G(eta_l (a - a' - p d)),
a convolution of the source gridlet with a kernel slice whose in-gridlet
separations satisfy |a_i - a'_i| <= p - 1.  On a cyclic grid of 2p points per
axis those separations keep distinct residues, so every per-pair sum is exact
there, and a zone's offsets add per frequency.  Checked in plain NumPy FFTs
against the direct zone sum written from the oracle's Toeplitz blocks, at
levels 2 (periodic and isolated zones) and 3 (189 offsets per parity class),
and a counter-example with 2p - 2 points.
"""
import numpy as np
import pytest

from oracle import fmm as ofmm


def _direct_zone(M, tab, J, p, n, offsets_of, periodic):
    """sum_d K_d M[t + d] per target, K_d from the oracle's Toeplitz block."""
    out = np.zeros((n, n, n, p ** 3))
    Mf = M.reshape(n, n, n, p ** 3)
    for t in np.ndindex(n, n, n):
        for d in offsets_of(t):
            s = np.asarray(t) + np.asarray(d)
            if periodic:
                s %= n
            elif np.any(s < 0) or np.any(s >= n):
                continue
            out[t] += ofmm._toeplitz_block(tab, J, p, np.asarray(d)) @ Mf[tuple(s)]
    return out


def _spectral_zone(M, tab, J, p, n, offsets_of, periodic, G=None):
    """The same sums by per-node transforms on G = 2p points per axis."""
    G = 2 * p if G is None else G
    pad = np.zeros((n, n, n, G, G, G))
    pad[..., :p, :p, :p] = M
    spec = np.fft.fftn(pad, axes=(3, 4, 5))
    w = np.arange(G)
    w = np.where(w < G // 2, w, w - G)
    ok = np.abs(w) < p
    kernels = {}
    out = np.zeros_like(spec)
    for t in np.ndindex(n, n, n):
        for d in offsets_of(t):
            s = np.asarray(t) + np.asarray(d)
            if periodic:
                s %= n
            elif np.any(s < 0) or np.any(s >= n):
                continue
            if d not in kernels:
                K = np.zeros((G, G, G))
                jx, jy, jz = (w[ok] - p * d[0] + J, w[ok] - p * d[1] + J, w[ok] - p * d[2] + J)
                K[np.ix_(ok, ok, ok)] = tab[np.ix_(jx, jy, jz)]
                kernels[d] = np.fft.fftn(K)
            out[t] += kernels[d] * spec[tuple(s)]
    y = np.real(np.fft.ifftn(out, axes=(3, 4, 5)))[..., :p, :p, :p]
    return y.reshape(n, n, n, p ** 3)


@pytest.mark.parametrize("level,p,kind,periodic", [
    (2, 3, "S1", True), (2, 4, "N", False), (3, 2, "S1", True), (3, 3, "X", True),
])
def test_spectral_zone_sums_equal_the_direct_ones(level, p, kind, periodic):
    n = 2 ** level
    N = n * p
    rng = np.random.default_rng(level * 10 + p)
    M = rng.standard_normal((n, n, n, p, p, p))
    tab, J = ofmm.m2l_table(kind, N, level, p)
    if level == 2:
        zone = ofmm.level2_offsets() if periodic else ofmm.level2_offsets_isolated()
        offsets_of = lambda t: zone
    else:
        zones = {c: ofmm.interaction_offsets(c) for c in np.ndindex(2, 2, 2)}
        offsets_of = lambda t: zones[tuple(int(v) % 2 for v in t)]
    ref = _direct_zone(M, tab, J, p, n, offsets_of, periodic)
    got = _spectral_zone(M, tab, J, p, n, offsets_of, periodic)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_fewer_than_2p_points_alias():
    level, p = 2, 4
    n = 4
    M = np.random.default_rng(3).standard_normal((n, n, n, p, p, p))
    tab, J = ofmm.m2l_table("S1", n * p, level, p)
    zone = ofmm.level2_offsets()
    ref = _direct_zone(M, tab, J, p, n, lambda t: zone, True)
    short = _spectral_zone(M, tab, J, p, n, lambda t: zone, True, G=2 * p - 2)
    assert np.max(np.abs(short - ref)) > 1e-3 * np.max(np.abs(ref))
