"""Pins of the step-by-step reference FMM (Sec. 2, Eqs. 5-7): exact special
cases, moment matching, index sets, symmetries, convergence with p."""
import itertools

import numpy as np
import pytest

from oracle import conv, fmm, green
from paper_2011_07099_amd import fields

KINDS = ("X", "S1", "K")


def _rho(N, seed):
    r = np.random.default_rng(seed).standard_normal((N, N, N))
    return r - r.mean()


def _lagrange(nodes, x):
    # textbook Lagrange basis l_a(x) = prod_{b != a} (x - t_b) / (t_a - t_b)
    out = np.ones((len(nodes), len(x)))
    for a, ta in enumerate(nodes):
        for b, tb in enumerate(nodes):
            if a != b:
                out[a] *= (x - tb) / (ta - tb)
    return out


@pytest.mark.parametrize("p", [1, 2, 4, 6, 8, 10])
def test_moment_matching_equals_lagrange(p):
    # the Vandermonde solution V^-1 W of Sec. 2 is polynomial interpolation's
    # Lagrange basis evaluated at the source points
    t = fmm.gridlet_coords(p)
    for s in (1, 2, 4, 8, 16):
        v = (np.arange(s) + 0.5 - s / 2) * (p / s)
        np.testing.assert_allclose(fmm.p2m_1d(p, s), _lagrange(t, v), atol=1e-10)
    T = fmm.m2m_1d(p)
    for o in (0, 1):
        u = (o - 0.5) * p / 2 + t / 2
        np.testing.assert_allclose(T[o], _lagrange(t, u), atol=1e-10)


@pytest.mark.parametrize("p", [2, 4, 8])
def test_m2m_preserves_moments(p):
    # Eq. 5: parent gridlet reproduces the moments 0 <= n_i <= p-1 of the two
    # child gridlets (coordinates about the parent centre, parent gridlet units)
    rng = np.random.default_rng(p)
    t = fmm.gridlet_coords(p)
    T = fmm.m2m_1d(p)
    child = rng.standard_normal((2, p))
    parent = T[0] @ child[0] + T[1] @ child[1]
    for n in range(p):
        lhs = np.sum(parent * t ** n)
        rhs = sum(np.sum(child[o] * ((o - 0.5) * p / 2 + t / 2) ** n) for o in (0, 1))
        assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(rhs)) * (p / 2) ** n


@pytest.mark.parametrize("p", [2, 4, 8])
def test_l2l_l2p_reproduce_polynomials(p):
    # Eq. 7 transpose = interpolation: exact for degree < p per axis
    t = fmm.gridlet_coords(p)
    T = fmm.m2m_1d(p)
    A = fmm.p2m_1d(p, 16)
    v = (np.arange(16) + 0.5 - 8) * (p / 16)
    for deg in range(p):
        f = lambda x: (0.3 * x + 0.7) ** deg
        for o in (0, 1):
            u = (o - 0.5) * p / 2 + t / 2
            np.testing.assert_allclose(T[o].T @ f(t), f(u), atol=1e-10 * max(1, np.abs(f(u)).max()))
        np.testing.assert_allclose(A.T @ f(t), f(v), atol=1e-10 * max(1, np.abs(f(v)).max()))


def test_index_set_counts():
    assert len(fmm.near_offsets()) == 27
    union = set()
    for c in itertools.product((0, 1), repeat=3):
        offs = fmm.interaction_offsets(c)
        assert len(offs) == 189 and len(set(offs)) == 189
        union |= set(offs)
    assert len(union) == 316
    assert len(fmm.level2_offsets()) == 37
    # the M2L table holds (4p)^3 distinct |j| values: 32768 at p = 8 (Sec. 4)
    p = 8
    js = set()
    for d in union:
        for a in range(-(p - 1), p):
            js.add(abs(p * d[0] + a))
    assert max(js) == 4 * p - 1 and (max(js) + 1) ** 3 == 32768


@pytest.mark.parametrize("L", [3, 4])
def test_every_source_counted_once(L):
    # near zone + interaction zones of the leaf and of every ancestor down to
    # level 2 cover each leaf of the box exactly once (Sec. 2 three-part sum)
    n = 2 ** L
    for b in [(0, 0, 0), (1, 2, 3), (n - 1, 5 % n, 2)]:
        cnt = np.zeros((n, n, n), int)
        for e in fmm.near_offsets():
            cnt[tuple((np.add(b, e)) % n)] += 1
        for l in range(L, 1, -1):
            shift = L - l
            bl = tuple(v >> shift for v in b)
            nl = 2 ** l
            offs = fmm.level2_offsets() if l == 2 else fmm.interaction_offsets(tuple(v % 2 for v in bl))
            for d in offs:
                src = tuple((np.add(bl, d)) % nl)
                # every leaf below that level-l node
                w = 2 ** shift
                cnt[src[0] * w:(src[0] + 1) * w, src[1] * w:(src[1] + 1) * w, src[2] * w:(src[2] + 1) * w] += 1
        assert np.all(cnt == 1)


@pytest.mark.parametrize("kind", KINDS)
def test_two_levels_with_gridlet_equal_to_leaf_is_exact(kind):
    # Sec. 3: "with just 2 levels the PM and FMM-HPM results are identical by
    # construction" — gridlet = leaf cells (s = p), near + level-2 zones cover all
    for N, p in [(8, 2), (16, 4)]:
        rho = _rho(N, 11)
        phi = fmm.fmm(rho, 2, p, kind)
        ref = conv.pm(rho, kind)
        np.testing.assert_allclose(phi, ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("kind", KINDS)
def test_near_and_leaf_zone_pairs_exact_when_gridlet_is_leaf(kind):
    # every source/target pair takes exactly one path; near-zone pairs are the
    # direct sum, and with s = p the leaf-level gridlet is the cells, so pairs in
    # the leaf's interaction zone are exact too.  Only coarser paths approximate.
    N, L, p = 32, 3, 4
    src = (5, 9, 30)
    rho = np.zeros((N, N, N))
    rho[src] = N ** 3      # unit mass, not mean-subtracted: linearity suffices
    phi = fmm.fmm(rho, L, p, kind)
    g = conv.lattice_table(kind, N)
    s = N >> L
    nL = 2 ** L
    bs = np.array(src) // s
    checked = 0
    for bt in itertools.product(range(nL), repeat=3):
        d = (np.array(bs) - np.array(bt) + nL // 2) % nL - nL // 2
        near = np.max(np.abs(d)) <= 1
        par = tuple(v % 2 for v in bt)
        izl = tuple(d) in set(fmm.interaction_offsets(par))
        if not (near or izl):
            continue
        for c in [(0, 0, 0), (3, 1, 2)]:
            t = np.array(bt) * s + np.array(c)
            expect = g[tuple((t - np.array(src)) % N)]
            assert abs(phi[tuple(t)] - expect) < 1e-11 * max(1, abs(expect))
            checked += 1
    assert checked == 2 * (27 + 189)


@pytest.mark.parametrize("kind", KINDS)
def test_reciprocity(kind):
    # K_{-d} = K_d^T, M2M/L2L and P2M/L2P are transposes: the FMM operator is
    # symmetric, <rho1, F rho2> = <rho2, F rho1>
    N, L, p = 32, 3, 4
    r1, r2 = _rho(N, 1), _rho(N, 2)
    a = np.sum(r1 * fmm.fmm(r2, L, p, kind))
    b = np.sum(r2 * fmm.fmm(r1, L, p, kind))
    assert abs(a - b) < 1e-12 * abs(a)


@pytest.mark.parametrize("kind", KINDS)
def test_shift_by_level2_node_and_cube_symmetries(kind):
    # the uniform periodic tree maps onto itself under shifts by a level-2 node
    # (N/4 cells) and under the 48 symmetries of the cube (G is symmetric)
    N, L, p = 32, 3, 4
    rho = _rho(N, 13)
    phi = fmm.fmm(rho, L, p, kind)
    tol = 1e-12 * np.abs(phi).max()
    for sh in [(N // 4, 0, 0), (0, N // 2, 3 * N // 4)]:
        np.testing.assert_allclose(fmm.fmm(np.roll(rho, sh, (0, 1, 2)), L, p, kind),
                                   np.roll(phi, sh, (0, 1, 2)), atol=tol)
    for perm in [(1, 0, 2), (2, 0, 1)]:
        np.testing.assert_allclose(fmm.fmm(np.transpose(rho, perm), L, p, kind),
                                   np.transpose(phi, perm), atol=tol)
    for ax in [(0,), (1, 2)]:
        np.testing.assert_allclose(fmm.fmm(np.flip(rho, ax), L, p, kind), np.flip(phi, ax), atol=tol)


def test_error_falls_with_p_for_gs1():
    # Fig. 5 / Sec. 4: the FMM-vs-PM difference with G_S1 falls with N_g
    N, L = 64, 3
    rho = fields.lognormal(N, 2.0, 1.0, seed=2)
    ref = conv.pm(rho, "S1")
    errs = []
    for p in (2, 4, 6, 8):
        d = fmm.fmm(rho, L, p, "S1") - ref
        errs.append(np.sqrt(np.sum(d ** 2) / np.sum(ref ** 2)))
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[-1] < 1e-4      # the 1e-4 L2 target at p = 8


def test_gx_aliasing_far_worse_than_gs1():
    # Figs. 3/4, Sec. 3: the kink of G_X at half the box makes the FMM-vs-PM
    # error ~2-3 orders of magnitude larger than with G_S1 (corner source)
    N, L, p = 64, 3, 8
    rho = fields.corner_source(N)
    e = {}
    for kind in ("X", "S1"):
        ref = conv.pm(rho, kind)
        d = fmm.fmm(rho, L, p, kind) - ref
        e[kind] = np.sqrt(np.sum(d ** 2) / np.sum(ref ** 2))
    assert e["X"] > 100 * e["S1"], e


@pytest.mark.parametrize("kind,N,L", (("S1", 32, 3), ("K", 32, 3), ("S1", 64, 4)))
def test_sampled_targets_match_full_grid(kind, N, L):
    # with targets the oracle sums the zones of the target leaves and their
    # ancestors only; the result at those cells must not change
    p = 4
    rho = _rho(N, 21)
    full = fmm.fmm(rho, L, p, kind)
    tg = np.random.default_rng(3).integers(0, N, (40, 3))
    np.testing.assert_allclose(fmm.fmm(rho, L, p, kind, targets=tg),
                               full[tg[:, 0], tg[:, 1], tg[:, 2]], atol=1e-13 * np.abs(full).max())
