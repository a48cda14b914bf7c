"""Step-by-step FP64 reference of the natively periodic FMM (CPU, NumPy).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Geometry (Sec. 2; readings listed in the design notes):
* unit periodic box, N^3 cells of side h = 1/N; uniform oct-tree with levels
  l = 2..L, 2^l nodes per dimension at level l, node width w_l = 2^-l; leaves at
  level L hold s = N / 2^L cells per dimension;
* every node carries a "gridlet": p^3 effective masses on a uniform,
  cell-centred mini-mesh of spacing eta_l = w_l / p covering the node
  (p is the paper's N_g); 1D gridlet coordinates about the node centre, in units
  of eta_l, are t_a = a + 1/2 - p/2;
* Phi(target) = near zone (27 nodes, direct sum) + interaction zone of the leaf
  + the parent's local field, recursively down to level 2 (Sec. 2, three-part sum).

Steps (in the paper's order):
* P2M  — gridlet masses whose Cartesian moments Q_n, 0 <= n_i <= p-1, match
  those of the leaf's cell masses (Sec. 2, the Vandermonde system for M_p);
* M2M  — Eq. 5, M^{l} = T^{C_S} M^{l+1}, with T fixed by the same moment
  matching between the child gridlet and the parent gridlet;
* M2L  — Eq. 6, Phi_r = sum_s G(d + eta (r - s)) M_s over the interaction zone;
  at level 2 the zone is every non-neighbour node of the periodic 4^3 level;
* L2L  — Eq. 7, Phi^{l+1} = T^T Phi^{l};  L2P is the same transpose of P2M;
* near — direct sum over the 27 neighbour leaves with the lattice G.
"""
import itertools

import numpy as np

from . import green as _g


# ---------------------------------------------------------------------------
# gridlet geometry and the moment-matching operators
# ---------------------------------------------------------------------------

def gridlet_coords(p):
    """Uniform cell-centred mini-mesh covering a node: t_a = a + 1/2 - p/2,
    a = 0..p-1, in units of the gridlet spacing (Sec. 2, effective masses on
    "the uniform mini-mesh covering the FMM node")."""
    return np.arange(p, dtype=np.float64) + 0.5 - 0.5 * p


def moment_matching_weights(p, src):
    """Weights W[a, c] such that gridlet masses M_a = sum_c W[a, c] m_c have the
    same 1D moments sum M_a t_a^n = sum_c m_c src_c^n for n = 0..p-1.

    This is the paper's Vandermonde system (Sec. 2: Q_n = (1/n!) sum_p M_p r_p^n,
    the 1/n! cancelling on both sides) solved directly, one dimension at a time
    (the moment set 0 <= n_i <= p-1 is a tensor product).  ``src`` are the source
    coordinates in gridlet units about the same centre.  Coordinates are scaled
    by the gridlet half-width before forming powers; the solution of the system
    does not depend on that scale.
    """
    t = gridlet_coords(p)
    scale = max(0.5 * p, 1.0)
    n = np.arange(p)
    V = (t[None, :] / scale) ** n[:, None]           # V[n, a] = t_a^n
    S = (np.asarray(src, np.float64)[None, :] / scale) ** n[:, None]  # S[n, c]
    return np.linalg.solve(V, S)                     # W = V^-1 S, shape (p, len(src))


def p2m_1d(p, s):
    """1D P2M operator A[a, c]: leaf cell centres v_c = (c + 1/2 - s/2) (p/s)
    in gridlet units (cells of width h = eta_L p / s) onto the leaf gridlet."""
    v = (np.arange(s, dtype=np.float64) + 0.5 - 0.5 * s) * (p / s)
    return moment_matching_weights(p, v)


def interpolant_derivative_weights(p, v):
    """Derivative of the gridlet interpolation weights: D[a, c] = d/dv of the
    weight of gridlet point a at v = v_c (gridlet units).

    The weights of ``moment_matching_weights`` reproduce every power v^n,
    n < p (sum_a W[a, c] t_a^n = v_c^n), so they are the values of the
    degree p-1 Lagrange basis polynomials at v_c; differentiating the moment
    conditions in v_c gives sum_a D[a, c] t_a^n = n v_c^(n-1), solved with the
    same Vandermonde matrix.  This is the gradient of the local expansion that
    L2P evaluates (Sec. 3: FMM accelerations come from the expansion)."""
    t = gridlet_coords(p)
    scale = max(0.5 * p, 1.0)
    n = np.arange(p)
    V = (t[None, :] / scale) ** n[:, None]
    u = np.asarray(v, np.float64)[None, :] / scale
    dS = n[:, None] * u ** np.maximum(n[:, None] - 1, 0) / scale
    return np.linalg.solve(V, dS)


def m2m_1d(p):
    """1D M2M operators T[o][a, a'] of Eq. 5 for child position o in {0, 1}
    along one axis.  The child centre sits at (o - 1/2) p/2 parent-gridlet units
    from the parent centre; child gridlet spacing is half the parent's, so child
    gridlet a' sits at u = (o - 1/2) p/2 + t_{a'}/2."""
    t = gridlet_coords(p)
    return [moment_matching_weights(p, (o - 0.5) * 0.5 * p + 0.5 * t) for o in (0, 1)]


def apply3(op, x, axes):
    """Apply the 1D operator op (shape (q, r)) along three trailing axes of x:
    out[..., i, j, k] = sum_{a,b,c} op[i, a] op[j, b] op[k, c] x[..., a, b, c]."""
    return np.einsum("ia,jb,kc,...abc->...ijk", op, op, op, x, optimize=True)


def apply3T(op, x):
    """Transposed tensor-product operator (Eq. 7 form):
    out[..., a, b, c] = sum_{i,j,k} op[i, a] op[j, b] op[k, c] x[..., i, j, k]."""
    return np.einsum("ia,jb,kc,...ijk->...abc", op, op, op, x, optimize=True)


# ---------------------------------------------------------------------------
# tree index sets (Sec. 2, Fig. 2)
# ---------------------------------------------------------------------------

def near_offsets():
    """Near zone: the target node and its 26 immediate neighbours (27)."""
    return [d for d in itertools.product((-1, 0, 1), repeat=3)]


def interaction_offsets(parity):
    """Interaction zone at levels >= 3 for a target node of parity c (its index
    mod 2 per axis): children of the parent's 27 neighbours that are not
    neighbours of the target.  Per axis the children span d in [-2-c, 3-c];
    removing |d|_inf <= 1 leaves 216 - 27 = 189 offsets."""
    rng = [range(-2 - c, 4 - c) for c in parity]
    return [d for d in itertools.product(*rng) if max(abs(v) for v in d) > 1]


def level2_offsets():
    """Interaction zone at level 2 of the periodic box (Sec. 2, "periodicity
    enters only at level 2"): the 4^3 level seen from any node, minus the 27 near
    nodes, each node once.  Representatives d in [-2, 1]^3 with |d|_inf = 2
    (reading: a node two steps away along an axis is the same node in either
    direction, counted once) — 64 - 27 = 37 offsets."""
    return [d for d in itertools.product(range(-2, 2), repeat=3) if max(abs(v) for v in d) > 1]


def level2_offsets_isolated():
    """Level-2 interaction zone of the isolated (non-periodic) twin: every node
    of the 4^3 level that is not a neighbour of the target, as d = u - t in
    [-3, 3]^3 with |d|_inf >= 2 (316 offsets; for a given target only those
    with u inside the box exist)."""
    return [d for d in itertools.product(range(-3, 4), repeat=3) if max(abs(v) for v in d) > 1]


# ---------------------------------------------------------------------------
# Green's function samples
# ---------------------------------------------------------------------------

def _green_grid(kind, N, coords, a, h_self):
    return _g.green_product_grid(kind, N, coords, coords, coords, a=a, h_self=h_self)


def m2l_table(kind, N, level, p, a=(-0.125,)):
    """G(eta_l j) for j in [-(4p-1), 4p-1]^3: every separation between gridlet
    points of a node and of a node of its interaction zone (Eq. 6 argument
    d + eta (r - s) with |d_i| <= 3 w_l).  Returned with offset J = 4p-1."""
    J = 4 * p - 1
    eta = 1.0 / (2 ** level * p)
    coords = eta * np.arange(-J, J + 1)
    return _green_grid(kind, N, coords, a, None), J


def near_table(kind, N, s, a=(-0.125,)):
    """Lattice G(h j) for j in [-(2s-1), 2s-1]^3 (every separation between a
    leaf cell and a cell of its near zone), self value at j = 0."""
    J = 2 * s - 1
    h = 1.0 / N
    coords = h * np.arange(-J, J + 1)
    return _green_grid(kind, N, coords, a, h), J


def near_accel_tables(kind, N, s, a=(-0.125,)):
    """Near-zone acceleration kernels D_i(h j), j in [-(2s-1), 2s-1]^3, i = x, y, z:
    minus the 4th-order central difference of the lattice G along axis i,
        D_i(j) = -(8 (G(j + e_i) - G(j - e_i)) - (G(j + 2 e_i) - G(j - 2 e_i))) / (12 h),
    the acceleration of a unit cell mass that PM's differencing of the
    potential produces (Sec. 3).  Built from G on [-(2s+1), 2s+1]^3 (self value
    at 0).  Returned as ([D_x, D_y, D_z], J)."""
    J = 2 * s - 1
    h = 1.0 / N
    Gw = _green_grid(kind, N, h * np.arange(-J - 2, J + 3), a, h)
    out = []
    for ax in range(3):
        def sh(k):
            return tuple(slice(2 + k, 2 + k + 2 * J + 1) if i == ax else slice(2, 2 * J + 3)
                         for i in range(3))
        out.append(-(8.0 * (Gw[sh(1)] - Gw[sh(-1)]) - (Gw[sh(2)] - Gw[sh(-2)])) / (12.0 * h))
    return out, J


def _toeplitz_block(tab, J, q, d):
    """Dense K[(x), (y)] = tab[x - y - q d + J] for node-local points x, y in
    [0, q)^3 (flattened z-fastest): the operator coupling a node to the node at
    offset d, as in Eq. 6 / the near-zone sum."""
    r = np.arange(q)
    jx = r[:, None] - r[None, :] - q * d[0] + J
    jy = r[:, None] - r[None, :] - q * d[1] + J
    jz = r[:, None] - r[None, :] - q * d[2] + J
    K = tab[jx[:, None, None, :, None, None], jy[None, :, None, None, :, None],
            jz[None, None, :, None, None, :]]
    return K.reshape(q ** 3, q ** 3)


# ---------------------------------------------------------------------------
# the FMM
# ---------------------------------------------------------------------------

def _near_sum(tab, J, mb, periodic):
    """Direct near-zone sum over the 27 neighbour leaves for every cell:
    out[b, c] = sum_{e, c'} tab[c - c' - s e + J] mb[b + e, c'], leaves wrapped
    periodically, or absent outside the box for the isolated twin.  ``mb`` are
    the cell masses in leaf-block layout (nL, nL, nL, s, s, s)."""
    nL, s = mb.shape[0], mb.shape[3]
    out = np.zeros((nL, nL, nL, s ** 3))
    mflat = mb.reshape(nL, nL, nL, s ** 3)
    if not periodic:  # a layer of empty leaves around the box
        mflat = np.pad(mflat, ((1, 1), (1, 1), (1, 1), (0, 0)))
    bi = np.arange(nL)
    for e in near_offsets():
        K = _toeplitz_block(tab, J, s, e)
        if periodic:
            ix, iy, iz = (bi + e[0]) % nL, (bi + e[1]) % nL, (bi + e[2]) % nL
        else:
            ix, iy, iz = bi + e[0] + 1, bi + e[1] + 1, bi + e[2] + 1
        src = mflat[ix[:, None, None], iy[None, :, None], iz[None, None, :]]
        out += src @ K.T
    return out.reshape(nL, nL, nL, s, s, s)


def fmm(rho, L, p, kind="S1", a=(-0.125,), targets=None, stages=False,
        m2l_tables=None, periodic=True, near_tables=None):
    """Natively periodic FMM potential of the density ``rho`` (N^3, FP64).

    With ``periodic=False``: the non-periodic twin of Sec. 3 (Eq. 3), the same
    tree, gridlets and operators with the free-space G_0 (``kind`` ignored)
    and no periodic images; every zone keeps only source nodes inside the box.

    Returns Phi on the full grid, or at the (T, 3) integer ``targets`` cells.
    With ``stages=True`` also returns a dict of intermediates:
    ``M[l]`` and ``Phi[l]`` (shape (n, n, n, p, p, p)), ``far`` and ``near``.
    ``m2l_tables`` optionally overrides the per-level M2L G samples
    (dict level -> (table, J)), e.g. to test a corrected Green's function,
    and ``near_tables`` the near-zone samples G(h j) ((table, J), J = 2s - 1).
    """
    rho = np.asarray(rho, np.float64)
    N = rho.shape[0]
    assert rho.shape == (N, N, N)
    assert L >= 2 and N % (2 ** L) == 0
    s = N >> L
    nL = 2 ** L
    h = 1.0 / N
    m = rho * h ** 3                                    # cell masses
    mb = m.reshape(nL, s, nL, s, nL, s).transpose(0, 2, 4, 1, 3, 5)

    # ---- upward pass: P2M (Sec. 2 effective masses) then M2M (Eq. 5) ----
    A = p2m_1d(p, s)
    T = m2m_1d(p)
    M = {L: apply3(A, mb, None)}
    for l in range(L - 1, 1, -1):
        child = M[l + 1]
        n = 2 ** l
        par = np.zeros((n, n, n, p, p, p))
        for o in itertools.product((0, 1), repeat=3):
            c = child[o[0]::2, o[1]::2, o[2]::2]
            par += np.einsum("ia,jb,kc,...abc->...ijk", T[o[0]], T[o[1]], T[o[2]], c,
                             optimize=True)
        M[l] = par

    # ---- M2L (Eq. 6) per level, then L2L (Eq. 7) ----
    Phi = {}
    for l in range(2, L + 1):
        n = 2 ** l
        if m2l_tables is not None and l in m2l_tables:
            tab, J = m2l_tables[l]
        else:
            tab, J = m2l_table(kind if periodic else "N", N, l, p, a)
        Ml = M[l].reshape(n, n, n, p ** 3)
        out = np.zeros((n, n, n, p ** 3))
        # target nodes, grouped by parity class (the interaction zone depends on
        # it at levels >= 3); when ``targets`` is given, only the leaves holding
        # requested targets and their ancestors (the only nodes whose field
        # reaches those targets through Eq. 7)
        allb = np.indices((n, n, n)).reshape(3, -1).T
        if targets is not None:
            leaves = np.asarray(targets, np.int64).reshape(-1, 3) // s
            allb = np.unique(leaves >> (L - l), axis=0)
        if l == 2:
            groups = {(0, 0, 0): (allb, level2_offsets() if periodic else level2_offsets_isolated())}
        else:
            groups = {}
            for c in itertools.product((0, 1), repeat=3):
                sel = allb[np.all(allb % 2 == np.asarray(c), axis=1)]
                groups[c] = (sel, interaction_offsets(c))
        # offsets shared by several classes are built once
        users = {}
        for c, (tb, offs) in groups.items():
            for d in offs:
                users.setdefault(d, []).append(tb)
        for d, tbs in users.items():
            K = _toeplitz_block(tab, J, p, d)
            for tb in tbs:
                if len(tb) == 0:
                    continue
                sb = tb + np.asarray(d)
                if periodic:
                    sb = sb % n
                else:  # sources outside the box are absent
                    keep = np.all((sb >= 0) & (sb < n), axis=1)
                    tb, sb = tb[keep], sb[keep]
                    if len(tb) == 0:
                        continue
                src = Ml[sb[:, 0], sb[:, 1], sb[:, 2]]
                out[tb[:, 0], tb[:, 1], tb[:, 2]] += src @ K.T
        out = out.reshape(n, n, n, p, p, p)
        if l > 2:
            # L2L (Eq. 7): the parent's local field interpolated onto the child
            par = Phi[l - 1]
            for o in itertools.product((0, 1), repeat=3):
                out[o[0]::2, o[1]::2, o[2]::2] += np.einsum(
                    "ia,jb,kc,...ijk->...abc", T[o[0]], T[o[1]], T[o[2]], par, optimize=True)
        Phi[l] = out

    # ---- downward to cells: L2P (transpose of P2M) and the near zone ----
    if near_tables is not None:
        ntab, NJ = near_tables
    else:
        ntab, NJ = near_table(kind if periodic else "N", N, s, a)
    if targets is None:
        far = apply3T(A, Phi[L])                        # [b..., c...]
        near = _near_sum(ntab, NJ, mb, periodic)
        phi_blk = far + near
        res = phi_blk.transpose(0, 3, 1, 4, 2, 5).reshape(N, N, N)
        if stages:
            return res, dict(M=M, Phi=Phi, far=far, near=near)
        return res

    tg = np.asarray(targets, dtype=np.int64).reshape(-1, 3)
    b = tg // s
    c = tg % s
    # far: L2P at the target cells only
    PL = Phi[L][b[:, 0], b[:, 1], b[:, 2]]                       # (T, p, p, p)
    far = np.einsum("ti,tj,tk,tijk->t", A.T[c[:, 0]], A.T[c[:, 1]], A.T[c[:, 2]], PL)
    near = np.zeros(len(tg))
    r = np.arange(s)
    for e in near_offsets():
        sb = b + np.asarray(e)
        inside = np.all((sb >= 0) & (sb < nL), axis=1) if not periodic else np.ones(len(sb), bool)
        sb = sb % nL
        src = mb[sb[:, 0], sb[:, 1], sb[:, 2]] * inside[:, None, None, None]  # (T, s, s, s)
        jx = c[:, 0, None] - r[None, :] - s * e[0] + NJ
        jy = c[:, 1, None] - r[None, :] - s * e[1] + NJ
        jz = c[:, 2, None] - r[None, :] - s * e[2] + NJ
        Kr = ntab[jx[:, :, None, None], jy[:, None, :, None], jz[:, None, None, :]]
        near += np.sum(Kr * src, axis=(1, 2, 3))
    res = far + near
    if stages:
        return res, dict(M=M, Phi=Phi, far=far, near=near)
    return res


def fmm_accel(rho, L, p, kind="S1", a=(-0.125,), periodic=True):
    """Accelerations g = -grad(Phi) of the FMM taken from the expansion
    (Sec. 3: PM differences its potential, the FMM differentiates its
    expansion).  Reading adopted for the two parts of a target's field:

    * far part (interaction zones of every level, carried down by Eq. 7): the
      analytic gradient of the leaf's local expansion, i.e. of the degree p-1
      interpolant that L2P evaluates, at the cell centre;
    * near part (27 leaves, direct): the direct sum with the kernels of
      ``near_accel_tables``, so that, as for the potential, the near zone
      carries no expansion error.

    Returns (g, phi): g of shape (3, N, N, N) and the potential of ``fmm``.
    ``periodic=False`` gives the non-periodic twin."""
    rho = np.asarray(rho, np.float64)
    N = rho.shape[0]
    s = N >> L
    nL = 2 ** L
    h = 1.0 / N
    phi, st = fmm(rho, L, p, kind, a, stages=True, periodic=periodic)
    A = p2m_1d(p, s)
    v = (np.arange(s, dtype=np.float64) + 0.5 - 0.5 * s) * (p / s)
    Ad = interpolant_derivative_weights(p, v)
    eta = 1.0 / (nL * p)                               # leaf gridlet spacing
    mb = (rho * h ** 3).reshape(nL, s, nL, s, nL, s).transpose(0, 2, 4, 1, 3, 5)
    D, J = near_accel_tables(kind if periodic else "N", N, s, a)
    g = np.empty((3, N, N, N))
    for ax in range(3):
        ops = [Ad if i == ax else A for i in range(3)]
        far = -np.einsum("ai,bj,ck,...abc->...ijk", ops[0], ops[1], ops[2], st["Phi"][L],
                         optimize=True) / eta
        tot = far + _near_sum(D[ax], J, mb, periodic)
        g[ax] = tot.transpose(0, 3, 1, 4, 2, 5).reshape(N, N, N)
    return g, phi
