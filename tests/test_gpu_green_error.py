"""The Green's-function error of Sec. 3 (Eq. 3) measured with the GPU FMM:
accelerations from the expansion, periodic G_S(a_1) run minus PM, less the
non-periodic twin's error (sources translated by half the box, the error
translated back), for the paper's fixtures on the 128^3 mesh with a 3-level
tree (16^3-cell leaves).  PM accelerations are the oracle's (FP64, point
sources in closed form).  The GPU runs in FP32 with every level's
interaction zone in FP64.

* Corner source, p = 4, 6, 8: L2 and L_MAX of |Delta g| at Table 1's a_1 and
  at a_1 = -1/8 against the oracle's values (tests/golden/dg_corner_oracle.txt,
  written by make_dg_corner.py from the oracle alone); the difference is the
  GPU's FP32 arithmetic.
* The fit of Sec. 3: a_1 minimising L2 by the downhill simplex, per p, with
  the GPU evaluating Delta g; the fitted a_1 and the error at it against
  Table 1 (tests/golden/table1_3d.txt).  Also a_1 minimising L_MAX, and
  (a_1, a_2) minimising L2, which must not do worse than one coefficient.
* Ten random sources (Fig. 5): the Green's-function error of G_S1 and the
  multipole-expansion error (the twin's own error) for p = 4 .. 8.
* The 4-level tree (Fig. 5, bottom row: 256^3, L = 4): the corner source's
  Green's-function and expansion errors of G_S1 for p = 4, 6, 8.
* Figs. 3-4: with the "exact-in-real-space" G_X the corner source's error
  exceeds 100 % of the characteristic acceleration (aliasing at half the box);
  G_S1 lowers it by about three orders of magnitude (the colour bar of Fig. 4
  is 100x smaller).
* The variant whose map is t + O(t^7) (a_1 = -25/128, a_2 = 3/128): Sec. 3
  reports that it makes the error markedly worse than G_S1.  The GPU's error
  of the variant, and its ratio to G_S1's, against the oracle's
  (tests/golden/dg_corner_t7_oracle.txt, written by make_dg_corner.py --t7
  from the oracle alone).  The oracle finds the variant worse from p = 6 on,
  increasingly with p, and better at p = 4.
* Deviation of the force from the Newtonian form (Fig. 6 analogue, the
  GADGET-4 comparison left out): the G_S1 FMM acceleration of the corner
  source against the exact periodic Newtonian force (Ewald summation, oracle)
  and against the nearest image's -x/(4 pi r^3), |g - g_N| / |g_N| binned by
  distance.  The deviation is G_S1's own: PM with G_S1 gives the same curve
  (medians agree to 5% in every bin past 4 cells), and PM with G_K matches the
  exact periodic force to 1e-4 past 8 cells.  G_S1's force is Newtonian to a
  few 1e-3 out to L/8 and deviates by 2e-2 at L/8 - L/4 and 0.2-0.5 beyond:
  G_S1 is chosen to make the FMM agree with PM(G_S1), not with the periodic
  Newtonian force.
"""
import os

import numpy as np
import pytest

from oracle import fit, metric

pytestmark = pytest.mark.gpu

N, L = 128, 3
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return rows


class _Runner:
    """Periodic G_S plan and twin plan for one p, with unit point masses."""

    def __init__(self, p):
        import torch
        from paper_2011_07099_amd.pfmm import Plan
        self.torch = torch
        self.p = p
        self.P = Plan(N, L, p, "S", a1=-0.125, accel="expansion", fp64_levels=L - 1)
        self.NP = Plan(N, L, p, "X", isolated=True, accel="expansion", fp64_levels=L - 1)
        self.phi = torch.empty((N, N, N), dtype=torch.float32, device="cuda")
        self.acc = torch.empty((3, N, N, N), dtype=torch.float32, device="cuda")

    def _accel(self, plan, cells, masses):
        t = self.torch
        rho = t.zeros((N, N, N), dtype=t.float32, device="cuda")
        for c, m in zip(cells, masses):
            rho[c[0], c[1], c[2]] += float(m) * N ** 3
        plan.solve(rho, self.phi, self.acc)
        t.cuda.synchronize()
        return self.acc.cpu().numpy().astype(np.float64)

    def twin_error(self, cells, masses):
        sh = metric.twin_shift(N)
        moved = (np.asarray(cells) + sh) % N
        g = self._accel(self.NP, moved, masses)
        pm = metric.point_sources_accel(N, cells, masses, periodic=False, shift=sh)
        return metric.untranslate(g - pm, sh)

    def periodic_error(self, cells, masses, a1, a2=0.0):
        self.P.set_a1(a1)
        self.P.set_a2(a2)
        g = self._accel(self.P, cells, masses)
        return g - metric.point_sources_accel(N, cells, masses, "S", (a1, a2))

    def close(self):
        self.P.close()
        self.NP.close()


@pytest.fixture(scope="module", params=[4, 6, 8], ids=lambda p: "p%d" % p)
def runner(request):
    r = _Runner(request.param)
    r.corner_twin = r.twin_error([[0, 0, 0]], [1.0])
    yield r
    r.close()


def test_corner_delta_g_vs_oracle(runner):
    p = runner.p
    rows = [r for r in _rows("dg_corner_oracle.txt") if int(r[0]) == p]
    for _, a1, l2_ref, lmax_ref in rows:
        if np.isnan(a1):
            l2, lmax = metric.norms(np.linalg.norm(runner.corner_twin, axis=0))
        else:
            e = runner.periodic_error([[0, 0, 0]], [1.0], a1)
            l2, lmax = metric.norms(metric.delta_g(e, runner.corner_twin))
        print("corner p=%d a1=%s: L2 %.4e (oracle %.4e)  L_MAX %.4e (oracle %.4e)"
              % (p, a1, l2, l2_ref, lmax, lmax_ref))
        assert abs(l2 / l2_ref - 1) < 0.01 and abs(lmax / lmax_ref - 1) < 0.02


def test_corner_fit_of_a1(runner):
    p = runner.p
    table = {int(r[0]): r for r in _rows("table1_3d.txt")}
    _, lmax_paper, l2_paper, a1_paper = table[p]

    def l2_of(v):
        e = runner.periodic_error([[0, 0, 0]], [1.0], float(v[0]))
        return metric.norms(metric.delta_g(e, runner.corner_twin))[0]

    x, l2, nev = fit.nelder_mead(l2_of, [-0.125], 0.005, xtol=2e-4, maxiter=60)
    e = runner.periodic_error([[0, 0, 0]], [1.0], float(x[0]))
    _, lmax = metric.norms(metric.delta_g(e, runner.corner_twin))
    print("fit p=%d: a1 = %.5f (Table 1 %.6f), L2 %.3e (Table 1 %.3e), L_MAX %.3e "
          "(Table 1 %.3e), %d evaluations" % (p, x[0], a1_paper, l2, l2_paper, lmax, lmax_paper, nev))
    assert nev < 40  # converged on the simplex size
    assert abs(x[0] - a1_paper) < 0.03
    assert l2 < 2.5 * l2_paper and lmax < 2.5 * lmax_paper

    # the L_MAX norm by the same simplex (Sec. 3: little change in a_1)
    def lmax_of(v):
        e = runner.periodic_error([[0, 0, 0]], [1.0], float(v[0]))
        return metric.norms(metric.delta_g(e, runner.corner_twin))[1]

    xm, lm, nevm = fit.nelder_mead(lmax_of, [-0.125], 0.005, xtol=2e-4, maxiter=60)
    print("fit of L_MAX p=%d: a1 = %.5f, L_MAX %.3e, %d evaluations" % (p, xm[0], lm, nevm))
    # Sec. 3 reports little change of a_1 with the norm; measured here:
    # -0.153 / -0.133 / -0.127 against the L2 fit's -0.124 / -0.126 / -0.124
    # (printed, not held to a window).  What a minimum guarantees: the L_MAX
    # fit's L_MAX is no larger than L_MAX at the L2 fit's a_1.
    assert lm <= lmax * (1 + 1e-9)

    # two coefficients (a_1, a_2): Sec. 3 finds the second term of little use
    def l2_of2(v):
        e = runner.periodic_error([[0, 0, 0]], [1.0], float(v[0]), float(v[1]))
        return metric.norms(metric.delta_g(e, runner.corner_twin))[0]

    x2, l22, nev2 = fit.nelder_mead(l2_of2, [float(x[0]), 0.0], 0.004, xtol=2e-4, maxiter=120)
    e = runner.periodic_error([[0, 0, 0]], [1.0], float(x2[0]), float(x2[1]))
    lmax2 = metric.norms(metric.delta_g(e, runner.corner_twin))[1]
    print("fit of (a1, a2) p=%d: a1 = %.5f a2 = %.5f, L2 %.3e (one coefficient %.3e), "
          "L_MAX %.3e (%.3e), %d evaluations" % (p, x2[0], x2[1], l22, l2, lmax2, lmax, nev2))
    assert l22 <= l2 * (1 + 1e-9)


def test_ten_random_sources_gf_and_me_error(runner):
    p = runner.p
    rng = np.random.default_rng(1010)
    cells = rng.integers(0, N, size=(10, 3))
    masses = np.full(10, 0.125)  # exact in FP32
    twin = runner.twin_error(cells, masses)
    e = runner.periodic_error(cells, masses, -0.125)
    gf = metric.norms(metric.delta_g(e, twin))
    me = metric.norms(np.linalg.norm(twin, axis=0))
    print("10 random sources p=%d: GF error L2 %.3e L_MAX %.3e | ME error L2 %.3e L_MAX %.3e"
          % (p, gf[0], gf[1], me[0], me[1]))
    assert gf[0] < 3.0 * me[0]


def test_t7_variant_against_gs1(runner):
    p = runner.p
    rows = {(r[1], r[2]): r[3:] for r in _rows("dg_corner_t7_oracle.txt") if int(r[0]) == p}
    ref_s1, ref_t7 = rows[(-0.125, 0.0)], rows[(-25.0 / 128.0, 3.0 / 128.0)]
    base = metric.norms(metric.delta_g(runner.periodic_error([[0, 0, 0]], [1.0], -0.125),
                                       runner.corner_twin))
    t7 = metric.norms(metric.delta_g(
        runner.periodic_error([[0, 0, 0]], [1.0], -25.0 / 128.0, 3.0 / 128.0), runner.corner_twin))
    ratio, ref_ratio = t7[0] / base[0], ref_t7[0] / ref_s1[0]
    print("t^7 variant p=%d: L2 %.3e (oracle %.3e) L_MAX %.3e (oracle %.3e) | ratio to G_S1: "
          "L2 %.3f (oracle %.3f), L_MAX %.3f (oracle %.3f)"
          % (p, t7[0], ref_t7[0], t7[1], ref_t7[1], ratio, ref_ratio, t7[1] / base[1],
             ref_t7[1] / ref_s1[1]))
    # the GPU's FP32 arithmetic: 1% in L2, 2% in L_MAX, as for the other rows
    assert abs(t7[0] / ref_t7[0] - 1) < 0.01 and abs(t7[1] / ref_t7[1] - 1) < 0.02
    assert abs(ratio / ref_ratio - 1) < 0.02
    # the direction Sec. 3 reports holds wherever the oracle finds it
    if ref_ratio > 1:
        assert ratio > 1


BINS = [1, 2, 4, 8, 16, 32, 64, 112]


def _binned_median(dev, r):
    # cells where the reference force vanishes (the box's symmetry points) drop out
    out = []
    for lo, hi in zip(BINS[:-1], BINS[1:]):
        v = dev[(r >= lo) & (r < hi)]
        out.append(float(np.median(v[np.isfinite(v)])))
    return out


def test_deviation_from_newtonian_force(runner):
    p = runner.p
    runner.P.set_a1(-0.125)
    runner.P.set_a2(0.0)
    g = runner._accel(runner.P, [[0, 0, 0]], [1.0])
    exact = metric.periodic_point_accel(N, (0, 0, 0))
    j = np.arange(N)
    d = np.minimum(j, N - j).astype(np.float64)
    r = np.sqrt(d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2)
    x = np.stack(np.meshgrid(*([np.where(j < N // 2, j, j - N) / N] * 3), indexing="ij"))
    with np.errstate(divide="ignore", invalid="ignore"):
        newton = -x / (4 * np.pi * np.sum(x * x, axis=0) ** 1.5)
        dev = np.linalg.norm(g - exact, axis=0) / np.linalg.norm(exact, axis=0)
        dev_n = np.linalg.norm(g - newton, axis=0) / np.linalg.norm(newton, axis=0)
        pm = metric.point_sources_accel(N, [[0, 0, 0]], [1.0], "S1")
        dev_pm = np.linalg.norm(pm - exact, axis=0) / np.linalg.norm(exact, axis=0)
    fmm_b, newt_b, pm_b = _binned_median(dev, r), _binned_median(dev_n, r), _binned_median(dev_pm, r)
    for (lo, hi), a, b, c in zip(zip(BINS[:-1], BINS[1:]), fmm_b, newt_b, pm_b):
        print("p=%d r in [%3d, %3d) cells: median |g - g_N|/|g_N| vs periodic %.2e "
              "(PM(G_S1) %.2e), vs nearest image %.2e" % (p, lo, hi, a, c, b))
    for lo, a, c in zip(BINS[:-1], fmm_b, pm_b):
        if lo >= 4:
            assert abs(a - c) <= 0.05 * c


@pytest.mark.parametrize("p", [4, 6, 8])
def test_corner_errors_on_the_four_level_tree(p):
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    N4, L4 = 256, 4
    sh = metric.twin_shift(N4)
    out = {}
    phi = torch.empty((N4, N4, N4), dtype=torch.float32, device="cuda")
    acc = torch.empty((3, N4, N4, N4), dtype=torch.float32, device="cuda")
    for name, kw, cell in (("P", dict(green="S1"), 0), ("NP", dict(green="X", isolated=True), sh)):
        with Plan(N4, L4, p, accel="expansion", fp64_levels=L4 - 1, **kw) as pl:
            rho = torch.zeros((N4, N4, N4), dtype=torch.float32, device="cuda")
            rho[cell, cell, cell] = float(N4) ** 3
            pl.solve(rho, phi, acc)
            torch.cuda.synchronize()
            out[name] = acc.cpu().numpy().astype(np.float64)
        del rho
    e_p = out["P"] - metric.point_sources_accel(N4, [[0, 0, 0]], [1.0], "S1")
    e_np = metric.untranslate(out["NP"] - metric.point_sources_accel(
        N4, [[0, 0, 0]], [1.0], periodic=False, shift=sh), sh)
    gf = metric.norms(metric.delta_g(e_p, e_np))
    me = metric.norms(np.linalg.norm(e_np, axis=0))
    print("corner, 256^3 L=4, p=%d: GF error L2 %.3e L_MAX %.3e | ME error L2 %.3e L_MAX %.3e"
          % (p, gf[0], gf[1], me[0], me[1]))
    # Fig. 5: the Green's-function error stays below or about the expansion error
    assert gf[0] < 2.0 * me[0]


def test_gx_aliasing_against_gs1():
    # Figs. 3-4 use N_g = 6
    from paper_2011_07099_amd.pfmm import Plan
    p = 6
    r = _Runner(p)
    try:
        twin = r.twin_error([[0, 0, 0]], [1.0])
        with Plan(N, L, p, "X", accel="expansion", fp64_levels=L - 1) as px:
            g = r._accel(px, [[0, 0, 0]], [1.0])
        e_x = g - metric.point_sources_accel(N, [[0, 0, 0]], [1.0], "X")
        gx = metric.norms(metric.delta_g(e_x, twin))
        gs = metric.norms(metric.delta_g(r.periodic_error([[0, 0, 0]], [1.0], -0.125), twin))
    finally:
        r.close()
    print("corner, p=6: G_X L2 %.3e L_MAX %.3e | G_S1 L2 %.3e L_MAX %.3e | ratio L_MAX %.0f"
          % (gx[0], gx[1], gs[0], gs[1], gx[1] / gs[1]))
    assert gx[1] > 1.0 and gx[1] > 300 * gs[1]
