"""Write dg_corner_oracle.txt: the oracle's Green's-function error (Eq. 3) for
the corner point source of Sec. 3 (unit mass in cell (0,0,0) of a 128^3 mesh,
3-level tree, 16^3-cell leaves) at N_g = p = 4, 6, 8, for G_S with a_1 from
Table 1 and a_1 = -1/8 (G_S1).  Calls only the oracle (FP64, CPU; about ten
minutes).  Run from the repository root:  python tests/golden/make_dg_corner.py

With ``--t7`` it writes dg_corner_t7_oracle.txt instead: the same error for
the G_S variant with two coefficients whose map is t + O(t^7) (Sec. 3; a_1 =
-25/128, a_2 = 3/128) beside G_S1, at p = 4, 6, 8.
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
from oracle import fmm as ofmm, metric  # noqa: E402

N, L = 128, 3
A1 = {4: [-0.138598, -0.125], 6: [-0.120236, -0.125], 8: [-0.120236, -0.125]}


T7 = (-25.0 / 128.0, 3.0 / 128.0)


def corner_errors(p, a1s):
    h = 1.0 / N
    sh = metric.twin_shift(N)
    rho = np.zeros((N, N, N))
    rho[sh, sh, sh] = 1.0 / h ** 3
    g, _ = ofmm.fmm_accel(rho, L, p, periodic=False)
    e_np = metric.untranslate(g - metric.point_sources_accel(N, [[0, 0, 0]], [1.0], periodic=False,
                                                              shift=sh), sh)
    rho = np.zeros((N, N, N))
    rho[0, 0, 0] = 1.0 / h ** 3
    rows = [(p, None) + metric.norms(np.linalg.norm(e_np, axis=0))]
    for a1 in a1s:
        a = tuple(a1) if isinstance(a1, tuple) else (a1,)
        g, _ = ofmm.fmm_accel(rho, L, p, "S", a=a)
        e_p = g - metric.point_sources_accel(N, [[0, 0, 0]], [1.0], "S", a)
        rows.append((p, a1) + metric.norms(metric.delta_g(e_p, e_np)))
    return rows


def main_t7():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dg_corner_t7_oracle.txt")
    lines = ["# Oracle (FP64) Green's-function error Delta g (Eq. 3) of the corner point",
             "# source, 128^3, L = 3, for G_S1 (a_1 = -1/8, a_2 = 0) and the variant whose",
             "# map is t + O(t^7) (a_1 = -25/128, a_2 = 3/128; Sec. 3).  Written by",
             "# make_dg_corner.py --t7.",
             "# columns: p  a_1  a_2  L2  L_MAX"]
    for p in (4, 6, 8):
        for p_, a, l2, lmax in corner_errors(p, [(-0.125, 0.0), T7])[1:]:
            lines.append("%d %r %r %.6e %.6e" % (p_, a[0], a[1], l2, lmax))
            print(lines[-1], flush=True)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dg_corner_oracle.txt")
    lines = ["# Oracle (FP64) Green's-function error Delta g (Eq. 3) of the corner point",
             "# source, 128^3, L = 3, G_S(a_1); twin source translated by N/2 and its error",
             "# translated back.  Rows with a_1 = nan give the twin's own error",
             "# (the multipole-expansion error).  Written by make_dg_corner.py.",
             "# columns: p  a_1  L2  L_MAX"]
    for p, a1s in A1.items():
        for p_, a1, l2, lmax in corner_errors(p, a1s):
            lines.append("%d %s %.6e %.6e" % (p_, "nan" if a1 is None else repr(a1), l2, lmax))
            print(lines[-1], flush=True)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main_t7() if "--t7" in sys.argv[1:] else main()
