"""Downhill simplex minimiser for the G_S coefficients (CPU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 3 fits the free a_k of the G_S ansatz by minimising a norm of the
FMM-vs-PM error, and notes that the downhill simplex method (Nelder & Mead
1965) serves as well.  This is that method, written from its published
definition: reflection 1, expansion 2, contraction 1/2, shrink 1/2.
"""
import numpy as np


def nelder_mead(f, x0, step, xtol=1e-6, ftol=None, maxiter=200):
    """Minimise f over R^n from x0 with an initial simplex of edge ``step``
    along each axis.  Stops when every vertex lies within ``xtol`` of the best
    one (max-norm) and, if ``ftol`` is given, the function values differ by at
    most ``ftol``; or after ``maxiter`` iterations.  Returns
    (x_best, f_best, evaluations)."""
    x0 = np.atleast_1d(np.asarray(x0, np.float64))
    n = x0.size
    simplex = [x0.copy()]
    for i in range(n):
        v = x0.copy()
        v[i] += step
        simplex.append(v)
    vals = [f(v) for v in simplex]
    nev = n + 1
    for _ in range(maxiter):
        order = np.argsort(vals)
        simplex = [simplex[i] for i in order]
        vals = [vals[i] for i in order]
        spread = max(np.max(np.abs(v - simplex[0])) for v in simplex[1:])
        if spread <= xtol and (ftol is None or vals[-1] - vals[0] <= ftol):
            break
        centroid = np.mean(simplex[:-1], axis=0)
        worst = simplex[-1]
        xr = centroid + (centroid - worst)                 # reflection
        fr = f(xr)
        nev += 1
        if fr < vals[0]:
            xe = centroid + 2.0 * (centroid - worst)       # expansion
            fe = f(xe)
            nev += 1
            simplex[-1], vals[-1] = (xe, fe) if fe < fr else (xr, fr)
        elif fr < vals[-2]:
            simplex[-1], vals[-1] = xr, fr
        else:
            if fr < vals[-1]:                              # outside contraction
                xc = centroid + 0.5 * (xr - centroid)
            else:                                          # inside contraction
                xc = centroid + 0.5 * (worst - centroid)
            fc = f(xc)
            nev += 1
            if fc < min(fr, vals[-1]):
                simplex[-1], vals[-1] = xc, fc
            else:                                          # shrink towards the best
                for i in range(1, n + 1):
                    simplex[i] = simplex[0] + 0.5 * (simplex[i] - simplex[0])
                    vals[i] = f(simplex[i])
                    nev += 1
    i = int(np.argmin(vals))
    return simplex[i], vals[i], nev
