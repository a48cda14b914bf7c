"""Periodic 4th-order finite-difference accelerations (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 3 (definition of the error): accelerations are taken from the potential by
4th-order central differences, which the paper reports as converged.
"""
import numpy as np


def accel_fd4(phi):
    """a = -grad(Phi) with the 4th-order central stencil
    dPhi/dx_i ~ (-Phi[i+2] + 8 Phi[i+1] - 8 Phi[i-1] + Phi[i-2]) / (12 h),
    periodic; returns an array of shape (3, N, N, N) (components x, y, z)."""
    phi = np.asarray(phi, np.float64)
    N = phi.shape[0]
    h = 1.0 / N
    out = np.empty((3,) + phi.shape)
    for ax in range(3):
        d = (-np.roll(phi, -2, ax) + 8.0 * np.roll(phi, -1, ax)
             - 8.0 * np.roll(phi, 1, ax) + np.roll(phi, 2, ax)) / (12.0 * h)
        out[ax] = -d
    return out
