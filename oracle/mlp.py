"""FP64 reference of the learned table correction (CPU) — TEST INFRASTRUCTURE ONLY.

The paper defines the optimal Green's function G_* as the one with which the
FMM reproduces the PM solution (Sec. 3, Eq. 8) and proposes to parameterise
it by many free values (Sec. 4).  The correction studied here multiplies every
interaction-zone table entry by (1 + delta), delta = KAPPA * f(features) from
a network 5 -> 64 -> 64 -> 1 with SiLU activations and the fixed output scale
KAPPA = 1e-4:

    features(j, level, p) = (u1/(4p), u2/(4p), u3/(4p), level/8, p/10),
    (u1 >= u2 >= u3) = |j| sorted descending  (invariant under the cube's
    48 symmetries, so the corrected table stays symmetric),
    weights theta = W1[64][5] b1[64] W2[64][64] b2[64] W3[64] b3.
"""
import numpy as np

N_PARAMS = 4609
KAPPA = 1e-4


def unpack(theta):
    t = np.asarray(theta, np.float64)
    assert t.size == N_PARAMS
    W1 = t[0:320].reshape(64, 5)
    b1 = t[320:384]
    W2 = t[384:4480].reshape(64, 64)
    b2 = t[4480:4544]
    W3 = t[4544:4608]
    b3 = t[4608]
    return W1, b1, W2, b2, W3, b3


def silu(z):
    return z / (1.0 + np.exp(-z))


def features(j, level, p):
    """Feature rows for integer table offsets j of shape (..., 3)."""
    a = np.sort(np.abs(np.asarray(j, np.int64)), axis=-1)[..., ::-1]
    K = 4.0 * p
    lev = np.full(a.shape[:-1] + (1,), level / 8.0)
    pp = np.full(a.shape[:-1] + (1,), p / 10.0)
    return np.concatenate([a / K, lev, pp], axis=-1)


def forward(theta, x):
    """Network output for feature rows x (..., 5), FP64."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    h1 = silu(x @ W1.T + b1)
    h2 = silu(h1 @ W2.T + b2)
    return h2 @ W3 + b3


def corrected_table(table, level, p, theta):
    """T[j] = table[j] (1 + KAPPA f(features(j))) on a centred (2C+1)^3 table."""
    E = table.shape[0]
    C = (E - 1) // 2
    r = np.arange(-C, C + 1)
    j = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1)
    return table * (1.0 + KAPPA * forward(theta, features(j, level, p)))
