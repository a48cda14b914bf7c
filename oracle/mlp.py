"""FP64 reference of the learned table correction (CPU) — TEST INFRASTRUCTURE ONLY.

The paper defines the optimal Green's function G_* as the one with which the
FMM reproduces the PM solution (Sec. 3, Eq. 8) and proposes to parameterise
it by many free values (Sec. 4).  The correction studied here multiplies every
interaction-zone table entry by (1 + delta), delta = KAPPA * f(features) from
a network 8 -> 64 -> 64 -> 1 with SiLU activations and the fixed output scale
KAPPA = 1e-4.  Its input is the table offset j = a - a' - p d of Eq. 6
reduced to what the cube's 48 symmetries leave invariant (so the corrected
table stays symmetric), plus the level and p:

    (u1 >= u2 >= u3) = |j| sorted descending,
    features(j, level, p) = (u1/(4p), u2/(4p), u3/(4p),
                             (u1 mod p)/p, (u2 mod p)/p, (u3 mod p)/p,
                             level/8, p/10),

where u_i mod p is the in-gridlet residue of the offset along that axis (the
part a - a' of j up to the sign of the axis).  Weights
theta = W1[64][8] b1[64] W2[64][64] b2[64] W3[64] b3.
"""
import numpy as np

N_IN = 8
N_HID = 64
O_W1, O_B1 = 0, N_HID * N_IN
O_W2 = O_B1 + N_HID
O_B2 = O_W2 + N_HID * N_HID
O_W3 = O_B2 + N_HID
O_B3 = O_W3 + N_HID
N_PARAMS = O_B3 + 1
KAPPA = 1e-4


def unpack(theta):
    t = np.asarray(theta, np.float64)
    assert t.size == N_PARAMS
    W1 = t[O_W1:O_B1].reshape(N_HID, N_IN)
    b1 = t[O_B1:O_W2]
    W2 = t[O_W2:O_B2].reshape(N_HID, N_HID)
    b2 = t[O_B2:O_W3]
    W3 = t[O_W3:O_B3]
    b3 = t[O_B3]
    return W1, b1, W2, b2, W3, b3


def silu(z):
    return z / (1.0 + np.exp(-z))


def features(j, level, p):
    """Feature rows for integer table offsets j of shape (..., 3)."""
    a = np.sort(np.abs(np.asarray(j, np.int64)), axis=-1)[..., ::-1]
    K = 4.0 * p
    lev = np.full(a.shape[:-1] + (1,), level / 8.0)
    pp = np.full(a.shape[:-1] + (1,), p / 10.0)
    return np.concatenate([a / K, (a % p) / float(p), lev, pp], axis=-1)


def forward(theta, x):
    """Network output for feature rows x (..., N_IN), FP64."""
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
