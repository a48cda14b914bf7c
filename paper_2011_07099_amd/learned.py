"""Training driver for the learned correction of the interaction-zone tables.

Every computation runs on the device in libpfmm's kernels: the training
target of a field is its exact periodic convolution (pfmm_plan_direct), the
gradient comes from the library's adjoint sweep and network backward pass
(pfmm_learned_accumulate), the update from its Adam kernel
(pfmm_learned_step).  This module only generates the seeded fields, orders
the minibatches and stores weights (.npz, no pickle).  ``train_table`` does
the same for the grid-valued tables (one free value per cube-symmetry orbit
of table entries), with Adam on those values directly.

``fit_output`` trains the network's output layer exactly (the loss is
quadratic in it).  ``fit_gstar`` fits G_* as one grid-valued function used
everywhere, near zone and PM included (Eq. 8's setting).

Defaults follow the training workload: 512 lognormal 64^3 fields (P(k) ~
k^-2, sigma_delta = 1, seeds 10000 + i), L = 3, p = 6, G_S1.
"""
import numpy as np

from . import fields
from .pfmm import MLP_PARAMS, Plan


# weight layout of the network (the library's): W1[64][8] b1[64] W2[64][64]
# b2[64] W3[64] b3
N_IN, N_HID = 8, 64
O_B1 = N_HID * N_IN
O_W2 = O_B1 + N_HID
O_B2 = O_W2 + N_HID * N_HID
O_W3 = O_B2 + N_HID
O_B3 = O_W3 + N_HID


def init_weights(seed=0, scale=1.0):
    """Random hidden layers, zero output layer: the untrained network is
    exactly the uncorrected Green's function.  W1 is He-normal times
    `scale`; each first-layer unit's bias puts its SiLU knee through a random
    point of the unit cube of inputs (the features lie in [0, 1]), so the
    hidden units bend inside the data instead of all at the origin.  W2 is
    He-normal with zero biases."""
    rng = np.random.default_rng(seed)
    th = np.zeros(MLP_PARAMS, np.float32)
    W1 = rng.standard_normal((N_HID, N_IN)) * np.sqrt(2.0 / N_IN) * scale
    x0 = rng.uniform(size=(N_HID, N_IN))
    th[0:O_B1] = W1.ravel()
    th[O_B1:O_W2] = -np.sum(W1 * x0, axis=1)
    th[O_W2:O_B2] = rng.standard_normal(N_HID * N_HID) * np.sqrt(2.0 / N_HID)
    return th


def save(path, theta, **meta):
    np.savez(path, theta=np.asarray(theta, np.float32), **{k: np.asarray(v) for k, v in meta.items()})


def load(path):
    with np.load(path, allow_pickle=False) as z:
        return z["theta"].astype(np.float32)


def _fields_and_targets(plan, N, n_fields, alpha, sigma, seed0):
    import torch
    rhos, targets = [], []
    for i in range(n_fields):
        rho = fields.lognormal(N, alpha, sigma, seed=seed0 + i).astype(np.float32)
        r = torch.from_numpy(rho).cuda()
        t = torch.empty_like(r)
        plan.direct(r, t)
        rhos.append(r)
        targets.append(t)
    torch.cuda.synchronize()
    return rhos, targets


def _run_epochs(plan, rhos, targets, epochs, batch, seed0, log):
    def mean_loss():
        return float(np.mean([plan.loss(r, t) for r, t in zip(rhos, targets)]))

    history = [mean_loss()]
    if log:
        log("before training: mean loss %.4e" % history[0])
    n_fields = len(rhos)
    order = np.arange(n_fields)
    rng = np.random.default_rng(seed0)
    for ep in range(epochs):
        rng.shuffle(order)
        for b0 in range(0, n_fields, batch):
            for i in order[b0:b0 + batch]:
                plan.train_accumulate(rhos[i], targets[i])
            plan.train_step()
        history.append(mean_loss())
        if log:
            log("epoch %d: mean loss %.4e" % (ep, history[-1]))
    return history


def train(N=64, L=3, p=6, n_fields=512, epochs=2, batch=16, lr=2e-3, seed0=10000,
          alpha=2.0, sigma=1.0, green="S1", theta=None, log=None):
    """Train on n_fields seeded fields.  Returns (weights, history) where the
    history holds the mean loss over all training fields before training and
    after every epoch."""
    plan = Plan(N, L, p, green)
    rhos, targets = _fields_and_targets(plan, N, n_fields, alpha, sigma, seed0)
    plan.train_begin(init_weights() if theta is None else theta, lr)
    history = _run_epochs(plan, rhos, targets, epochs, batch, seed0, log)
    w = plan.learned_weights()
    plan.close()
    return w, history


def train_table(N=64, L=3, p=6, n_fields=512, epochs=2, batch=16, lr=2e-6, seed0=10000,
                alpha=2.0, sigma=1.0, green="S1", log=None):
    """Train the grid-valued tables (one free relative correction per
    cube-symmetry orbit of table entries and level, from exactly G) on the
    same fields and loss as ``train``.  Returns (delta, history)."""
    plan = Plan(N, L, p, green)
    rhos, targets = _fields_and_targets(plan, N, n_fields, alpha, sigma, seed0)
    plan.table_train_begin(lr)
    history = _run_epochs(plan, rhos, targets, epochs, batch, seed0, log)
    d = plan.table_values()
    plan.close()
    return d, history


def _conjugate_gradients(loss_at, grad_at, n, iters, log):
    """Polak-Ribiere nonlinear conjugate gradients from delta = 0, restarted
    when the direction is not a descent one.  Each line search fits a
    parabola along the direction from the slope and one trial loss (exact
    when the loss is quadratic) and keeps the step only if the loss falls.
    Returns (delta, history of the loss)."""
    delta = np.zeros(n)
    f0 = loss_at(delta)
    history = [f0]
    g = grad_at(delta)
    d = -g
    for it in range(iters):
        slope = float(g @ d)
        if slope >= 0:                 # not a descent direction: restart
            d = -g
            slope = float(g @ d)
        # trial step: a relative change of 1e-6 in the largest entry
        h = 1e-6 / max(float(np.max(np.abs(d))), 1e-30)
        f1 = loss_at(delta + h * d)
        c2 = (f1 - f0 - slope * h) / (h * h)
        step = -slope / (2.0 * c2) if c2 > 0 else h
        trial = delta + step * d
        ft = loss_at(trial)
        if ft >= f0:                   # the quadratic model failed (rounding): keep delta
            if log:
                log("iteration %d: no decrease (%.4e >= %.4e), stop" % (it, ft, f0))
            break
        delta, f0 = trial, ft
        history.append(f0)
        g_new = grad_at(delta)
        beta = max(0.0, float(g_new @ (g_new - g)) / max(float(g @ g), 1e-300))
        d = -g_new + beta * d
        g = g_new
        if log:
            log("iteration %d: mean loss %.4e, step %.3e, max |delta| %.3e"
                % (it, f0, step, float(np.max(np.abs(delta)))))
    return delta, history


def fit_table(N=64, L=3, p=6, n_fields=64, iters=10, seed0=10000, alpha=2.0, sigma=1.0,
              green="S1", log=None):
    """Fit the grid-valued tables by nonlinear conjugate gradients
    (Polak-Ribiere, restarted when the direction is not a descent one) on the
    summed loss over n_fields fields.  The loss is exactly quadratic in delta,
    so each line search is exact from the slope (gradient . direction) and one
    more loss evaluation.  Gradients and losses come from the device (adjoint
    sweep, pfmm_learned_accumulate / pfmm_learned_loss); this driver only
    combines the (L - 1) x orbits values.  Returns (delta, history of the mean
    training loss)."""
    plan = Plan(N, L, p, green)
    rhos, targets = _fields_and_targets(plan, N, n_fields, alpha, sigma, seed0)
    plan.table_train_begin(1e-9)
    n = plan.table_params()

    def loss_at(x):
        plan.set_table(x.astype(np.float32))
        return float(np.mean([plan.loss(r, t) for r, t in zip(rhos, targets)]))

    def grad_at(x):
        plan.set_table(x.astype(np.float32))
        for r, t in zip(rhos, targets):
            plan.train_accumulate(r, t)
        return plan.table_grad().astype(np.float64) / n_fields

    delta, history = _conjugate_gradients(loss_at, grad_at, n, iters, log)
    plan.close()
    return delta.astype(np.float32), history


def fit_gstar(N=64, L=4, p=4, n_fields=16, iters=10, seed0=10000, alpha=2.0, sigma=1.0,
              green="S1", log=None):
    """Fit G_* = G (1 + delta[orbit]) as one grid-valued function on the mesh,
    used by the near zone, every level's tables and the PM solution (Sec. 3,
    Eq. 8; Sec. 4), by the same conjugate gradients on the mean loss of the
    FMM against PM, both with G_*, over n_fields seeded fields.  The target
    moves with delta, so the loss is a ratio of quadratics rather than a
    quadratic; the line search keeps only steps that lower it.  Gradients and
    losses come from the device (pfmm_gstar_accumulate, pfmm_gstar_loss).
    Needs p to divide the leaf width N / 2^L (the default is Eq. 8's own
    setting, the gridlet equal to the leaf's cells, with four levels).
    Returns (delta, history of the mean training loss)."""
    import torch
    plan = Plan(N, L, p, green)
    rhos = [torch.from_numpy(fields.lognormal(N, alpha, sigma, seed=seed0 + i).astype(np.float32))
            .cuda() for i in range(n_fields)]
    n = plan.gstar_params()

    def loss_at(x):
        plan.set_gstar(x.astype(np.float32))
        return float(np.mean([plan.gstar_loss(r) for r in rhos]))

    def grad_at(x):
        plan.set_gstar(x.astype(np.float32))
        for r in rhos:
            plan.gstar_accumulate(r)
        return plan.gstar_grad().astype(np.float64) / n_fields

    delta, history = _conjugate_gradients(loss_at, grad_at, n, iters, log)
    plan.close()
    return delta.astype(np.float32), history


def fit_output(N=64, L=3, p=6, n_fields=64, n_valid=8, seed0=10000, alpha=2.0, sigma=1.0,
               green="S1", seed=0, scale=8.0,
               ridges=(1e-6, 1e-5, 1e-4, 3e-4, 1e-3, 3e-3, 1e-2, 3e-2, 1e-1), h=1.0, log=None):
    """Train the network's output layer exactly.  The FMM is linear in its
    tables and the tables are linear in the output layer (W3, b3) for fixed
    hidden layers, so the training loss is exactly quadratic in those 65
    weights: L(c) = L0 + g.c + c.H.c / 2.  The device gives g (adjoint sweep,
    table gradient and network backward pass over the n_fields training
    fields) and every column of H as a difference of two such gradients (the
    gradient of a quadratic is affine, so any step h is exact up to
    rounding).  The minimiser solves (H + r I) c = -g for each ridge factor r
    (relative to the mean eigenvalue of H); the one with the lowest loss on
    n_valid further fields, with the BF16 inference tables the library uses
    for PFMM_GREEN_LEARNED, is kept (the plain G if none beats it).  The
    hidden layers keep their random initialisation (init_weights(seed,
    scale)); a first-layer scale of 8 gives units that bend within a few
    table offsets.  Returns (weights, info)."""
    plan = Plan(N, L, p, green)
    rhos, targets = _fields_and_targets(plan, N, n_fields, alpha, sigma, seed0)
    vr, vt = _fields_and_targets(plan, N, n_valid, alpha, sigma, seed0 + n_fields)
    if log:
        log("%d training and %d validation fields with their targets" % (n_fields, n_valid))
    th0 = init_weights(seed, scale)
    nout = N_HID + 1

    def grad_out(th):
        plan.train_begin(th, 1e-3)
        for r, t in zip(rhos, targets):
            plan.train_accumulate(r, t)
        return plan.learned_grads(2)[1][O_W3:O_B3 + 1].astype(np.float64) / len(rhos)

    def mean_loss(th, rs, ts, bf16):
        if bf16:
            plan.set_learned(th, bf16=True)
        else:
            plan.train_begin(th, 1e-3)
        return float(np.mean([plan.loss(r, t) for r, t in zip(rs, ts)]))

    g0 = grad_out(th0)
    H = np.empty((nout, nout))
    for k in range(nout):
        th = th0.copy()
        th[O_W3 + k] = h
        H[:, k] = (grad_out(th) - g0) / h
        if log and (k % 8 == 7 or k == nout - 1):
            log("Hessian columns %d / %d" % (k + 1, nout))
    H = 0.5 * (H + H.T)
    ev = np.linalg.eigvalsh(H)
    base_train = mean_loss(th0, rhos, targets, False)
    base_valid = mean_loss(th0, vr, vt, False)
    info = {"train_loss_g": base_train, "valid_loss_g": base_valid,
            "hessian_eigs": [float(ev[0]), float(ev[-1])], "fits": []}
    if log:
        log("G: train %.4e valid %.4e; Hessian eigenvalues %.3e .. %.3e"
            % (base_train, base_valid, ev[0], ev[-1]))
    best = (base_valid, th0, None)
    mean_ev = float(np.mean(np.abs(ev)))
    for rr in ridges:
        c = np.linalg.solve(H + rr * mean_ev * np.eye(nout), -g0)
        th = th0.copy()
        th[O_W3:O_B3 + 1] = c.astype(np.float32)
        pred = base_train + float(g0 @ c) + 0.5 * float(c @ H @ c)
        tr = mean_loss(th, rhos, targets, False)
        v32 = mean_loss(th, vr, vt, False)
        va = mean_loss(th, vr, vt, True)
        info["fits"].append({"ridge": rr, "predicted_train": pred, "train": tr, "valid_fp32": v32,
                             "valid_bf16": va, "norm_c": float(np.linalg.norm(c))})
        if log:
            log("ridge %.0e: train %.4e (predicted %.4e), valid %.4e (fp32) %.4e (bf16), |c| %.3g"
                % (rr, tr, pred, v32, va, np.linalg.norm(c)))
        if va < best[0]:
            best = (va, th, rr)
    info["ridge"] = best[2]
    info["valid_loss"] = best[0]
    plan.close()
    return best[1], info
