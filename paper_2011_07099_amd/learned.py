"""Training driver for the learned correction of the interaction-zone tables.

Every computation runs on the device in libpfmm's kernels: the training
target of a field is its exact periodic convolution (pfmm_plan_direct), the
gradient comes from the library's adjoint sweep and network backward pass
(pfmm_learned_accumulate), the update from its Adam kernel
(pfmm_learned_step).  This module only generates the seeded fields, orders
the minibatches and stores weights (.npz, no pickle).  ``train_table`` does
the same for the grid-valued tables (one free value per cube-symmetry orbit
of table entries), with Adam on those values directly.

Defaults follow the training workload: 512 lognormal 64^3 fields (P(k) ~
k^-2, sigma_delta = 1, seeds 10000 + i), L = 3, p = 6, G_S1.
"""
import numpy as np

from . import fields
from .pfmm import MLP_PARAMS, Plan


def init_weights(seed=0):
    """He-normal hidden layers, zero output layer: the untrained network is
    exactly the uncorrected Green's function."""
    rng = np.random.default_rng(seed)
    th = np.zeros(MLP_PARAMS, np.float32)
    th[0:320] = rng.standard_normal(320) * np.sqrt(2.0 / 5.0)
    th[384:4480] = rng.standard_normal(4096) * np.sqrt(2.0 / 64.0)
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
    delta = np.zeros(n)

    def loss_at(x):
        plan.set_table(x.astype(np.float32))
        return float(np.mean([plan.loss(r, t) for r, t in zip(rhos, targets)]))

    def grad_at(x):
        plan.set_table(x.astype(np.float32))
        for r, t in zip(rhos, targets):
            plan.train_accumulate(r, t)
        return plan.table_grad().astype(np.float64) / n_fields

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
    plan.close()
    return delta.astype(np.float32), history
