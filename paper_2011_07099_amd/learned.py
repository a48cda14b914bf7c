"""Training driver for the learned correction of the interaction-zone tables.

Every computation runs on the device in libpfmm's kernels: the training
target of a field is its exact periodic convolution (pfmm_plan_direct), the
gradient comes from the library's adjoint sweep and network backward pass
(pfmm_learned_accumulate), the update from its Adam kernel
(pfmm_learned_step).  This module only generates the seeded fields, orders
the minibatches and stores weights (.npz, no pickle).

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


def train(N=64, L=3, p=6, n_fields=512, epochs=2, batch=16, lr=2e-3, seed0=10000,
          alpha=2.0, sigma=1.0, green="S1", theta=None, log=None):
    """Train on n_fields seeded fields.  Returns (weights, history) where the
    history holds the mean loss over all training fields before training and
    after every epoch."""
    import torch
    plan = Plan(N, L, p, green)
    rhos, targets = [], []
    for i in range(n_fields):
        rho = fields.lognormal(N, alpha, sigma, seed=seed0 + i).astype(np.float32)
        r = torch.from_numpy(rho).cuda()
        t = torch.empty_like(r)
        plan.direct(r, t)
        rhos.append(r)
        targets.append(t)
    torch.cuda.synchronize()
    plan.train_begin(init_weights() if theta is None else theta, lr)

    def mean_loss():
        return float(np.mean([plan.loss(r, t) for r, t in zip(rhos, targets)]))

    history = [mean_loss()]
    if log:
        log("before training: mean loss %.4e" % history[0])
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
    w = plan.learned_weights()
    plan.close()
    return w, history
