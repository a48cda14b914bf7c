"""Learned correction of the interaction-zone tables.

* Gradients: the device gradient of the relative mean-removed loss with
  respect to table entries and to network weights, against central finite
  differences of the CPU FP64 pipeline (oracle reference FMM with tables
  corrected by the oracle network).  The device forward is FP32, so the
  residual it differentiates carries ~1e-7 |phi| of rounding against a
  residual of ~1e-3 |phi| at p = 4: tolerance 1e-3 relative.
* Fallback and inference: zero output layer = plain G; NULL restores G.
* Training: Adam lowers the loss; the exact output-layer fit (the loss is
  quadratic in the output layer) lowers the FMM-vs-PM error on unseen 64^3
  and 128^3 fields, with PM(G_S1) from the oracle as the judge and the
  library's BF16 inference tables.
"""
import numpy as np
import pytest

from oracle import conv, fmm as ofmm, mlp as omlp
from paper_2011_07099_amd import fields

from gpu_util import f32

pytestmark = pytest.mark.gpu


def _loss(phi, target):
    d = phi - target
    d = d - d.mean()
    t = target - target.mean()
    return float(np.sum(d * d) / np.sum(t * t))


def _oracle_loss(rho, L, p, tables, target):
    return _loss(ofmm.fmm(rho, L, p, "S1", m2l_tables=tables), target)


def test_gradients_match_finite_differences_of_the_oracle():
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    N, L, p = 32, 3, 4
    rho = f32(fields.lognormal(N, 2.0, 1.0, seed=31))
    target = f32(conv.pm(rho, "S1"))
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(omlp.N_PARAMS).astype(np.float32) * 0.05
    theta[omlp.O_W3:omlp.O_B3] = rng.standard_normal(64).astype(np.float32) * 200.0
    theta = theta.astype(np.float64).astype(np.float32)
    th64 = theta.astype(np.float64)
    with Plan(N, L, p, "S1") as pl:
        pl.train_begin(theta, 1e-3)
        r = torch.from_numpy(rho.astype(np.float32)).cuda()
        t = torch.from_numpy(target.astype(np.float32)).cuda()
        loss_gpu = pl.train_accumulate(r, t)
        tg = {l: pl.learned_grads(l)[0] for l in (2, 3)}
        wg = pl.learned_grads(2)[1]
    base = {}
    for l in (2, 3):
        tab, J = ofmm.m2l_table("S1", N, l, p)
        tab[J, J, J] = 0.0
        base[l] = omlp.corrected_table(tab, l, p, th64)
    tables = {l: (base[l], 4 * p - 1) for l in (2, 3)}
    loss_cpu = _oracle_loss(rho, L, p, tables, target)
    print("loss gpu", loss_gpu, "cpu", loss_cpu)
    assert abs(loss_gpu / loss_cpu - 1) < 1e-3
    # table entries: the largest gradients of each level
    for l in (2, 3):
        g = tg[l]
        idx = np.argsort(np.abs(g).ravel())[-3:]
        for flat in idx:
            j = np.unravel_index(flat, g.shape)
            eps = 1e-6 * abs(base[l][j])
            tp = dict(tables)
            a = base[l].copy(); a[j] += eps
            b = base[l].copy(); b[j] -= eps
            fd = (_oracle_loss(rho, L, p, {**tables, l: (a, 4 * p - 1)}, target)
                  - _oracle_loss(rho, L, p, {**tables, l: (b, 4 * p - 1)}, target)) / (2 * eps)
            print("level", l, "entry", j, "gpu", g[j], "fd", fd)
            assert abs(g[j] - fd) <= 1e-3 * abs(fd)
    # weights: a few of each layer
    def loss_of(th):
        tb = {}
        for l in (2, 3):
            tab, J = ofmm.m2l_table("S1", N, l, p)
            tab[J, J, J] = 0.0
            tb[l] = (omlp.corrected_table(tab, l, p, th), J)
        return _oracle_loss(rho, L, p, tb, target)
    for k in (3, omlp.O_B1 + 10, omlp.O_W2 + 16, omlp.O_B2 + 1, omlp.O_W3 + 6, omlp.O_B3):
        eps = 1e-4
        a = th64.copy(); a[k] += eps
        b = th64.copy(); b[k] -= eps
        fd = (loss_of(a) - loss_of(b)) / (2 * eps)
        print("weight", k, "gpu", wg[k], "fd", fd)
        assert abs(wg[k] - fd) <= 1e-3 * abs(fd) + 1e-6 * np.abs(wg).max()


def test_fallback_and_inference():
    import torch
    from paper_2011_07099_amd.learned import init_weights
    from paper_2011_07099_amd.pfmm import Plan
    N, L, p = 32, 3, 6
    rho = torch.from_numpy(f32(fields.lognormal(N, 2.0, 1.0, seed=32)).astype(np.float32)).cuda()
    outs = []
    with Plan(N, L, p, "S1") as pl:
        for w in (None, init_weights(1), None):
            pl.set_learned(w)
            phi = torch.empty_like(rho)
            pl.solve(rho, phi)
            outs.append(phi.cpu())
        th = init_weights(2)
        th[omlp.O_W3:omlp.O_B3] = 100.0
        pl.set_learned(th)
        t64 = pl.level_table(3).cpu().numpy()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    # BF16 inference of the same network on the device vs the FP64 oracle network
    tab, J = ofmm.m2l_table("S1", N, 3, p)
    ref = omlp.corrected_table(tab, 3, p, th.astype(np.float64)).ravel()
    ok = np.isfinite(ref)
    rel = np.abs(t64[ok] - ref[ok]) / np.abs(ref[ok])
    print("bf16 inference table rel err", rel.max())
    # bf16 weights and activations give the network output to ~2^-7 of its
    # size; the tables differ from the FP64 oracle by that times kappa |f|
    dmax = np.max(np.abs(ref[ok] / tab.ravel()[ok] - 1))
    print("max |delta|", dmax)
    assert rel.max() < 1e-2 * dmax


def test_training_reduces_loss_and_reports_gain_on_unseen_fields():
    # G_S1 is close to the best interaction-zone table at p = 6 (a uniform
    # relative change of 1e-4 of the level-2 table raises the loss 60x), so
    # the attainable gain is small; the test requires that training lowers
    # the training loss, that the trained network does not hurt unseen fields
    # by more than 0.1 % of their error, and reports the gain.
    import torch
    from paper_2011_07099_amd.learned import train
    from paper_2011_07099_amd.pfmm import Plan
    N, L, p = 64, 3, 6
    w, hist = train(N=N, L=L, p=p, n_fields=24, epochs=6, batch=8, lr=3e-4, seed0=40000)
    print("training loss before / after", hist[0], hist[-1])
    assert hist[-1] < hist[0]
    errs = {}
    for name, weights in (("G_S1", None), ("learned", w)):
        e = []
        with Plan(N, L, p, "S1") as pl:
            pl.set_learned(weights)
            for i in range(4):
                rho = f32(fields.lognormal(N, 2.0, 1.0, seed=50000 + i))
                r = torch.from_numpy(rho.astype(np.float32)).cuda()
                phi = torch.empty_like(r)
                pl.solve(r, phi)
                e.append(_loss(phi.cpu().numpy().astype(np.float64), conv.pm(rho, "S1")))
        errs[name] = float(np.mean(e))
    gain = errs["G_S1"] / errs["learned"]
    print("unseen mean relative L2^2 error", errs, "gain", gain)
    assert errs["learned"] <= errs["G_S1"] * (1 + 1e-3)


def test_output_layer_fit_gains_on_unseen_fields():
    # 16 training fields of 64^3 at p = 6, the hidden layers at their random
    # initialisation (first-layer scale 8), the output layer solved exactly;
    # measured gains 1.034 (64^3) and 1.029 (128^3), at the level of the
    # grid-valued tables' 1.027 with 2 x 2600 free values
    import torch
    from paper_2011_07099_amd.learned import fit_output
    from paper_2011_07099_amd.pfmm import Plan
    L, p = 3, 6
    w, info = fit_output(N=64, L=L, p=p, n_fields=16, n_valid=8, seed0=40000, seed=0)
    print("output-layer fit:", {k: v for k, v in info.items() if k != "fits"})
    assert info["ridge"] is not None
    gains = {}
    for N, n, seed0 in ((64, 4, 50000), (128, 2, 60000)):
        errs = {}
        for name, weights in (("G_S1", None), ("learned", w)):
            e = []
            with Plan(N, L, p, "S1") as pl:
                pl.set_learned(weights)         # BF16 inference
                for i in range(n):
                    rho = f32(fields.lognormal(N, 2.0, 1.0, seed=seed0 + i))
                    r = torch.from_numpy(rho.astype(np.float32)).cuda()
                    phi = torch.empty_like(r)
                    pl.solve(r, phi)
                    e.append(_loss(phi.cpu().numpy().astype(np.float64), conv.pm(rho, "S1")))
            errs[name] = float(np.mean(e))
        gains[N] = errs["G_S1"] / errs["learned"]
        print("%d^3 unseen: %s, gain %.4f" % (N, errs, gains[N]))
    assert gains[64] > 1.01 and gains[128] > 1.005
