"""Batches of independent fields (mixed N, p, G and precision) under a
captured HIP graph, against the CPU FP64 reference FMM per field.

Work goes to three persistent kernels: the portable one (FP32 contractions
with FP64 per-offset running totals; FP64 levels in FP64), the BF16 split
matrix-core kernel (near zones of split-precision plans with 8^3-cell
sub-blocks) and the FP64 matrix-core kernel (FP64 levels at p = 8).  FP32
fields keep the single-field FP32 tolerance with a 2x margin, 2e-5 of
max|phi|; split-precision fields the single-field split tolerance, 1e-4."""
import os

import numpy as np
import pytest

from oracle import fmm as ofmm
from paper_2011_07099_amd import fields

from gpu_util import f32, rel_max

pytestmark = pytest.mark.gpu

BATCH_TOL = 2e-5
SPLIT_TOL = 1e-4

SPECS = [  # (N, L, p, green, seed)
    (32, 3, 4, "S1", 101), (32, 3, 8, "X", 102), (64, 3, 6, "S1", 103),
    (16, 2, 4, "K", 104), (64, 3, 8, "S1", 105), (32, 2, 6, "S1", 106),
]


def _make(specs, precision="fp32"):
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    plans, rhos, phis, host = [], [], [], []
    for spec in specs:
        N, L, p, g, seed = spec[:5]
        rho = f32(fields.lognormal(N, 2.0, 1.0, seed=seed))
        host.append(rho)
        plans.append(Plan(N, L, p, g, precision=spec[5] if len(spec) > 5 else precision,
                          near=spec[6] if len(spec) > 6 else "direct",
                          m2l=spec[7] if len(spec) > 7 else "gemm"))
        rhos.append(torch.from_numpy(rho.astype(np.float32)).cuda())
        phis.append(torch.full_like(rhos[-1], float("nan")))
    return plans, rhos, phis, host


def test_batch_fields_match_reference_fmm():
    import torch
    from paper_2011_07099_amd.pfmm import Batch
    plans, rhos, phis, host = _make(SPECS)
    with Batch(plans, rhos, phis) as b:
        b.solve()
        torch.cuda.synchronize()
        info = b.info()
    print("batch info", info)
    assert info["items"] > 0 and all(g["width"] in (1, 2, 4) for g in info["groups"])
    for (N, L, p, g, seed), phi, rho in zip(SPECS, phis, host):
        ref = ofmm.fmm(rho, L, p, g)
        e = rel_max(phi.cpu().numpy().astype(np.float64), ref)
        print("batch field", (N, L, p, g), "rel max", e)
        assert e < BATCH_TOL
    for pl in plans:
        pl.close()


SPLIT_SPECS = [  # (N, L, p, green, seed, precision)
    (64, 3, 8, "S1", 201, "bf16x3"),    # split near zone, 8^3 leaves; FP64 levels on the matrix cores
    (128, 3, 8, "S1", 202, "bf16x3"),   # split near zone, 16^3 leaves as 2^3 sub-blocks per leaf
    (64, 3, 6, "S1", 203, "bf16x3"),    # split near zone; p = 6 levels in the portable kernel
    (32, 3, 8, "X", 204, "bf16x3"),     # 4^3 leaves: portable near zone
    (64, 3, 8, "K", 205, "fp32"),       # FP32 plan in the same batch
]


def test_matrix_core_items_match_reference_fmm():
    import torch
    from paper_2011_07099_amd.pfmm import Batch
    plans, rhos, phis, host = _make(SPLIT_SPECS)
    with Batch(plans, rhos, phis) as b:
        b.solve()
        torch.cuda.synchronize()
        info = b.info()
    print("batch info", info)
    for (N, L, p, g, seed, prec), phi, rho in zip(SPLIT_SPECS, phis, host):
        ref = ofmm.fmm(rho, L, p, g)
        e = rel_max(phi.cpu().numpy().astype(np.float64), ref)
        print("batch field", (N, L, p, g, prec), "rel max", e)
        assert e < (SPLIT_TOL if prec == "bf16x3" else BATCH_TOL)
    for pl in plans:
        pl.close()


def test_graph_replays_match_with_eager_work_between():
    import torch
    from paper_2011_07099_amd.pfmm import Batch, Plan
    specs = SPECS[:4] + SPLIT_SPECS[:1]
    plans, rhos, phis, host = _make(specs)
    other = Plan(32, 3, 4, "S1")
    orho = torch.from_numpy(f32(fields.lognormal(32, 2.0, 1.0, seed=7)).astype(np.float32)).cuda()
    ophi = torch.empty_like(orho)
    with Batch(plans, rhos, phis) as b:
        outs = []
        for r in range(4):
            for f in phis:
                f.fill_(float("nan"))
            b.solve()
            other.solve(orho, ophi)          # eager work between replays
            torch.cuda.synchronize()
            outs.append([f.cpu().clone() for f in phis])
    for r in range(1, 4):
        for a, c in zip(outs[0], outs[r]):
            assert torch.equal(a, c)
    for spec, phi, rho in zip(specs, outs[0], host):
        N, L, p, g = spec[:4]
        e = rel_max(phi.numpy().astype(np.float64), ofmm.fmm(rho, L, p, g))
        assert e < (SPLIT_TOL if spec[5:] == ("bf16x3",) else BATCH_TOL)
    other.close()
    for pl in plans:
        pl.close()


def test_tuning_cache_round_trip(tmp_path, monkeypatch):
    """Each FP32 group of portable items is tuned on its own items; the choice
    goes to the cache and the next batch of the same groups reads it back."""
    import json
    import torch
    from paper_2011_07099_amd.pfmm import Batch
    path = tmp_path / "tune.json"
    monkeypatch.setenv("PFMM_TUNE_CACHE", str(path))
    plans, rhos, phis, host = _make(SPECS[:3])
    with Batch(plans, rhos, phis) as b:
        first = b.info()
    cached = json.loads(path.read_text())
    print("tuned", first, "cache", cached)
    f32 = [g for g in first["groups"] if not g["fp64"]]
    assert f32, first
    for g in first["groups"]:
        key = "batch-q%d-f32-%s" % (g["q"], "near" if g["near"] else "zone")
        if g["fp64"]:
            assert g["width"] == 1 and min(g["ms"]) < 0
        else:
            assert min(g["ms"]) > 0 and g["width"] in (1, 2, 4)
            assert g["ms"][(1, 2, 4).index(g["width"])] == min(g["ms"])
            assert cached[key] == g["width"]
    with Batch(plans, rhos, phis) as b:
        second = b.info()
        b.solve()
        torch.cuda.synchronize()
    for g1, g2 in zip(first["groups"], second["groups"]):
        assert g1["width"] == g2["width"] and (g2["fp64"] or max(g2["ms"]) < 0)
    for (N, L, p, g, seed), phi, rho in zip(SPECS[:3], phis, host):
        assert rel_max(phi.cpu().numpy().astype(np.float64), ofmm.fmm(rho, L, p, g)) < BATCH_TOL
    for pl in plans:
        pl.close()


FFT_SPECS = [  # (N, L, p, green, seed, precision, near zone)
    (64, 3, 8, "S1", 301, "bf16x3", "fft"),   # 8^3 leaves
    (128, 3, 8, "S1", 302, "bf16x3", "fft"),  # 16^3 leaves
    (32, 3, 4, "S1", 303, "fp32", "fft"),     # 4^3 leaves
    (64, 3, 6, "K", 304, "fp32", "fft"),
    (64, 3, 8, "X", 305, "bf16x3", "direct"),  # a direct near zone in the same batch
]


def test_fft_near_zone_fields_in_batches():
    """Plans with the FFT near zone in a batch: their per-leaf transforms and
    stencil run in the batch graph beside the persistent kernels; every field
    against the reference FMM, and two graph launches bit for bit."""
    import torch
    from paper_2011_07099_amd.pfmm import Batch
    plans, rhos, phis, host = _make(FFT_SPECS)
    with Batch(plans, rhos, phis) as b:
        outs = []
        for r in range(2):
            for f in phis:
                f.fill_(float("nan"))
            b.solve()
            torch.cuda.synchronize()
            outs.append([f.cpu().clone() for f in phis])
    for a, c in zip(outs[0], outs[1]):
        assert torch.equal(a, c)
    for spec, phi, rho in zip(FFT_SPECS, outs[0], host):
        N, L, p, g, seed, prec, near = spec
        e = rel_max(phi.numpy().astype(np.float64), ofmm.fmm(rho, L, p, g))
        print("batch field", spec, "rel max", e)
        assert e < (SPLIT_TOL if prec == "bf16x3" else BATCH_TOL)
    for pl in plans:
        pl.close()


SPECTRAL_SPECS = [  # (N, L, p, green, seed, precision, near zone, interaction zones)
    (64, 3, 8, "S1", 401, "bf16x3", "fft", "spectral"),
    (128, 3, 8, "S1", 402, "fp32", "fft", "spectral"),
    (32, 3, 4, "S1", 403, "fp32", "direct", "spectral"),
    (64, 3, 4, "X", 405, "bf16x3", "direct", "spectral"),  # split direct near zone
    (64, 3, 6, "K", 404, "fp32", "fft", "gemm"),            # zones as work items
    (32, 3, 6, "S1", 406, "fp32", "fft", "spectral"),      # p = 6 spectral
]


def test_spectral_zone_fields_in_batches():
    """Plans with spectral interaction zones in a batch: their levels run as
    the plan's own launches in the graph (zone sums written, parents added by
    the downward passes); every field against the reference FMM, two graph
    launches bit for bit."""
    import torch
    from paper_2011_07099_amd.pfmm import Batch
    plans, rhos, phis, host = _make(SPECTRAL_SPECS)
    with Batch(plans, rhos, phis) as b:
        outs = []
        for r in range(2):
            for f in phis:
                f.fill_(float("nan"))
            b.solve()
            torch.cuda.synchronize()
            outs.append([f.cpu().clone() for f in phis])
    for a, c in zip(outs[0], outs[1]):
        assert torch.equal(a, c)
    for spec, phi, rho in zip(SPECTRAL_SPECS, outs[0], host):
        N, L, p, g, seed, prec, near, m2l = spec
        e = rel_max(phi.numpy().astype(np.float64), ofmm.fmm(rho, L, p, g))
        print("batch field", spec, "rel max", e)
        assert e < (SPLIT_TOL if (prec == "bf16x3" and near == "direct") else BATCH_TOL)
    for pl in plans:
        pl.close()
