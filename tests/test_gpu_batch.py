"""Batches of independent fields (mixed N and p) in one persistent launch
under a captured HIP graph, against the CPU FP64 reference FMM per field.

The batch runs every contraction in FP32 with FP64 per-offset running totals
(coarse levels included), so the FP32 tolerance of the single-field tests
applies with a 2x margin for the FP32 coarse levels: 2e-5 of max|phi|."""
import os

import numpy as np
import pytest

from oracle import fmm as ofmm
from paper_2011_07099_amd import fields

from gpu_util import f32, rel_max

pytestmark = pytest.mark.gpu

BATCH_TOL = 2e-5

SPECS = [  # (N, L, p, green, seed)
    (32, 3, 4, "S1", 101), (32, 3, 8, "X", 102), (64, 3, 6, "S1", 103),
    (16, 2, 4, "K", 104), (64, 3, 8, "S1", 105), (32, 2, 6, "S1", 106),
]


def _make(specs):
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    plans, rhos, phis, host = [], [], [], []
    for N, L, p, g, seed in specs:
        rho = f32(fields.lognormal(N, 2.0, 1.0, seed=seed))
        host.append(rho)
        plans.append(Plan(N, L, p, g))
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
    assert info["tile_width"] in (1, 2, 4) and info["items"] > 0
    for (N, L, p, g, seed), phi, rho in zip(SPECS, phis, host):
        ref = ofmm.fmm(rho, L, p, g)
        e = rel_max(phi.cpu().numpy().astype(np.float64), ref)
        print("batch field", (N, L, p, g), "rel max", e)
        assert e < BATCH_TOL
    for pl in plans:
        pl.close()


def test_graph_replays_match_with_eager_work_between():
    import torch
    from paper_2011_07099_amd.pfmm import Batch, Plan
    plans, rhos, phis, host = _make(SPECS[:4])
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
    for (N, L, p, g, seed), phi, rho in zip(SPECS[:4], outs[0], host):
        e = rel_max(phi.numpy().astype(np.float64), ofmm.fmm(rho, L, p, g))
        assert e < BATCH_TOL
    other.close()
    for pl in plans:
        pl.close()


def test_tuning_cache_round_trip(tmp_path, monkeypatch):
    import torch
    from paper_2011_07099_amd.pfmm import Batch
    path = tmp_path / "tune.json"
    monkeypatch.setenv("PFMM_TUNE_CACHE", str(path))
    plans, rhos, phis, host = _make(SPECS[:3])
    with Batch(plans, rhos, phis) as b:
        first = b.info()
    assert path.exists() and min(first["tuned_ms"]) > 0
    with Batch(plans, rhos, phis) as b:
        second = b.info()
        b.solve()
        torch.cuda.synchronize()
    print("tuned", first, "cached", second, path.read_text())
    assert second["tile_width"] == first["tile_width"]
    assert max(second["tuned_ms"]) < 0          # taken from the cache, not timed
    for pl in plans:
        pl.close()
