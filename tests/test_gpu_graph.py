"""A single pfmm_solve captured into a HIP graph from the plan's stream (the
header's promise: the whole solve, near zone on the plan's second stream
included through its event fork and join, is ordered on the plan's stream and
allocates nothing).  The graph is replayed several times with another plan's
eager solve and a device synchronisation between replays; every replay must
equal the eager solve bit for bit, potential and accelerations, in FP32 and
in split precision.
"""
import numpy as np
import pytest

from paper_2011_07099_amd import fields

from gpu_util import f32

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_solve_replays_from_a_graph_bit_for_bit(prec):
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    N, L, p = 64, 3, 8
    rho = torch.from_numpy(f32(fields.lognormal(N, 2.0, 1.0, seed=95)).astype(np.float32)).cuda()
    s = torch.cuda.Stream()
    phi_e = torch.empty_like(rho)
    acc_e = torch.empty((3, N, N, N), dtype=torch.float32, device="cuda")
    phi = torch.empty_like(rho)
    acc = torch.empty_like(acc_e)
    other_out = torch.empty_like(rho)
    with Plan(N, L, p, "S1", precision=prec, stream=s) as pl, Plan(N, 3, 4, "X") as other:
        with torch.cuda.stream(s):
            pl.solve(rho, phi_e, acc_e)       # eager reference (and warm-up)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            pl.solve(rho, phi, acc)
        torch.cuda.synchronize()
        for rep in range(4):
            phi.fill_(float("nan"))
            acc.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            same = torch.equal(phi, phi_e) and torch.equal(acc, acc_e)
            print(prec, "graph replay", rep, "bit-identical to the eager solve:", same)
            assert same
            other.solve(rho, other_out)       # unrelated eager work between replays
            torch.cuda.synchronize()
