"""The HPM interaction zones by FFT convolution (the M2L the paper runs,
Sec. 2), through the C ABI, against the oracle's step-by-step FMM and the
library's own block-Toeplitz GEMM path.

* Gridlet potentials of every level (Eq. 6 + Eq. 7) and the mesh potential
  against the reference FMM: level 2 on the periodic (4p)^3 grid, levels >= 3
  on zero-padded (8p)^3 grids, one per target, batched; FP64 transforms for
  the levels the plan keeps in FP64 (2-3 by default), FP32 for the rest, and
  one case with every level in FP32.  Tolerance 2e-5 of the largest value
  (FP32 FFT rounding grows like log(M^3) over the grid; the zone sums cancel
  10^2-10^3 fold).
* The same solve through the GEMM path agrees to the same tolerance.
* Options the FFT path does not serve are refused: isolated plans, batches.
"""
import numpy as np
import pytest

from oracle import fmm as ofmm
from paper_2011_07099_amd import fields

from gpu_util import f32, rel_max

pytestmark = pytest.mark.gpu


def _solve_stages(rho, L, p, green, m2l, fp64_levels=None):
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    N = rho.shape[0]
    r = torch.from_numpy(np.ascontiguousarray(rho, dtype=np.float32)).cuda()
    phi = torch.empty_like(r)
    n = lambda l: 2 ** l
    with Plan(N, L, p, green, fp64_levels=fp64_levels, m2l=m2l) as pl:
        pl.solve(r, phi)
        Phi = {l: pl.locals(l).cpu().numpy().astype(np.float64).reshape((n(l),) * 3 + (p,) * 3)
               for l in range(2, L + 1)}
        torch.cuda.synchronize()
    return phi.cpu().numpy().astype(np.float64), Phi


@pytest.mark.parametrize("N,L,p,green,f64", [
    (32, 3, 4, "S1", 0),
    (64, 3, 6, "X", None),
    (64, 3, 8, "S1", None),
    (128, 4, 4, "K", None),
    (64, 2, 8, "S1", None),
    (32, 3, 3, "X", None),     # odd p: 24^3 grids at levels >= 3
    (32, 3, 5, "S1", 0),       # odd p, every level in FP32
    (16, 2, 2, "K", None),     # the smallest tree
])
def test_fft_zones_match_reference_and_gemm(N, L, p, green, f64):
    rho = f32(fields.lognormal(N, 2.0, 1.0, seed=81 + N + p))
    phi, Phi = _solve_stages(rho, L, p, green, "fft", f64)
    ref, st = ofmm.fmm(rho, L, p, green, stages=True)
    for l in range(2, L + 1):
        e = rel_max(Phi[l], st["Phi"][l])
        print("FFT zones", (N, L, p, green), "Phi level", l, "%.3e" % e)
        assert e < 2e-5
    e = rel_max(phi, ref)
    g, _ = _solve_stages(rho, L, p, green, "gemm", f64)
    eg = rel_max(phi, g)
    print("FFT zones", (N, L, p, green), "potential vs reference %.3e, vs GEMM path %.3e" % (e, eg))
    assert e < 2e-5 and eg < 2e-5


def test_fft_zones_refuse_isolated_and_batches():
    import torch
    from paper_2011_07099_amd.pfmm import Batch, Plan, PfmmError
    with Plan(32, 3, 4, "X", m2l="fft") as pl:
        with pytest.raises(PfmmError):
            pl.set_isolated(True)
        r = torch.zeros((32, 32, 32), device="cuda")
        out = torch.empty_like(r)
        with pytest.raises(PfmmError):
            Batch([pl], [r], [out])
    with Plan(32, 3, 4, "X", isolated=True) as pl:
        with pytest.raises(PfmmError):
            pl.set_m2l("fft")
