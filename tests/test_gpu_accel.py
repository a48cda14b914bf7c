"""Accelerations taken from the expansion on the GPU (Sec. 3: the FMM's
accelerations come from its expansion, PM's from differencing its potential),
through the C ABI, against the oracle's ``fmm_accel``: the far part is the
gradient of each leaf's local expansion, the near part sums each source
cell's differenced-G acceleration over the 27 leaves.

* Periodic and isolated plans, FP32 and split precision, the portable near
  zone (s < 8) and the 8^3-sub-block matrix-core near zone (s >= 8), FP32 and
  FP64 leaf levels.  Tolerance: FP32 rounding of the near-zone sums and of
  the interpolant gradient, 2e-5 of max|g| (FP32) and 2e-4 (split; the near
  kernels' values are held as three bf16 terms, the sources as two).
* G_S with a free a_2: the a_1 = -25/128, a_2 = 3/128 variant (the map
  t + O(t^7)) against the oracle's G_S with the same coefficients.
"""
import numpy as np
import pytest

from oracle import fmm as ofmm
from paper_2011_07099_amd import fields

from gpu_util import f32, rel_max, solve

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,L,p,prec,iso,f64,tol", [
    (32, 3, 4, "fp32", False, None, 2e-5),
    (32, 2, 6, "fp32", True, None, 2e-5),
    (64, 3, 8, "fp32", False, 2, 2e-5),
    (64, 3, 8, "bf16x3", False, None, 2e-4),
    (64, 3, 8, "bf16x3", True, None, 2e-4),
])
def test_expansion_accel_vs_oracle(N, L, p, prec, iso, f64, tol):
    rho = f32(fields.lognormal(N, 1.5, 1.0, seed=61 + N + p))
    green = "X" if iso else "S1"
    out = solve(rho, L, p, green, accel=True, precision=prec, isolated=iso,
                accel_mode="expansion", fp64_levels=f64)
    ref, ref_phi = ofmm.fmm_accel(rho, L, p, green, periodic=not iso)
    e = rel_max(out["accel"], ref)
    ep = rel_max(out["phi"], ref_phi)
    print("expansion accel", (N, L, p, prec, "isolated" if iso else "periodic", f64),
          "max err / max|g| = %.3e, potential %.3e" % (e, ep))
    assert e < tol and ep < tol


def test_gs_second_coefficient_t7_variant():
    N, L, p = 32, 3, 6
    rho = f32(fields.lognormal(N, 1.5, 1.0, seed=67))
    a = (-25.0 / 128.0, 3.0 / 128.0)
    out = solve(rho, L, p, "S", a1=a[0], a2=a[1], accel=True, accel_mode="expansion")
    ref, ref_phi = ofmm.fmm_accel(rho, L, p, "S", a=a)
    e, ep = rel_max(out["accel"], ref), rel_max(out["phi"], ref_phi)
    print("G_S t^7 variant: accel %.3e potential %.3e" % (e, ep))
    assert e < 2e-5 and ep < 2e-5


@pytest.mark.parametrize("N,L,p,green,a", [
    (32, 3, 8, "S1", None),    # s = 4 < p: the interpolant is evaluated between fewer cells
    (8, 3, 2, "S1", None),     # s = 1
    (32, 3, 5, "K", None),     # odd p, G_K
    (32, 3, 4, "E", (0.1,)),   # Ewald G_E
])
def test_expansion_accel_edge_cases(N, L, p, green, a):
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    rho = f32(fields.lognormal(N, 2.0, 1.0, seed=68 + N + p))
    r = torch.from_numpy(rho.astype(np.float32)).cuda()
    phi = torch.empty_like(r)
    acc = torch.empty((3, N, N, N), dtype=torch.float32, device="cuda")
    kw = {"rs": a[0]} if green == "E" else {}
    with Plan(N, L, p, green, accel="expansion", **kw) as pl:
        pl.solve(r, phi, acc)
        torch.cuda.synchronize()
    ref, _ = ofmm.fmm_accel(rho, L, p, green, a=a if a else (-0.125,))
    e = rel_max(acc.cpu().numpy().astype(np.float64), ref)
    print("expansion accel edge", (N, L, p, green), "%.3e" % e)
    assert e < 2e-5
