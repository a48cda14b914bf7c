"""Interaction zones as spectral stencils (per-node transforms on the 2p
cyclic grid, the zone's offsets summed per frequency, FP64), through the C
ABI, against the oracle's step-by-step FMM and the block-Toeplitz GEMM path.

* Locals of every level (Eq. 6 + Eq. 7) and the mesh potential against the
  reference FMM, periodic and isolated, p = 4, 6 and 8, G_S1, G_K and G_X.
  The FP32 levels' rounding sets the tolerance, 2e-5, as for the other M2L
  routes.  With every level kept in FP64 the spectral and GEMM locals differ
  by FP64 rounding only: their FP32 read-backs agree to 2e-7 of max.
* PFMM_OPT_ZONES_FP32 (the 16^3 leaf level's zones summed in FP32 columns
  with FP64 totals) at 128^3, L = 4, p = 4 and 6, under the same FP32
  tolerance: the FP32 roundings of the sources and kernel values
  (2^-24 each) over 189 offsets leave a few 1e-7 of the locals.
* The split-precision plan with spectral zones at the 256^3 headline size,
  with FP64 and with FP32 leaf columns, is covered by the headline parity
  test.
* Both transform routes together (FFT near zone and spectral zones) with
  accelerations from the expansion, periodic and isolated, against the
  oracle's fmm_accel (measured 1-6e-7; tolerance 2e-5).
* p = 5 is refused (p = 4, 6, 8 only; batches with spectral plans:
  test_gpu_batch.py).
"""
import numpy as np
import pytest

from oracle import fmm as ofmm
from paper_2011_07099_amd import fields

from gpu_util import f32, rel_max

pytestmark = pytest.mark.gpu


def _solve_stages(rho, L, p, green, m2l, fp64_levels=None, isolated=False, precision="fp32",
                  zones_fp32=False):
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    N = rho.shape[0]
    r = torch.from_numpy(np.ascontiguousarray(rho, dtype=np.float32)).cuda()
    phi = torch.empty_like(r)
    n = lambda l: 2 ** l
    with Plan(N, L, p, green, fp64_levels=fp64_levels, isolated=isolated, m2l=m2l,
              precision=precision, zones_fp32=zones_fp32) as pl:
        pl.solve(r, phi)
        Phi = {l: pl.locals(l).cpu().numpy().astype(np.float64).reshape((n(l),) * 3 + (p,) * 3)
               for l in range(2, L + 1)}
        torch.cuda.synchronize()
    return phi.cpu().numpy().astype(np.float64), Phi


@pytest.mark.parametrize("N,L,p,green,f64,iso,prec,zf", [
    (32, 3, 4, "S1", 0, False, "fp32", False),       # every level in FP32
    (64, 3, 8, "S1", None, False, "fp32", False),    # default FP64 levels 2-3
    (64, 3, 8, "S1", None, False, "bf16x3", False),  # split near zone beside spectral zones
    (128, 4, 4, "K", None, False, "fp32", False),
    (128, 4, 4, "K", None, False, "fp32", True),     # the 16^3 leaf level in FP32 columns
    (128, 4, 6, "S1", None, False, "fp32", True),    # the same at p = 6
    (64, 2, 8, "S1", None, False, "fp32", False),    # the smallest periodic tree
    (32, 3, 4, "X", None, True, "fp32", False),      # isolated twin (316-offset level 2)
    (64, 3, 8, "X", None, True, "fp32", False),
    (64, 3, 6, "S1", None, False, "fp32", False),    # p = 6: 12-point transforms, 1008 frequencies
    (128, 4, 6, "X", None, True, "fp32", False),     # p = 6 isolated, a 16^3 leaf level
])
def test_spectral_zones_match_reference_and_gemm(N, L, p, green, f64, iso, prec, zf):
    rho = f32(fields.lognormal(N, 2.0, 1.0, seed=281 + N + p))
    phi, Phi = _solve_stages(rho, L, p, green, "spectral", f64, iso, prec, zf)
    ref, st = ofmm.fmm(rho, L, p, green, stages=True, periodic=not iso)
    for l in range(2, L + 1):
        e = rel_max(Phi[l], st["Phi"][l])
        print("spectral zones", (N, L, p, green, iso), "Phi level", l, "%.3e" % e)
        assert e < 2e-5
    e = rel_max(phi, ref)
    g, _ = _solve_stages(rho, L, p, green, "gemm", f64, iso, prec)
    eg = rel_max(phi, g)
    print("spectral zones", (N, L, p, green, iso, prec, "FP32 leaf columns" if zf else "FP64"),
          "potential vs reference %.3e, vs GEMM path %.3e" % (e, eg))
    tol = 2e-5 if prec == "fp32" else 1e-4
    assert e < tol and eg < tol


@pytest.mark.parametrize("N,L,p,green,iso", [
    (32, 3, 4, "S1", False), (64, 3, 8, "K", False), (32, 3, 8, "X", True),
    (64, 3, 6, "S1", False),    # p = 6: direct 6-point DFTs, 96-entry twiddle table
    (128, 4, 6, "K", False),    # p = 6 periodic with a 16^3 leaf level (the two-target stencil)
])
def test_spectral_zones_in_fp64_match_the_fp64_gemm(N, L, p, green, iso):
    """Every level in FP64: the spectral and GEMM locals differ by FP64
    rounding only, so their FP32 read-backs agree to one FP32 rounding.  A
    wrong twiddle or a transform that aliases would show far above it."""
    rho = f32(fields.lognormal(N, 2.0, 1.0, seed=291 + N + p))
    _, Phi = _solve_stages(rho, L, p, green, "spectral", 30, iso)
    _, G = _solve_stages(rho, L, p, green, "gemm", 30, iso)
    for l in range(2, L + 1):
        e = rel_max(Phi[l], G[l])
        print("spectral vs GEMM zones, FP64 levels", (N, L, p, green, iso), "Phi level", l, "%.3e" % e)
        assert e < 2e-7


def test_spectral_zones_refusals():
    from paper_2011_07099_amd.pfmm import Plan, PfmmError
    with Plan(64, 3, 5, "S1") as pl:   # transforms for p = 4, 6, 8 only
        with pytest.raises(PfmmError):
            pl.set_m2l("spectral")


@pytest.mark.parametrize("N,L,p,iso", [(32, 3, 4, True), (64, 3, 8, False), (64, 4, 4, True)])
def test_spectral_zones_with_fft_near_zone_and_expansion_accel(N, L, p, iso):
    """Both transform routes together (FFT near zone, spectral zones), with
    accelerations from the expansion: potential and accelerations against the
    oracle's fmm_accel, periodic and isolated."""
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    green = "X" if iso else "S1"
    rho = f32(fields.lognormal(N, 1.5, 1.0, seed=301 + N + p))
    r = torch.from_numpy(rho.astype(np.float32)).cuda()
    phi = torch.empty_like(r)
    acc = torch.empty((3, N, N, N), dtype=torch.float32, device="cuda")
    with Plan(N, L, p, green, isolated=iso, accel="expansion", near="fft", m2l="spectral") as pl:
        pl.solve(r, phi, acc)
        torch.cuda.synchronize()
    ref, ref_phi = ofmm.fmm_accel(rho, L, p, green, periodic=not iso)
    e = rel_max(acc.cpu().numpy().astype(np.float64), ref)
    ep = rel_max(phi.cpu().numpy().astype(np.float64), ref_phi)
    print("FFT near zone + spectral zones + expansion accel", (N, L, p, iso),
          "max err / max|g| = %.3e, potential %.3e" % (e, ep))
    assert e < 2e-5 and ep < 2e-5
