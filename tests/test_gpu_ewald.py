"""The Ewald Green's function G_E (Sec. 1) in the library, through the C ABI,
against the oracle's G_E (pinned there by Ewald's identity).

* Level and near tables (FP64 on the device, the Fourier part damped by
  exp(-k^2 r_S^2/4), the real-space part erfc-screened): 1e-12 relative, at
  two splitting radii, after changing r_S on a live plan.
* Two levels with gridlet = leaf: the FMM equals PM with G_E (FP32 rounding,
  1e-5 of max|phi|), as for every G.
* A 3-level FMM with G_E against the reference FMM.
* The direct periodic solve of a plan (pfmm_plan_direct) follows a change of
  the Green's function's parameter (G_S a_1, G_E r_S).
"""
import numpy as np
import pytest

from oracle import conv, fmm as ofmm
from paper_2011_07099_amd import fields

from gpu_util import f32, rel_max

pytestmark = pytest.mark.gpu


def _white(N, seed):
    r = np.random.default_rng(seed).standard_normal((N, N, N))
    return r - r.mean()


@pytest.mark.parametrize("N,L,p", [(32, 3, 4), (64, 3, 6)])
def test_ewald_tables_match_oracle(N, L, p):
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    with Plan(N, L, p, "E") as pl:
        for rs in (0.1, 0.07):
            pl.set_ewald_rs(rs)
            for l in range(2, L + 1):
                got = pl.level_table(l).cpu().numpy().reshape((8 * p - 1,) * 3)
                ref, J = ofmm.m2l_table("E", N, l, p, (rs,))
                ok = np.isfinite(ref)
                ok[J, J, J] = False
                err = np.max(np.abs(got[ok] - ref[ok])) / np.max(np.abs(ref[ok]))
                print("G_E r_S", rs, N, "level", l, "table rel err", err)
                assert err < 1e-12
            got = pl.near_table().cpu().numpy().reshape((4 * pl.s - 1,) * 3)
            torch.cuda.synchronize()
            ref, _ = ofmm.near_table("E", N, N >> L, (rs,))
            err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
            print("G_E r_S", rs, N, "near table rel err", err)
            assert err < 1e-12


def _solve(rho, L, p, green, **kw):
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    N = rho.shape[0]
    r = torch.from_numpy(np.ascontiguousarray(rho, dtype=np.float32)).cuda()
    phi = torch.empty_like(r)
    with Plan(N, L, p, green, **kw) as pl:
        pl.solve(r, phi)
        torch.cuda.synchronize()
    return phi.cpu().numpy().astype(np.float64)


def test_ewald_two_levels_gridlet_equals_leaf_is_direct():
    rho = f32(_white(32, 71))
    gpu = _solve(rho, 2, 8, "E", rs=0.08)
    e = rel_max(gpu, conv.pm(rho, "E", (0.08,)))
    print("G_E L=2 s=p vs PM(G_E)", e)
    assert e < 1e-5


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x3", 1e-4)])
def test_ewald_fmm_matches_reference(prec, tol):
    rho = f32(fields.lognormal(64, 2.0, 1.0, seed=72))
    gpu = _solve(rho, 3, 8, "E", rs=0.1, precision=prec)
    ref = ofmm.fmm(rho, 3, 8, "E", (0.1,))
    e = rel_max(gpu, ref)
    print("G_E 64^3 L=3 p=8", prec, "vs reference FMM", e)
    assert e < tol


def test_direct_solve_follows_the_green_parameter():
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    N = 16
    rho = f32(_white(N, 73))
    r = torch.from_numpy(rho.astype(np.float32)).cuda()
    out = torch.empty_like(r)
    for green, setter, values, ref_a in [
            ("S", "set_a1", (-0.125, -0.14), lambda v: (v,)),
            ("E", "set_ewald_rs", (0.1, 0.06), lambda v: (v,))]:
        with Plan(N, 2, 4, green) as pl:
            for v in values:
                getattr(pl, setter)(v)
                pl.direct(r, out)
                torch.cuda.synchronize()
                e = rel_max(out.cpu().numpy().astype(np.float64), conv.pm(rho, green, ref_a(v)))
                print("direct solve", green, setter, v, e)
                assert e < 1e-5
