"""Helpers shared by the GPU tests: run the HIP library on an FP64 density and
bring results back as NumPy arrays; error norms."""
import numpy as np


def f32(rho):
    """The density exactly as the GPU sees it (FP32), in FP64 for the oracle."""
    return np.asarray(rho, np.float32).astype(np.float64)


def solve(rho, L, p, green, accel=False, precision="fp32", a1=None, stages=False,
          fp64_levels=None, isolated=False, accel_mode="fd4", a2=None, near="direct",
          m2l="gemm", fold=False, zones_fp32=False):
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    N = rho.shape[0]
    r = torch.from_numpy(np.ascontiguousarray(rho, dtype=np.float32)).cuda()
    phi = torch.empty_like(r)
    acc = torch.empty((3, N, N, N), dtype=torch.float32, device="cuda") if accel else None
    out = {}
    with Plan(N, L, p, green, precision=precision, a1=a1, fp64_levels=fp64_levels,
              isolated=isolated, accel=accel_mode, a2=a2, near=near, m2l=m2l, fold=fold,
              zones_fp32=zones_fp32) as pl:
        pl.solve(r, phi, acc)
        if stages:
            n = lambda l: 2 ** l
            out["M"] = {l: pl.multipoles(l).cpu().numpy().astype(np.float64)
                        .reshape((n(l),) * 3 + (p,) * 3) for l in range(2, L + 1)}
            out["Phi"] = {l: pl.locals(l).cpu().numpy().astype(np.float64)
                          .reshape((n(l),) * 3 + (p,) * 3) for l in range(2, L + 1)}
        torch.cuda.synchronize()
        out["phi"] = phi.cpu().numpy().astype(np.float64)
        if accel:
            out["accel"] = acc.cpu().numpy().astype(np.float64)
    return out


def rel_max(a, ref):
    """max |a - ref| / max |ref|"""
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def rel_l2(a, ref, remove_mean=False):
    if remove_mean:
        a = a - a.mean()
        ref = ref - ref.mean()
    return float(np.sqrt(np.sum((a - ref) ** 2) / np.sum(ref ** 2)))
