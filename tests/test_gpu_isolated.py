"""The non-periodic twin on the GPU (Sec. 3, Eq. 3: the FMM with the
free-space G_0 and no periodic images, used to separate the expansion error
from the Green's-function error), through the C ABI, against the oracle's
twin.

* Two levels with gridlet = leaf (s = p): the twin equals the direct
  isolated sum (zero-padded FFT) up to FP32 rounding (1e-5 of max|phi|).
* The potential against the oracle's non-periodic FMM, FP32 (1e-5) and split
  precision (1e-4), with every zone clipped at the box: the level-2 zone of
  316 offsets on the FP64 matrix cores (p = 8) or the portable kernel, the
  near zone with and without 8^3-cell sub-blocks, a leaf level on the split
  kernel (128^3, L = 4).  At 128^3 on 4096 sampled cells (every in-leaf
  position, box faces and corners included).
* The option needs G_X; batches refuse isolated plans.
"""
import numpy as np
import pytest

from oracle import conv, fmm as ofmm
from paper_2011_07099_amd import fields

from gpu_util import f32, rel_max, solve

pytestmark = pytest.mark.gpu


def test_isolated_two_levels_gridlet_equals_leaf_is_direct():
    rho = f32(fields.lognormal(32, 2.0, 1.0, seed=51))
    gpu = solve(rho, 2, 8, "X", isolated=True)["phi"]
    e = rel_max(gpu, conv.isolated(rho))
    print("isolated 32^3 L=2 s=p vs direct isolated sum", e)
    assert e < 1e-5


@pytest.mark.parametrize("N,L,p,prec,tol", [
    (32, 3, 4, "fp32", 1e-5),
    (64, 3, 8, "fp32", 1e-5),
    (64, 3, 8, "bf16x3", 1e-4),
    (64, 3, 6, "bf16x3", 1e-4),
])
def test_isolated_matches_oracle_twin(N, L, p, prec, tol):
    rho = f32(fields.lognormal(N, 2.0, 1.0, seed=52 + N + p))
    gpu = solve(rho, L, p, "X", precision=prec, isolated=True)["phi"]
    e = rel_max(gpu, ofmm.fmm(rho, L, p, periodic=False))
    print("isolated", (N, L, p, prec), "vs oracle twin", e)
    assert e < tol


def test_isolated_128_sampled_including_faces():
    N, L, p = 128, 4, 8
    rho = f32(fields.lognormal(N, 1.5, 2.0, seed=57))
    s = N >> L
    k = np.arange(N // s)
    c = s * k + (3 * k + 7) % s            # every in-leaf position on each axis
    c[0], c[-1] = 0, N - 1                  # the box's own faces
    tg = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    ref = ofmm.fmm(rho, L, p, periodic=False, targets=tg)
    for prec, tol in (("fp32", 1e-5), ("bf16x3", 1e-4)):
        gpu = solve(rho, L, p, "X", precision=prec, isolated=True)["phi"]
        got = gpu[tg[:, 0], tg[:, 1], tg[:, 2]]
        e = np.max(np.abs(got - ref)) / np.max(np.abs(gpu))
        print("isolated 128^3 L=4", prec, "sampled vs oracle twin", e)
        assert e < tol


def test_isolated_option_rules():
    import torch
    from paper_2011_07099_amd.pfmm import Batch, PfmmError, Plan
    with Plan(32, 3, 4, "S1") as pl:
        with pytest.raises(PfmmError) as ex:
            pl.set_isolated(True)
        assert ex.value.status == 2
    rho = torch.zeros((32, 32, 32), dtype=torch.float32, device="cuda")
    phi = torch.empty_like(rho)
    with Plan(32, 3, 4, "X", isolated=True) as pl:
        with pytest.raises(PfmmError) as ex:
            Batch([pl], [rho], [phi])
        assert ex.value.status == 2
        pl.set_isolated(False)          # back to the periodic G_X plan
        pl.solve(rho, phi)
        torch.cuda.synchronize()
        assert torch.count_nonzero(phi).item() == 0
