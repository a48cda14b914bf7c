"""The leaf near zone by FFT convolution on the doubled grid (the route the
paper takes for a leaf's near zone, Sec. 2-3), through the C ABI.

* Mesh potential against the oracle's step-by-step FMM (direct near-zone
  sum) and against the library's direct near zone, periodic and isolated,
  leaf edges s = 1 .. 16, several G, FP32 and split precision for the rest of
  the tree.  Tolerance 2e-5 of max|phi|: FP32 rounding of (2s)^3 transforms
  (grows like log s) on top of the FP32 tree.
* PFMM_OPT_FOLD (P2M inside the forward transform, L2P inside the
  potential's inverse transform; library transforms at s = 8, 16 with
  p = 4, 8 and an FP32 leaf level): periodic and isolated cases at s = 8
  with p = 4 and 8, with and without expansion accelerations, and s = 16
  with p = 4 at sampled cells that run through every position inside a leaf
  (s = 16 with p = 8 is the headline test's).
* Accelerations from the expansion, whose three near-zone kernels reuse the
  forward transforms, against the oracle's ``fmm_accel``.
* Leaf and near-zone corner cases: one cell per leaf (s = 1, a 2^3 cyclic
  grid), the smallest periodic tree (4^3 leaves, where the +1 and -1
  neighbours of a leaf are distinct wrapped leaves), a density that is a single
  cell (the transformed kernel alone, including the self value), and zero.
* A solve with the FFT near zone captured into a HIP graph replays bit for
  bit; batches refuse such plans when the leaf transforms would be rocFFT's
  (s = 1, 2), and solves refuse buffers that are not 16-byte aligned (the
  leaf transforms move four cells per access).
"""
import numpy as np
import pytest

from oracle import fmm as ofmm
from paper_2011_07099_amd import fields

from gpu_util import f32, rel_max, solve

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,L,p,green,prec,iso,fold", [
    (32, 3, 4, "S1", "fp32", False, False),   # s = 4
    (64, 3, 8, "S1", "bf16x3", False, False),  # s = 8, split tree
    (64, 3, 8, "S1", "bf16x3", False, True),   # the same, P2M and L2P folded
    (64, 2, 8, "K", "fp32", False, False),     # s = 16, the smallest periodic tree
    (16, 4, 2, "X", "fp32", False, False),     # s = 1
    (32, 3, 4, "X", "fp32", True, False),      # isolated twin
    (64, 3, 6, "X", "fp32", True, False),
    (32, 4, 3, "S1", "fp32", False, False),    # s = 2, odd p
    (64, 3, 4, "S1", "fp32", False, True),     # s = 8, p = 4, folded
    (64, 3, 4, "X", "fp32", True, True),       # the same, isolated
])
def test_fft_near_zone_matches_reference_and_direct(N, L, p, green, prec, iso, fold):
    rho = f32(fields.lognormal(N, 1.5, 1.0, seed=171 + N + p))
    got = solve(rho, L, p, green, precision=prec, isolated=iso, near="fft", fold=fold)["phi"]
    ref = ofmm.fmm(rho, L, p, green, periodic=not iso)
    direct = solve(rho, L, p, green, precision=prec, isolated=iso)["phi"]
    e, ed = rel_max(got, ref), rel_max(got, direct)
    print("FFT near zone", (N, L, p, green, prec, "isolated" if iso else "periodic",
                            "folded" if fold else "separate P2M and L2P"),
          "vs reference %.3e, vs direct near zone %.3e" % (e, ed))
    tol = 2e-5 if prec == "fp32" else 1e-4
    assert e < tol and ed < tol


@pytest.mark.parametrize("N,L,p,prec,iso,fold", [
    (32, 3, 4, "fp32", False, False),
    (64, 3, 8, "bf16x3", False, False),
    (64, 3, 8, "bf16x3", False, True),
    (32, 2, 6, "fp32", True, False),
    (64, 3, 4, "fp32", True, False),   # isolated, 8^3 leaves
])
def test_fft_near_zone_expansion_accel(N, L, p, prec, iso, fold):
    rho = f32(fields.lognormal(N, 1.5, 1.0, seed=181 + N + p))
    green = "X" if iso else "S1"
    out = solve(rho, L, p, green, accel=True, precision=prec, isolated=iso,
                accel_mode="expansion", near="fft", fold=fold)
    ref, ref_phi = ofmm.fmm_accel(rho, L, p, green, periodic=not iso)
    e, ep = rel_max(out["accel"], ref), rel_max(out["phi"], ref_phi)
    print("FFT near zone, expansion accel", (N, L, p, prec, iso, fold),
          "max err / max|g| = %.3e, potential %.3e" % (e, ep))
    tol = 2e-5 if prec == "fp32" else 2e-4
    assert e < tol and ep < tol


def test_folded_p2m_l2p_at_16_cell_leaves_p4():
    N, L, p = 128, 3, 4
    s = N >> L
    rho = f32(fields.lognormal(N, 1.5, 1.0, seed=175))
    k = np.arange(N // s)
    # two cells per leaf and axis, together every position 0 .. 15
    c = np.concatenate([s * k + (7 * k + 15) % s, s * k + (7 * k + 15 + s // 2) % s])
    tg = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    assert len(np.unique(c % s)) == s
    got = solve(rho, L, p, "S1", near="fft", m2l="spectral", fold=True)["phi"]
    ref = ofmm.fmm(rho, L, p, "S1", targets=tg)
    e = np.max(np.abs(got[tg[:, 0], tg[:, 1], tg[:, 2]] - ref)) / np.max(np.abs(got))
    print("FFT near zone with P2M and L2P folded, s = 16, p = 4: sampled max err / max|phi| "
          "= %.3e" % e)
    assert e < 2e-5


def test_fft_near_zone_point_mass_and_zero():
    N, L, p = 32, 3, 4
    rho = np.zeros((N, N, N))
    rho[5, 30, 17] = 1.0
    got = solve(rho, L, p, "S1", near="fft")["phi"]
    ref = ofmm.fmm(rho, L, p, "S1")
    e = rel_max(got, ref)
    print("FFT near zone, single-cell density: %.3e" % e)
    assert e < 2e-5
    zero = solve(np.zeros((N, N, N)), L, p, "S1", near="fft")["phi"]
    assert np.all(zero == 0)


def test_fft_near_zone_graph_replay_and_batch_refusal():
    import torch
    from paper_2011_07099_amd.pfmm import Batch, Plan, PfmmError
    N, L, p = 64, 3, 8
    rho = torch.from_numpy(f32(fields.lognormal(N, 2.0, 1.0, seed=191)).astype(np.float32)).cuda()
    s = torch.cuda.Stream()
    phi_e = torch.empty_like(rho)
    phi = torch.empty_like(rho)
    other_out = torch.empty_like(rho)
    with Plan(N, L, p, "S1", precision="bf16x3", stream=s, near="fft") as pl, \
            Plan(N, 3, 4, "X") as other:
        with torch.cuda.stream(s):
            pl.solve(rho, phi_e)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            pl.solve(rho, phi)
        torch.cuda.synchronize()
        for rep in range(3):
            phi.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            same = torch.equal(phi, phi_e)
            print("FFT near zone graph replay", rep, "bit-identical:", same)
            assert same
            other.solve(rho, other_out)
            torch.cuda.synchronize()
    # batches take the FFT near zone only with the library's own transforms
    with Plan(16, 4, 2, "X", near="fft") as pl:   # one cell per leaf: rocFFT
        r = torch.zeros((16, 16, 16), device="cuda")
        out = torch.empty_like(r)
        with pytest.raises(PfmmError):
            Batch([pl], [r], [out])


def test_fft_near_zone_refuses_misaligned_buffers():
    import torch
    from paper_2011_07099_amd.pfmm import Plan, PfmmError
    N = 32
    rho = torch.zeros((N, N, N), device="cuda")
    buf = torch.empty(N ** 3 + 1, device="cuda")
    phi = buf[1:].view(N, N, N)   # 4 bytes past a 16-byte boundary
    with Plan(N, 3, 4, "S1", near="fft") as pl:
        with pytest.raises(PfmmError):
            pl.solve(rho, phi)
        pl.solve(rho, buf[:N ** 3].view(N, N, N))
        torch.cuda.synchronize()
