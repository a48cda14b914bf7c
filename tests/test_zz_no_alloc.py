"""pfmm_plan_direct_noalloc, the entry point for callers that cannot allocate:
the direct periodic convolution (Eq. 4) with the lattice table in the
library's static device array.  Each call must equal pfmm_plan_direct (same
table values, same kernel, same summation order: bit for bit), also when the
previous call on the device left a larger table of another G in the array:
two calls in a row, the second on a smaller mesh.  Beyond N = 64 it is
refused; isolated plans are refused as by pfmm_plan_direct."""
import ctypes

import numpy as np
import pytest

from paper_2011_07099_amd import fields

pytestmark = pytest.mark.gpu


def _noalloc(lib, pl, rho, phi):
    return lib.pfmm_plan_direct_noalloc(pl._h, ctypes.c_void_p(rho.data_ptr()),
                                        ctypes.c_void_p(phi.data_ptr()))


def test_noalloc_direct_equals_direct_on_two_calls_in_a_row():
    import torch
    from paper_2011_07099_amd import pfmm
    lib = pfmm.load()
    cases = [(64, 3, 4, "K", 61), (32, 3, 4, "S1", 62)]   # the second smaller, another G
    for rep in range(2):
        for N, L, p, g, seed in cases:
            rho = torch.from_numpy(fields.lognormal(N, 2.0, 1.0, seed=seed).astype(np.float32)).cuda()
            ref = torch.empty_like(rho)
            out = torch.full_like(rho, float("nan"))
            with pfmm.Plan(N, L, p, g) as pl:
                assert _noalloc(lib, pl, rho, out) == pfmm.OK, pfmm.last_error()
                pl.direct(rho, ref)
                torch.cuda.synchronize()
            same = torch.equal(out, ref)
            print("pass %d, N=%d G_%s: no-alloc direct bit-identical to pfmm_plan_direct: %s"
                  % (rep, N, g, same), flush=True)
            assert same


def test_noalloc_direct_refusals():
    import torch
    from paper_2011_07099_amd import pfmm
    lib = pfmm.load()
    rho = torch.zeros((128, 128, 128), dtype=torch.float32, device="cuda")
    phi = torch.empty_like(rho)
    with pfmm.Plan(128, 3, 4, "S1") as pl:
        assert _noalloc(lib, pl, rho, phi) == pfmm.ERR_UNSUPPORTED
    small = torch.zeros((32, 32, 32), dtype=torch.float32, device="cuda")
    with pfmm.Plan(32, 3, 4, "X", isolated=True) as pl:
        assert _noalloc(lib, pl, small, torch.empty_like(small)) == pfmm.ERR_UNSUPPORTED
    with pfmm.Plan(32, 3, 4, "S1") as pl:
        assert _noalloc(lib, pl, small, small) == pfmm.ERR_INVALID_ARG
