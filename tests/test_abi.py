"""The C ABI without a GPU: the library loads, exports every symbol that
include/pfmm.h declares, and rejects invalid arguments before touching the
device (host-side validation only; no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pfmm.h")).read()
    return sorted(set(re.findall(r"\b(pfmm_[a-z_0-9]+)\s*\(", src)))


def _lib():
    from paper_2011_07099_amd import pfmm
    if not os.path.exists(pfmm.LIB_PATH):
        pytest.skip("libpfmm.so not built")
    return pfmm.load()


def test_header_declares_the_binding_exports():
    from paper_2011_07099_amd import pfmm
    assert _declared() == sorted(pfmm.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in _declared():
        assert hasattr(lib, name), name


@pytest.mark.parametrize("N,L,p,g", [
    (12, 2, 4, 2),     # N not a power of two
    (4, 2, 2, 2),      # N too small
    (2048, 8, 4, 2),   # N too large
    (16, 1, 4, 2),     # L < 2
    (16, 5, 4, 2),     # 2^L > N
    (16, 3, 0, 2),     # p < 1
    (16, 3, 11, 2),    # p > 10
    (16, 3, 4, 9),     # unknown Green's function
    (16, 3, 4, 6),     # one past PFMM_GREEN_LEARNED
])
def test_invalid_plan_arguments(N, L, p, g):
    lib = _lib()
    h = ctypes.c_void_p(1)
    st = lib.pfmm_plan_create(N, L, p, g, ctypes.byref(h))
    assert st == 1 and h.value is None
    assert lib.pfmm_last_error().decode()


def test_unsupported_leaf_width():
    lib = _lib()
    h = ctypes.c_void_p()
    assert lib.pfmm_plan_create(1024, 4, 4, 2, ctypes.byref(h)) == 2  # s = 64


def _header_enums():
    src = open(os.path.join(ROOT, "include", "pfmm.h")).read()
    return {k: int(v) for k, v in re.findall(r"\b(PFMM_[A-Z0-9_]+)\s*=\s*(\d+)", src)}


def test_binding_constants_match_the_header():
    from paper_2011_07099_amd import pfmm
    e = _header_enums()
    assert (e["PFMM_OK"], e["PFMM_ERR_INVALID_ARG"], e["PFMM_ERR_UNSUPPORTED"],
            e["PFMM_ERR_OUT_OF_MEMORY"], e["PFMM_ERR_HIP"], e["PFMM_ERR_CAPTURE"],
            e["PFMM_ERR_BAD_HANDLE"]) == (pfmm.OK, pfmm.ERR_INVALID_ARG, pfmm.ERR_UNSUPPORTED,
                                          pfmm.ERR_OUT_OF_MEMORY, pfmm.ERR_HIP, pfmm.ERR_CAPTURE,
                                          pfmm.ERR_BAD_HANDLE) == tuple(range(7))
    for name, v in pfmm.GREEN.items():
        assert e["PFMM_GREEN_" + name] == v
    for name, v in pfmm.PREC.items():
        assert e["PFMM_PREC_" + name.upper()] == v
    for name, v in pfmm.M2L.items():
        assert e["PFMM_M2L_" + name.upper()] == v
    for name, v in pfmm.NEAR.items():
        assert e["PFMM_NEAR_" + name.upper()] == v
    for name in ("PRECISION", "STREAM", "GS_A1", "PROFILE", "FP64_LEVELS", "ISOLATED", "GS_A2",
                 "ACCEL", "EWALD_RS", "M2L", "NEAR", "LEARNED_WEIGHTS"):
        assert e["PFMM_OPT_" + name] == getattr(pfmm, "OPT_" + name)


def test_bad_handles():
    lib = _lib()
    for bogus in (0x1234,                  # an arbitrary address
                  (0x70 << 56) | (7 << 24),  # a plan token whose generation never existed
                  (0x71 << 56) | (1 << 24)):  # a batch token where a plan is expected
        h = ctypes.c_void_p(bogus)
        assert lib.pfmm_solve(h, None, None, None) == 6
        assert lib.pfmm_solve_f64(h, None, None, None) == 6
        assert lib.pfmm_plan_destroy(h) == 6
        assert lib.pfmm_plan_set(h, 1, ctypes.byref(ctypes.c_int32(0)), 4) == 6
        assert lib.pfmm_plan_info(h, None, None) == 6
        n = ctypes.c_int32()
        assert lib.pfmm_gstar_params(h, ctypes.byref(n)) == 6
        assert lib.pfmm_gstar_set(h, None) == 6
        assert lib.pfmm_gstar_loss(h, None, None) == 6
        assert "handle" in lib.pfmm_last_error().decode()
    assert lib.pfmm_plan_destroy(None) == 0
    assert lib.pfmm_plan_create(16, 3, 4, 2, None) == 1


def test_invalid_batch_arguments():
    lib = _lib()
    h = ctypes.c_void_p(1)
    assert lib.pfmm_batch_create(0, None, None, None, ctypes.byref(h)) == 1 and h.value is None
    arr = (ctypes.c_void_p * 1)(0x1234)
    assert lib.pfmm_batch_create(1, arr, arr, arr, ctypes.byref(h)) == 6
    assert lib.pfmm_batch_create(1, arr, arr, arr, None) == 1
    assert lib.pfmm_batch_solve(ctypes.c_void_p(0x1234)) == 6
    assert lib.pfmm_batch_solve(ctypes.c_void_p((0x70 << 56) | (1 << 24))) == 6  # a plan token
    assert lib.pfmm_batch_destroy(None) == 0
    assert lib.pfmm_solve_batch(0, None, None, None) == 1
    assert lib.pfmm_solve_batch(1, arr, arr, arr) == 6


def test_header_is_plain_c_and_links():
    """include/pfmm.h compiles as C99 on its own, and a C program that takes
    the address of every declared function links against libpfmm.so."""
    import shutil
    import subprocess
    from paper_2011_07099_amd import pfmm
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    work = os.path.join(ROOT, "_build", "abi_c")  # build scratch, ignored by git
    os.makedirs(work, exist_ok=True)
    src = os.path.join(work, "use.c")
    names = _declared()
    open(src, "w").write('#include "pfmm.h"\n#include <stdio.h>\nint main(void) {\n'
                   "  const void* f[] = {%s};\n"
                   '  printf("%%d\\n", (int)(sizeof f / sizeof f[0]));\n  return 0;\n}\n'
                   % ", ".join("(const void*)&" + n for n in names))
    inc = os.path.join(ROOT, "include")
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-I", inc, str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    if not os.path.exists(pfmm.LIB_PATH):
        pytest.skip("libpfmm.so not built")
    exe = os.path.join(work, "use")
    libdir = os.path.dirname(pfmm.LIB_PATH)
    r = subprocess.run([cc, "-std=c99", "-I", inc, str(src), "-o", str(exe), "-L", libdir,
                        "-lpfmm", "-Wl,-rpath," + libdir], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
