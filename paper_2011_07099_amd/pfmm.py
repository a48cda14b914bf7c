"""Thin ctypes binding of libpfmm (C ABI in include/pfmm.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  torch supplies device memory (``data_ptr()``) and streams.  The
library is loaded from this package directory; if it is missing, every call
raises — there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpfmm.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_OUT_OF_MEMORY, ERR_HIP, ERR_CAPTURE, ERR_BAD_HANDLE = \
    range(7)
GREEN = {"X": 0, "K": 1, "S1": 2, "S": 3, "E": 4, "LEARNED": 5}
PREC = {"fp32": 0, "bf16x3": 1, "fp64": 2}
OPT_PRECISION, OPT_STREAM, OPT_GS_A1, OPT_PROFILE, OPT_FP64_LEVELS, OPT_ISOLATED, OPT_GS_A2, \
    OPT_ACCEL, OPT_EWALD_RS, OPT_M2L, OPT_NEAR, OPT_LEARNED_WEIGHTS, OPT_FOLD, \
    OPT_ZONES_FP32 = range(1, 15)
M2L = {"gemm": 0, "fft": 1, "spectral": 2}
NEAR = {"direct": 0, "fft": 1}
ACCEL = {"fd4": 0, "expansion": 1}
STAGES = ("p2m", "m2m", "m2l", "l2l", "l2p", "near", "fd4")
BUF_MULTIPOLE, BUF_LOCAL, BUF_TABLE_LEVEL, BUF_TABLE_NEAR = 0, 1, 2, 3

# every symbol include/pfmm.h declares
EXPORTS = ("pfmm_plan_create", "pfmm_plan_set", "pfmm_solve", "pfmm_solve_f64", "pfmm_plan_read",
           "pfmm_plan_stage_times", "pfmm_plan_level_times", "pfmm_plan_kernel_times",
           "pfmm_plan_info", "pfmm_plan_destroy",
           "pfmm_batch_create", "pfmm_batch_solve", "pfmm_batch_info", "pfmm_batch_group",
           "pfmm_batch_destroy", "pfmm_solve_batch",
           "pfmm_plan_direct", "pfmm_plan_direct_noalloc", "pfmm_learned_set",
           "pfmm_learned_train_begin",
           "pfmm_learned_accumulate", "pfmm_learned_loss", "pfmm_learned_step", "pfmm_learned_get",
           "pfmm_learned_read_grad", "pfmm_table_params", "pfmm_table_set", "pfmm_table_get",
           "pfmm_table_train_begin", "pfmm_table_grad", "pfmm_gstar_params", "pfmm_gstar_set",
           "pfmm_gstar_get", "pfmm_gstar_loss", "pfmm_gstar_accumulate", "pfmm_gstar_grad",
           "pfmm_last_error")
MLP_PARAMS = 4801

_lib = None


class PfmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("pfmm status %d: %s" % (status, msg))
        self.status = status


def load():
    """Open libpfmm.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpfmm.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    lib.pfmm_plan_create.argtypes = [i32, i32, i32, i32, ctypes.POINTER(vp)]
    lib.pfmm_plan_set.argtypes = [vp, i32, vp, sz]
    lib.pfmm_solve.argtypes = [vp, vp, vp, vp]
    lib.pfmm_solve_f64.argtypes = [vp, vp, vp, vp]
    lib.pfmm_plan_read.argtypes = [vp, i32, i32, vp]
    lib.pfmm_plan_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(i32)]
    lib.pfmm_plan_level_times.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
    lib.pfmm_plan_kernel_times.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(i32)]
    lib.pfmm_plan_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_int64)]
    lib.pfmm_plan_destroy.argtypes = [vp]
    lib.pfmm_batch_create.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), ctypes.POINTER(vp)]
    lib.pfmm_batch_solve.argtypes = [vp]
    lib.pfmm_batch_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.pfmm_batch_group.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    lib.pfmm_batch_destroy.argtypes = [vp]
    lib.pfmm_solve_batch.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                     ctypes.POINTER(vp)]
    fp = ctypes.POINTER(ctypes.c_float)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.pfmm_plan_direct.argtypes = [vp, vp, vp]
    lib.pfmm_plan_direct_noalloc.argtypes = [vp, vp, vp]
    lib.pfmm_learned_set.argtypes = [vp, fp, i32]
    lib.pfmm_learned_train_begin.argtypes = [vp, fp, ctypes.c_double]
    lib.pfmm_learned_accumulate.argtypes = [vp, vp, vp, dp]
    lib.pfmm_learned_loss.argtypes = [vp, vp, vp, dp]
    lib.pfmm_table_params.argtypes = [vp, ctypes.POINTER(i32)]
    lib.pfmm_table_set.argtypes = [vp, fp]
    lib.pfmm_table_get.argtypes = [vp, fp]
    lib.pfmm_table_train_begin.argtypes = [vp, ctypes.c_double]
    lib.pfmm_table_grad.argtypes = [vp, fp]
    lib.pfmm_gstar_params.argtypes = [vp, ctypes.POINTER(i32)]
    lib.pfmm_gstar_set.argtypes = [vp, fp]
    lib.pfmm_gstar_get.argtypes = [vp, fp]
    lib.pfmm_gstar_loss.argtypes = [vp, vp, dp]
    lib.pfmm_gstar_accumulate.argtypes = [vp, vp, dp]
    lib.pfmm_gstar_grad.argtypes = [vp, fp]
    lib.pfmm_learned_step.argtypes = [vp]
    lib.pfmm_learned_get.argtypes = [vp, fp]
    lib.pfmm_learned_read_grad.argtypes = [vp, i32, dp, fp]
    lib.pfmm_last_error.restype = ctypes.c_char_p
    for f in EXPORTS[:-1]:
        getattr(lib, f).restype = i32
    _lib = lib
    return lib


def _check(st):
    if st != OK:
        raise PfmmError(st, load().pfmm_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A periodic-FMM plan: ``Plan(N, L, p, green)`` then ``solve(rho, phi[, accel])``.

    ``green`` is one of "X", "K", "S1", "S" (see include/pfmm.h).  ``stream``
    is a torch.cuda.Stream (default: torch's current stream at creation).
    """

    def __init__(self, N, L, p, green="S1", precision="fp32", a1=None, stream=None,
                 fp64_levels=None, isolated=False, a2=None, accel="fd4", rs=None, m2l="gemm",
                 near="direct", fold=False, zones_fp32=False):
        import torch
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.pfmm_plan_create(int(N), int(L), int(p), GREEN[green], ctypes.byref(h)))
        self._h = h
        self.N, self.L, self.p, self.green = int(N), int(L), int(p), green
        s = ctypes.c_int()
        _check(lib.pfmm_plan_info(self._h, ctypes.byref(s), None))
        self.s = s.value
        if stream is None:
            stream = torch.cuda.current_stream()
        self.set_stream(stream)
        if precision != "fp32":
            self.set_precision(precision)
        if a1 is not None:
            self.set_a1(a1)
        if a2 is not None:
            self.set_a2(a2)
        if rs is not None:
            self.set_ewald_rs(rs)
        if fp64_levels is not None:
            self.set_fp64_levels(fp64_levels)
        if isolated:
            self.set_isolated(True)
        if accel != "fd4":
            self.set_accel(accel)
        if m2l != "gemm":
            self.set_m2l(m2l)
        if near != "direct":
            self.set_near(near)
        if fold:
            self.set_fold(True)
        if zones_fp32:
            self.set_zones_fp32(True)

    def set_zones_fp32(self, on):
        """Spectral zones of a 16^3 leaf level (L = 4) summed in FP32 columns
        with FP64 totals; see PFMM_OPT_ZONES_FP32."""
        v = ctypes.c_int32(1 if on else 0)
        _check(load().pfmm_plan_set(self._h, OPT_ZONES_FP32, ctypes.byref(v), 4))

    def set_fold(self, on):
        """P2M and L2P inside the FFT near zone's leaf transforms (leaf edge 8
        or 16, p = 4 or 8, FP32 leaf level); see PFMM_OPT_FOLD."""
        v = ctypes.c_int32(1 if on else 0)
        _check(load().pfmm_plan_set(self._h, OPT_FOLD, ctypes.byref(v), 4))

    def set_near(self, mode):
        """Leaf near zone by "direct" summation (block Toeplitz) or "fft"
        (convolution on the doubled grid, one transform per leaf)."""
        v = ctypes.c_int32(NEAR[mode])
        _check(load().pfmm_plan_set(self._h, OPT_NEAR, ctypes.byref(v), 4))

    def set_m2l(self, mode):
        """Interaction zones by "gemm" (block Toeplitz), "fft" (the HPM FFT
        convolution, a comparator) or "spectral" (per-node transforms and a
        per-frequency stencil, FP64; p = 4, 6 or 8)."""
        v = ctypes.c_int32(M2L[mode])
        _check(load().pfmm_plan_set(self._h, OPT_M2L, ctypes.byref(v), 4))

    def set_accel(self, mode):
        """How solve forms accelerations: "fd4" (differences of the potential)
        or "expansion" (gradient of the local expansion plus the near zone's
        differenced kernels)."""
        v = ctypes.c_int32(ACCEL[mode])
        _check(load().pfmm_plan_set(self._h, OPT_ACCEL, ctypes.byref(v), 4))

    def set_isolated(self, on):
        """The non-periodic twin (G_X without images, sources outside the box
        absent); PFMM_GREEN_X plans only."""
        v = ctypes.c_int32(1 if on else 0)
        _check(load().pfmm_plan_set(self._h, OPT_ISOLATED, ctypes.byref(v), 4))

    def set_fp64_levels(self, n):
        v = ctypes.c_int32(int(n))
        _check(load().pfmm_plan_set(self._h, OPT_FP64_LEVELS, ctypes.byref(v), 4))

    def set_stream(self, stream):
        self.stream = stream
        v = ctypes.c_void_p(stream.cuda_stream)
        _check(load().pfmm_plan_set(self._h, OPT_STREAM, ctypes.byref(v), ctypes.sizeof(v)))

    def set_precision(self, precision):
        v = ctypes.c_int32(PREC[precision])
        _check(load().pfmm_plan_set(self._h, OPT_PRECISION, ctypes.byref(v), 4))
        self.precision = precision

    def set_a1(self, a1):
        v = ctypes.c_double(float(a1))
        _check(load().pfmm_plan_set(self._h, OPT_GS_A1, ctypes.byref(v), 8))

    def set_ewald_rs(self, rs):
        """Splitting radius r_S of the Ewald G_E (green "E")."""
        v = ctypes.c_double(float(rs))
        _check(load().pfmm_plan_set(self._h, OPT_EWALD_RS, ctypes.byref(v), 8))

    def set_a2(self, a2):
        v = ctypes.c_double(float(a2))
        _check(load().pfmm_plan_set(self._h, OPT_GS_A2, ctypes.byref(v), 8))

    def set_profile(self, on):
        """Stage timing: False (off), True or "serial" (stages one after another
        on the plan's stream), "live" (near zone beside the tree, as unprofiled)."""
        mode = {False: 0, True: 1, "serial": 1, "live": 2}[on]
        v = ctypes.c_int32(mode)
        _check(load().pfmm_plan_set(self._h, OPT_PROFILE, ctypes.byref(v), 4))

    def stage_times(self):
        """{stage: (ms, launches)} of the last profiled solve (synchronises)."""
        ms = (ctypes.c_double * len(STAGES))()
        n = (ctypes.c_int * len(STAGES))()
        _check(load().pfmm_plan_stage_times(self._h, ms, n))
        return {s: (ms[i], n[i]) for i, s in enumerate(STAGES)}

    def level_times(self, stage="m2l"):
        """{level: ms} of a per-level stage ("m2m", "m2l" or "l2l"), averaged
        over the recent profiled solves (synchronises)."""
        ms = (ctypes.c_double * (self.L + 1))()
        _check(load().pfmm_plan_level_times(self._h, STAGES.index(stage), ms))
        return {l: ms[l] for l in range(self.L + 1) if ms[l] > 0.0}

    def kernel_times(self, stage, level=0):
        """[ms per kernel] of a stage at a tree level (see pfmm_plan_kernel_times),
        averaged over the recent profiled solves (synchronises)."""
        ms = (ctypes.c_double * 8)()
        n = ctypes.c_int()
        _check(load().pfmm_plan_kernel_times(self._h, STAGES.index(stage), int(level), ms,
                                             ctypes.byref(n)))
        return [ms[i] for i in range(n.value)]

    def solve(self, rho, phi, accel=None):
        """FP32 density -> FP32 potential (and accelerations); float64 tensors
        go to the FP64 entry point (plans in precision "fp64" only)."""
        import torch
        n3 = self.N ** 3
        dt = rho.dtype
        if dt not in (torch.float32, torch.float64):
            raise ValueError("expected float32 or float64 tensors")
        for t, n in ((rho, n3), (phi, n3)) + (((accel, 3 * n3),) if accel is not None else ()):
            if t.dtype != dt or t.numel() != n:
                raise ValueError("expected tensors of one dtype with N^3 (accel 3 N^3) elements")
        f = load().pfmm_solve_f64 if dt == torch.float64 else load().pfmm_solve
        _check(f(self._h, _ptr(rho), _ptr(phi), _ptr(accel)))

    def set_learned_weights(self, weights):
        """The network's weights through PFMM_OPT_LEARNED_WEIGHTS (BF16 inference)."""
        w, _ = self._f32(weights)
        _check(load().pfmm_plan_set(self._h, OPT_LEARNED_WEIGHTS, w.ctypes.data_as(ctypes.c_void_p),
                                    w.nbytes))

    def direct(self, rho, phi):
        """Exact periodic convolution with the plan's G on the device (O(N^6))."""
        _check(load().pfmm_plan_direct(self._h, _ptr(rho), _ptr(phi)))

    def direct_noalloc(self, rho, phi):
        """The same without allocating (the library's static device array;
        N <= 64)."""
        _check(load().pfmm_plan_direct_noalloc(self._h, _ptr(rho), _ptr(phi)))

    # --- learned correction of the interaction-zone tables ---------------
    @staticmethod
    def _f32(w):
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.size != MLP_PARAMS:
            raise ValueError("weights must have %d entries" % MLP_PARAMS)
        return w, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))

    def set_learned(self, weights, bf16=True):
        """Correct the tables with the network (None: back to the plain G)."""
        if weights is None:
            _check(load().pfmm_learned_set(self._h, None, 0))
            return
        w, ptr = self._f32(weights)
        _check(load().pfmm_learned_set(self._h, ptr, 1 if bf16 else 0))

    def table_params(self):
        """Number of free values of the grid-valued tables (one per cube-
        symmetry orbit of table entries and level)."""
        n = ctypes.c_int()
        _check(load().pfmm_table_params(self._h, ctypes.byref(n)))
        return n.value

    def set_table(self, delta):
        """Grid-valued tables T = G (1 + delta[orbit]) (None: back to the plain G)."""
        import numpy as np
        if delta is None:
            _check(load().pfmm_table_set(self._h, None))
            return
        d = np.ascontiguousarray(delta, dtype=np.float32)
        if d.size != self.table_params():
            raise ValueError("delta must have table_params() entries")
        _check(load().pfmm_table_set(self._h, d.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def table_values(self):
        import numpy as np
        d = np.empty(self.table_params(), np.float32)
        _check(load().pfmm_table_get(self._h, d.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return d

    def table_train_begin(self, lr):
        """Train the grid-valued tables (from exactly G) with train_accumulate /
        train_step."""
        _check(load().pfmm_table_train_begin(self._h, float(lr)))

    def table_grad(self):
        """Gradient of the summed loss over the fields accumulated since the
        last step, d loss / d delta (clears it)."""
        import numpy as np
        g = np.empty(self.table_params(), np.float32)
        _check(load().pfmm_table_grad(self._h, g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return g

    # --- G_* as one grid-valued function everywhere (Eq. 8) ----------------
    def gstar_params(self):
        """Number of free values of G_* (one per cube-symmetry orbit of mesh
        separations)."""
        n = ctypes.c_int()
        _check(load().pfmm_gstar_params(self._h, ctypes.byref(n)))
        return n.value

    def set_gstar(self, delta):
        """G_* = G (1 + delta[orbit]) in the near zone, every level's tables
        and the direct solve; None restores G everywhere."""
        import numpy as np
        if delta is None:
            _check(load().pfmm_gstar_set(self._h, None))
            return
        d = np.ascontiguousarray(delta, np.float32)
        if d.size != self.gstar_params():
            raise ValueError("delta must have %d entries" % self.gstar_params())
        _check(load().pfmm_gstar_set(self._h, d.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def gstar_values(self):
        import numpy as np
        d = np.empty(self.gstar_params(), np.float32)
        _check(load().pfmm_gstar_get(self._h, d.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return d

    def gstar_loss(self, rho):
        """Relative mean-removed squared residual of the FMM against PM, both
        with the plan's G_*."""
        v = ctypes.c_double()
        _check(load().pfmm_gstar_loss(self._h, _ptr(rho), ctypes.byref(v)))
        return v.value

    def gstar_accumulate(self, rho):
        v = ctypes.c_double()
        _check(load().pfmm_gstar_accumulate(self._h, _ptr(rho), ctypes.byref(v)))
        return v.value

    def gstar_grad(self):
        """Gradient summed over the accumulated densities (clears it)."""
        import numpy as np
        g = np.empty(self.gstar_params(), np.float32)
        _check(load().pfmm_gstar_grad(self._h, g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return g

    def train_begin(self, weights, lr):
        w, ptr = self._f32(weights)
        _check(load().pfmm_learned_train_begin(self._h, ptr, float(lr)))

    def train_accumulate(self, rho, target):
        loss = ctypes.c_double()
        _check(load().pfmm_learned_accumulate(self._h, _ptr(rho), _ptr(target), ctypes.byref(loss)))
        return loss.value

    def loss(self, rho, target):
        """Relative mean-removed squared residual against target, no gradient."""
        v = ctypes.c_double()
        _check(load().pfmm_learned_loss(self._h, _ptr(rho), _ptr(target), ctypes.byref(v)))
        return v.value

    def train_step(self):
        _check(load().pfmm_learned_step(self._h))

    def learned_weights(self):
        import numpy as np
        w = np.empty(MLP_PARAMS, np.float32)
        _check(load().pfmm_learned_get(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return w

    def learned_grads(self, level):
        import numpy as np
        g = np.empty((8 * self.p - 1) ** 3, np.float64)
        w = np.empty(MLP_PARAMS, np.float32)
        _check(load().pfmm_learned_read_grad(self._h, int(level),
                                             g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return g.reshape((8 * self.p - 1,) * 3), w

    def read(self, buffer, level, out):
        _check(load().pfmm_plan_read(self._h, int(buffer), int(level), _ptr(out)))
        return out

    def multipoles(self, level):
        import torch
        out = torch.empty(8 ** level * self.p ** 3, dtype=torch.float32, device="cuda")
        return self.read(BUF_MULTIPOLE, level, out)

    def locals(self, level):
        import torch
        out = torch.empty(8 ** level * self.p ** 3, dtype=torch.float32, device="cuda")
        return self.read(BUF_LOCAL, level, out)

    def level_table(self, level):
        import torch
        out = torch.empty((8 * self.p - 1) ** 3, dtype=torch.float64, device="cuda")
        return self.read(BUF_TABLE_LEVEL, level, out)

    def near_table(self):
        import torch
        out = torch.empty((4 * self.s - 1) ** 3, dtype=torch.float64, device="cuda")
        return self.read(BUF_TABLE_NEAR, 2, out)

    def close(self):
        if getattr(self, "_h", None):
            _check(load().pfmm_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def last_error():
    """The calling thread's last message from the library ("" if none)."""
    return load().pfmm_last_error().decode()


def solve_batch(plans, rhos, phis):
    """pfmm_solve_batch: solve independent fields as one batch.  The first
    call with a given set of (plan, density, potential) builds and keeps its
    graph; later calls with the same set only launch it."""
    n = len(plans)
    if not (n == len(rhos) == len(phis)) or n == 0:
        raise ValueError("plans, rhos and phis must have the same non-zero length")
    for pl, r, f in zip(plans, rhos, phis):
        _ptr(r), _ptr(f)
        if r.numel() != pl.N ** 3 or f.numel() != pl.N ** 3:
            raise ValueError("tensor sizes must match the plans")
    P = (ctypes.c_void_p * n)(*[pl._h.value for pl in plans])
    R = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhos])
    F = (ctypes.c_void_p * n)(*[f.data_ptr() for f in phis])
    _check(load().pfmm_solve_batch(n, P, R, F))


class Batch:
    """Many independent fields solved by one graph launch (``pfmm_batch_*``).

    ``plans``: Plan objects (p <= 8); ``rhos``/``phis``: matching device
    tensors.  Creation tunes the persistent kernel's tile width (cached in the
    JSON file named by PFMM_TUNE_CACHE, if set) and captures the graph.
    """

    def __init__(self, plans, rhos, phis):
        lib = load()
        n = len(plans)
        if not (n == len(rhos) == len(phis)) or n == 0:
            raise ValueError("plans, rhos and phis must have the same non-zero length")
        for pl, r, f in zip(plans, rhos, phis):
            _ptr(r), _ptr(f)
            if r.numel() != pl.N ** 3 or f.numel() != pl.N ** 3:
                raise ValueError("tensor sizes must match the plans")
        self._keep = (list(plans), list(rhos), list(phis))
        P = (ctypes.c_void_p * n)(*[pl._h.value for pl in plans])
        R = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhos])
        F = (ctypes.c_void_p * n)(*[f.data_ptr() for f in phis])
        h = ctypes.c_void_p()
        _check(lib.pfmm_batch_create(n, P, R, F, ctypes.byref(h)))
        self._h = h

    def solve(self):
        _check(load().pfmm_batch_solve(self._h))

    def info(self):
        """{"items": total work items, "groups": [{"q", "fp64", "near",
        "width", "ms": timed ms at widths 1, 2, 4 (negative: not timed)}]}"""
        lib = load()
        items, ng = ctypes.c_int(), ctypes.c_int()
        _check(lib.pfmm_batch_info(self._h, ctypes.byref(items), ctypes.byref(ng)))
        groups = []
        for g in range(ng.value):
            desc = (ctypes.c_int * 4)()
            ms = (ctypes.c_double * 3)()
            _check(lib.pfmm_batch_group(self._h, g, desc, ms))
            groups.append({"q": desc[0], "fp64": bool(desc[1]), "near": bool(desc[2]),
                           "width": desc[3], "ms": list(ms)})
        return {"items": items.value, "groups": groups}

    def close(self):
        if getattr(self, "_h", None):
            _check(load().pfmm_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
