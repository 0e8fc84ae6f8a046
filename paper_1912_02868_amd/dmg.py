"""ctypes binding of libdmg (include/dmg.h).

Argument marshalling only: every operation runs in the HIP library.  Device
buffers are torch tensors on the GPU (complex128 for FP64 data, complex64 for
FP32 data), host buffers are numpy arrays; both are passed as plain pointers.
By default the library's device memory comes from torch's caching allocator and
its kernels run on torch's current stream.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmg.so")

DMG_OK = 0
DMG_W_NOT_CONVERGED = 1
DMG_E_INVALID = -1
DMG_E_NONFINITE = -2
DMG_E_HIP = -3
DMG_E_BUDGET = -4
DMG_E_NOMEM = -5
DMG_E_BREAKDOWN = -6
PTR_HOST, PTR_DEVICE = 0, 1
FP64, FP32, FP32_BF16, FP32_BF16C = 0, 1, 2, 3
PART_NULLVECS, PART_P, PART_BLOCKS, PART_SETUP_ITERS = 0, 1, 2, 3
OP_APPLY, OP_APPLY_DAG, OP_RESTRICT, OP_PROLONG = 0, 1, 2, 3

EXPORTED = [
    "dmg_context_create", "dmg_context_destroy", "dmg_last_error", "dmg_context_bytes_in_use",
    "dmg_context_set_budget",
    "dmg_gauge_create", "dmg_gauge_destroy", "dmg_apply_dirac",
    "dmg_setup", "dmg_hierarchy_destroy", "dmg_hierarchy_export", "dmg_hierarchy_part_bytes",
    "dmg_hierarchy_apply", "dmg_hierarchy_apply_batched", "dmg_hierarchy_apply_batched_static",
    "dmg_deflation_create", "dmg_deflation_build", "dmg_deflation_reset", "dmg_deflation_ready",
    "dmg_deflation_export", "dmg_deflation_destroy",
    "dmg_solve_params_default", "dmg_setup_params_default", "dmg_solve", "dmg_solve_batched", "dmg_solve_fine",
    "dmg_kernel_timer", "dmg_kernel_timer_read",
    "dmg_pool_create", "dmg_pool_admit", "dmg_pool_step", "dmg_pool_retire", "dmg_pool_slot_state",
    "dmg_pool_destroy",
    "dmg_batch_create", "dmg_batch_admit", "dmg_batch_step", "dmg_batch_retire", "dmg_batch_slot_state",
    "dmg_batch_destroy",
    "dmg_autotune", "dmg_autotune_force", "dmg_autotune_report",
]
SLOT_FREE, SLOT_RUNNING, SLOT_DONE = 0, 1, 2
POOL_MAX_SLOTS = 8
BATCH_MAX_LANES = 64
KT_COARSE_PROJ, KT_BLOCK_APPLY_INT, KT_BLOCK_BATCHED, KT_WILSON_BATCHED = 0, 1, 2, 3
TUNE_BLOCK, TUNE_WILSON = 0, 1


class DmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dmg error {code}: {msg}")
        self.code = code


class Allocator(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)),
                ("user", C.c_void_p)]


class SetupParams(C.Structure):
    _fields_ = [("nvec", C.c_int), ("null_tol", C.c_double), ("null_max_iters", C.c_int)]


class SolveParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("outer_m", C.c_int), ("max_outer_iters", C.c_int),
                ("smooth_steps", C.c_int), ("int_tol", C.c_double), ("int_m", C.c_int),
                ("int_max_iters", C.c_int), ("coarse_tol_first", C.c_double),
                ("coarse_tol_later", C.c_double), ("coarse_max_iters", C.c_int),
                ("precond", C.c_int), ("use_x0", C.c_int), ("coarse_persistent", C.c_int), ("int_mode", C.c_int),
                ("graphs", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("converged", C.c_int), ("fine_mvps", C.c_longlong),
                ("int_mvps", C.c_longlong), ("coarse_mvps", C.c_longlong), ("fine_equiv_mvps", C.c_double),
                ("true_rel_resid", C.c_double), ("coarse_calls", C.c_int), ("coarse_dr_calls", C.c_int),
                ("elapsed_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_live = []  # handles closed (newest first) at interpreter exit, before torch tears down


def _register(obj):
    import weakref
    _live.append(weakref.ref(obj))


def _close_all():
    for ref in reversed(_live):
        obj = ref()
        if obj is not None:
            try:
                obj.close()
            except Exception:
                pass
    _live.clear()


import atexit  # noqa: E402
atexit.register(_close_all)


def lib():
    """The loaded library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1912_02868_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i, d, sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
    pp = C.POINTER(C.c_void_p)
    sig = {
        "dmg_context_create": (i, [i, vp, C.POINTER(Allocator), sz, pp]),
        "dmg_context_destroy": (None, [vp]),
        "dmg_last_error": (C.c_char_p, [vp]),
        "dmg_context_bytes_in_use": (sz, [vp]),
        "dmg_context_set_budget": (i, [vp, sz]),
        "dmg_gauge_create": (i, [vp, i, i, vp, i, pp]),
        "dmg_gauge_destroy": (None, [vp]),
        "dmg_apply_dirac": (i, [vp, vp, d, i, i, vp, vp, i, i]),
        "dmg_setup": (i, [vp, vp, d, C.POINTER(SetupParams), vp, vp, i, i, pp]),
        "dmg_hierarchy_destroy": (None, [vp]),
        "dmg_hierarchy_export": (i, [vp, i, i, vp, sz]),
        "dmg_hierarchy_part_bytes": (sz, [vp, i, i]),
        "dmg_hierarchy_apply": (i, [vp, i, i, i, vp, vp, i]),
        "dmg_hierarchy_apply_batched": (i, [vp, i, i, i, vp, vp, i, i, i]),
        "dmg_hierarchy_apply_batched_static": (i, [vp, i, i, i, vp, vp, i, i]),
        "dmg_deflation_create": (i, [vp, i, i, pp]),
        "dmg_deflation_build": (i, [vp, vp, d, i]),
        "dmg_deflation_reset": (None, [vp]),
        "dmg_deflation_ready": (i, [vp]),
        "dmg_deflation_export": (i, [vp, vp, vp, C.POINTER(C.c_int)]),
        "dmg_deflation_destroy": (None, [vp]),
        "dmg_solve_params_default": (None, [C.POINTER(SolveParams)]),
        "dmg_setup_params_default": (None, [C.POINTER(SetupParams)]),
        "dmg_solve": (i, [vp, vp, vp, C.POINTER(SolveParams), vp, vp, i, i, C.POINTER(SolveStats)]),
        "dmg_solve_batched": (i, [vp, vp, vp, C.POINTER(SolveParams), vp, vp, i, i, C.POINTER(SolveStats)]),
        "dmg_solve_fine": (i, [vp, vp, i, i, i, d, i, vp, vp, i, i, C.POINTER(SolveStats)]),
        "dmg_kernel_timer": (i, [vp, i]),
        "dmg_pool_create": (i, [vp, i, C.POINTER(SolveParams), pp]),
        "dmg_pool_admit": (i, [vp, i, vp, vp, vp, i]),
        "dmg_pool_step": (i, [vp, i, C.POINTER(C.c_int)]),
        "dmg_pool_retire": (i, [vp, i, vp, i, C.POINTER(SolveStats)]),
        "dmg_pool_slot_state": (i, [vp, i]),
        "dmg_pool_destroy": (None, [vp]),
        "dmg_batch_create": (i, [vp, vp, i, C.POINTER(SolveParams), pp]),
        "dmg_batch_admit": (i, [vp, i, vp, i]),
        "dmg_batch_step": (i, [vp, i, C.POINTER(C.c_int)]),
        "dmg_batch_retire": (i, [vp, i, vp, i, C.POINTER(SolveStats)]),
        "dmg_batch_slot_state": (i, [vp, i]),
        "dmg_batch_destroy": (None, [vp]),
        "dmg_kernel_timer_read": (i, [vp, i, C.POINTER(C.c_double), C.POINTER(C.c_longlong),
                                      C.POINTER(C.c_longlong)]),
        "dmg_autotune": (i, [i]),
        "dmg_autotune_force": (i, [i, i]),
        "dmg_autotune_report": (sz, [C.c_char_p, sz]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def solve_params(**kw) -> SolveParams:
    p = SolveParams()
    lib().dmg_solve_params_default(C.byref(p))
    for k, v in kw.items():
        if k == "precond" and isinstance(v, str):
            v = {"fp64": FP64, "fp32": FP32, "fp32_bf16": FP32_BF16, "fp32_bf16c": FP32_BF16C}[v]
        setattr(p, k, v)
    return p


def setup_params(**kw) -> SetupParams:
    p = SetupParams()
    lib().dmg_setup_params_default(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _ptr(a):
    """(pointer, ptr_kind) of a torch GPU tensor or a host numpy array."""
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("host arrays must be C-contiguous")
        return a.ctypes.data_as(C.c_void_p), PTR_HOST
    import torch
    if isinstance(a, torch.Tensor):
        if not a.is_cuda:
            raise ValueError("torch tensors must live on the GPU (use numpy for host data)")
        if not a.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return C.c_void_p(a.data_ptr()), PTR_DEVICE
    raise TypeError(f"unsupported buffer type {type(a)}")


class Context:
    """A device, a stream and an HBM budget; device memory from torch's caching allocator."""

    def __init__(self, device: int = 0, budget: int = 0, torch_alloc: bool = True, stream=None):
        import torch
        self.device = device
        self._torch = torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self._alloc = None
        if torch_alloc:
            dev = device

            alloc_fn = torch.cuda.caching_allocator_alloc
            free_fn = torch.cuda.caching_allocator_delete

            def _a(nbytes, user):
                return alloc_fn(int(nbytes), dev, stream)

            def _f(ptr, user):
                try:
                    free_fn(ptr)
                except Exception:
                    pass  # interpreter shutdown: torch already released its pools

            self._alloc = Allocator(Allocator._fields_[0][1](_a), Allocator._fields_[1][1](_f), None)
        self.h = C.c_void_p()
        st = lib().dmg_context_create(device, C.c_void_p(stream.cuda_stream),
                                      C.byref(self._alloc) if self._alloc else None, budget, C.byref(self.h))
        if st != DMG_OK:
            raise DmgError(st, "context creation failed")
        _register(self)

    def check(self, st, what=""):
        if st < 0:
            raise DmgError(st, f"{what}: {lib().dmg_last_error(self.h).decode()}")
        return st

    def timer(self, *kernels: int):
        """Time the given kernels (KT_*) from now on, resetting the sums; no argument stops timing."""
        mask = 0
        for k in kernels:
            mask |= 1 << k
        self.check(lib().dmg_kernel_timer(self.h, mask), "kernel_timer")

    def timer_read(self, kernel: int):
        """(total ms, launches, work units) of a timed kernel since the timer was enabled."""
        ms, n, u = C.c_double(), C.c_longlong(), C.c_longlong()
        self.check(lib().dmg_kernel_timer_read(self.h, kernel, C.byref(ms), C.byref(n), C.byref(u)), "timer_read")
        return ms.value, n.value, u.value

    @property
    def bytes_in_use(self) -> int:
        return lib().dmg_context_bytes_in_use(self.h)

    def set_budget(self, nbytes: int):
        """HBM budget of later allocations (0: none)."""
        self.check(lib().dmg_context_set_budget(self.h, int(nbytes)), "set_budget")

    def close(self):
        if self.h:
            lib().dmg_context_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Gauge:
    def __init__(self, ctx: Context, theta: np.ndarray, antiperiodic: bool = True):
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        Nt, Nx, two = theta.shape
        assert two == 2
        self.ctx, self.Nx, self.Nt = ctx, Nx, Nt
        self.h = C.c_void_p()
        ctx.check(lib().dmg_gauge_create(ctx.h, Nx, Nt, theta.ctypes.data_as(C.c_void_p), int(antiperiodic),
                                         C.byref(self.h)), "gauge_create")
        _register(self)

    def close(self):
        if self.h:
            lib().dmg_gauge_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def apply_dirac(ctx: Context, g: Gauge, m0: float, x, out, dagger: bool = False, nrhs: int = 1):
    prec = FP32 if str(getattr(x, "dtype", "")).endswith("complex64") else FP64
    pin, kind = _ptr(x)
    pout, kind2 = _ptr(out)
    assert kind == kind2
    ctx.check(lib().dmg_apply_dirac(ctx.h, g.h, m0, int(dagger), prec, pin, pout, nrhs, kind), "apply_dirac")
    return out


class Hierarchy:
    def __init__(self, ctx: Context, g: Gauge, m0: float, start0, start1, inject: bool = False, params=None):
        self.ctx, self.g, self.m0 = ctx, g, m0
        p0, k0 = _ptr(start0)
        p1, k1 = _ptr(start1)
        assert k0 == k1
        prm = params or setup_params()
        self.h = C.c_void_p()
        ctx.check(lib().dmg_setup(ctx.h, g.h, m0, C.byref(prm), p0, p1, int(inject), k0, C.byref(self.h)), "setup")
        _register(self)

    def part_bytes(self, level, part) -> int:
        return lib().dmg_hierarchy_part_bytes(self.h, level, part)

    def export(self, level: int, part: int) -> np.ndarray:
        nb = self.part_bytes(level, part)
        if nb == 0:
            raise ValueError("no such part on this level")
        buf = np.empty(nb // 4, dtype=np.int32) if part == PART_SETUP_ITERS else np.empty(nb // 16, dtype=complex)
        self.ctx.check(lib().dmg_hierarchy_export(self.h, level, part, buf.ctypes.data_as(C.c_void_p), nb), "export")
        return buf

    def apply(self, level: int, op: int, x, out, bf16: bool = False, bf16c: bool = False):
        """Operator / transfer hook on single fields (bf16: complex64 fields, level-1 blocks in BF16;
        bf16c: complex64 fields, level-2 blocks rounded to BF16)."""
        prec = FP32 if str(getattr(x, "dtype", "")).endswith("complex64") else FP64
        if bf16:
            prec = FP32_BF16
        if bf16c:
            prec = FP32_BF16C
        pin, kind = _ptr(x)
        pout, _ = _ptr(out)
        self.ctx.check(lib().dmg_hierarchy_apply(self.h, level, op, prec, pin, pout, kind), "hierarchy_apply")
        return out

    def apply_batched(self, level: int, op: int, x, out, nrhs: int, mfma: bool = True, bf16: bool = False):
        """The multi-right-hand-side kernels on nrhs consecutive fields."""
        prec = FP32 if str(getattr(x, "dtype", "")).endswith("complex64") else FP64
        if bf16:
            prec = FP32_BF16
        pin, kind = _ptr(x)
        pout, _ = _ptr(out)
        self.ctx.check(lib().dmg_hierarchy_apply_batched(self.h, level, op, prec, pin, pout, nrhs, kind,
                                                         1 if mfma else 0), "hierarchy_apply_batched")
        return out

    def apply_batched_static(self, level: int, op: int, x, out, nrhs: int, mfma: bool = True, bf16: bool = False):
        """apply_batched without device allocation (the library's static scratch array); device
        tensors only, stream-ordered on the context's stream."""
        prec = FP32 if str(getattr(x, "dtype", "")).endswith("complex64") else FP64
        if bf16:
            prec = FP32_BF16
        pin, kind = _ptr(x)
        pout, kind2 = _ptr(out)
        if kind != PTR_DEVICE or kind2 != PTR_DEVICE:
            raise ValueError("apply_batched_static takes device tensors")
        self.ctx.check(lib().dmg_hierarchy_apply_batched_static(self.h, level, op, prec, pin, pout, nrhs,
                                                                1 if mfma else 0), "hierarchy_apply_batched_static")
        return out

    def close(self):
        if self.h:
            lib().dmg_hierarchy_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Deflation:
    def __init__(self, hier: Hierarchy, m: int = 30, k: int = 10):
        self.hier = hier
        self.h = C.c_void_p()
        hier.ctx.check(lib().dmg_deflation_create(hier.h, m, k, C.byref(self.h)), "deflation_create")
        _register(self)

    def build(self, rhs, tol: float = 1e-8):
        p, kind = _ptr(rhs)
        self.hier.ctx.check(lib().dmg_deflation_build(self.h, p, tol, kind), "deflation_build")

    def reset(self):
        lib().dmg_deflation_reset(self.h)

    @property
    def ready(self) -> bool:
        return bool(lib().dmg_deflation_ready(self.h))

    def export(self, n_coarse: int):
        k = C.c_int()
        self.hier.ctx.check(lib().dmg_deflation_export(self.h, None, None, C.byref(k)), "deflation_export")
        V = np.empty((k.value + 1) * n_coarse, dtype=complex)
        H = np.empty((k.value + 1) * k.value, dtype=complex)
        self.hier.ctx.check(lib().dmg_deflation_export(self.h, V.ctypes.data_as(C.c_void_p),
                                                       H.ctypes.data_as(C.c_void_p), None), "deflation_export")
        return V.reshape(k.value + 1, n_coarse).T.copy(), H.reshape(k.value, k.value + 1).T.copy()

    def close(self):
        if self.h:
            lib().dmg_deflation_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


FINE_CGNE, FINE_GMRES_DR, FINE_GMRES_PROJ = 0, 1, 2


def solve_fine(ctx: Context, hier: Hierarchy, method: int, b, x, nrhs: int = 1, tol: float = 1e-8,
               max_iters: int = 100000, m: int = 40, k: int = 10):
    """Fine-grid comparison solvers without multigrid; returns (status, [stats dicts])."""
    pb, kb = _ptr(b)
    px, kx = _ptr(x)
    assert kb == kx
    stats = (SolveStats * nrhs)()
    st = lib().dmg_solve_fine(ctx.h, hier.h, method, m, k, tol, max_iters, pb, px, nrhs, kb, stats)
    ctx.check(st, "solve_fine")
    return st, [s.as_dict() for s in stats]


def autotune(mode: int = 1) -> None:
    """Autotuning of the lockstep stencils' launch forms: 0 off, 1 on, 2 on and forget choices."""
    st = lib().dmg_autotune(mode)
    if st != 0:
        raise DmgError(st, "autotune: mode")


def autotune_force(kernel: int, form: int) -> None:
    """Use launch form `form` of TUNE_BLOCK / TUNE_WILSON for every shape (-1: tuned choice)."""
    st = lib().dmg_autotune_force(kernel, form)
    if st != 0:
        raise DmgError(st, "autotune_force")


def autotune_report() -> str:
    n = lib().dmg_autotune_report(None, 0)
    buf = C.create_string_buffer(n)
    lib().dmg_autotune_report(buf, n)
    return buf.value.decode()


def solve_batched(ctx: Context, hier: Hierarchy, defl, b, x, nrhs: int, params: SolveParams | None = None):
    """Solve D x = b for nrhs right-hand sides jointly (lockstep); returns (status, [stats dicts])."""
    prm = params or solve_params()
    pb, kb = _ptr(b)
    px, kx = _ptr(x)
    assert kb == kx
    stats = (SolveStats * nrhs)()
    st = lib().dmg_solve_batched(ctx.h, hier.h, defl.h if defl is not None else None, C.byref(prm), pb, px, nrhs,
                                 kb, stats)
    ctx.check(st, "solve_batched")
    return st, [s.as_dict() for s in stats]


def solve(ctx: Context, hier: Hierarchy, defl, b, x, nrhs: int = 1, params: SolveParams | None = None):
    """Solve D x = b (nrhs right-hand sides back to back); returns (status, [stats dicts])."""
    prm = params or solve_params()
    pb, kb = _ptr(b)
    px, kx = _ptr(x)
    assert kb == kx
    stats = (SolveStats * nrhs)()
    st = lib().dmg_solve(ctx.h, hier.h, defl.h if defl is not None else None, C.byref(prm), pb, px, nrhs, kb, stats)
    ctx.check(st, "solve")
    return st, [s.as_dict() for s in stats]


class Pool:
    """Slots of concurrent independent solves of any resident hierarchy; see dmg_pool_* in dmg.h."""

    def __init__(self, ctx: Context, capacity: int, params: SolveParams | None = None):
        self.ctx = ctx
        self.capacity = capacity
        self.h = C.c_void_p()
        prm = params or solve_params()
        ctx.check(lib().dmg_pool_create(ctx.h, capacity, C.byref(prm), C.byref(self.h)), "pool_create")
        _register(self)

    def admit(self, slot: int, hier: Hierarchy, defl, b) -> int:
        """Admit one right-hand side; returns the status (DMG_E_BUDGET leaves the slot free)."""
        pb, kb = _ptr(b)
        st = lib().dmg_pool_admit(self.h, slot, hier.h, defl.h if defl is not None else None, pb, kb)
        if st != DMG_E_BUDGET:
            self.ctx.check(st, "pool_admit")
        return st

    def step(self, min_iters: int = 1) -> int:
        n = C.c_int()
        self.ctx.check(lib().dmg_pool_step(self.h, min_iters, C.byref(n)), "pool_step")
        return n.value

    def state(self, slot: int) -> int:
        return lib().dmg_pool_slot_state(self.h, slot)

    def retire(self, slot: int, x):
        """Copy the slot's solution into x; returns (status, stats dict).  Errors raise."""
        px, kx = _ptr(x)
        stats = SolveStats()
        st = lib().dmg_pool_retire(self.h, slot, px, kx, C.byref(stats))
        self.ctx.check(st, "pool_retire")
        return st, stats.as_dict()

    def close(self):
        if self.h:
            lib().dmg_pool_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Lockstep lanes of one hierarchy with continuous admission; see dmg_batch_* in dmg.h."""

    def __init__(self, hier: Hierarchy, defl, capacity: int, params: SolveParams | None = None):
        self.hier = hier
        self.ctx = hier.ctx
        self.capacity = capacity
        self.h = C.c_void_p()
        prm = params or solve_params()
        self.ctx.check(lib().dmg_batch_create(hier.h, defl.h, capacity, C.byref(prm), C.byref(self.h)),
                       "batch_create")
        _register(self)

    def admit(self, slot: int, b) -> int:
        pb, kb = _ptr(b)
        st = lib().dmg_batch_admit(self.h, slot, pb, kb)
        if st != DMG_E_BUDGET:
            self.ctx.check(st, "batch_admit")
        return st

    def step(self, min_iters: int = 1) -> int:
        n = C.c_int()
        self.ctx.check(lib().dmg_batch_step(self.h, min_iters, C.byref(n)), "batch_step")
        return n.value

    def state(self, slot: int) -> int:
        return lib().dmg_batch_slot_state(self.h, slot)

    def retire(self, slot: int, x):
        px, kx = _ptr(x)
        stats = SolveStats()
        st = lib().dmg_batch_retire(self.h, slot, px, kx, C.byref(stats))
        self.ctx.check(st, "batch_retire")
        return st, stats.as_dict()

    def close(self):
        if self.h:
            lib().dmg_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
