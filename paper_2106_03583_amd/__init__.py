"""Python binding of libmbp (the multi-block FFT-accelerated Poisson solver).

Argument marshalling only: every step of a solve runs in the HIP library.
PyTorch supplies device memory (float64 CUDA/HIP tensors) and streams.

    import paper_2106_03583_amd as mbp
    plan = mbp.Plan(problem)                  # problem: workloads.Problem-like
    info = plan.solve(rhs, p, rtol=1e-10)     # rhs, p: float64 device tensors

The library is loaded from this directory (libmbp.so, built by
``paper_2106_03583_amd/build.py``); importing fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbp.so")

OK, PENDING = 0, 1
ERR_INVALID, ERR_NOMEM, ERR_HIP, ERR_NOT_CONVERGED = -1, -2, -3, -4
ERR_NONFINITE, ERR_INCOMPATIBLE, ERR_BUSY, ERR_TOO_LARGE, ERR_NO_DEVICE = -5, -6, -7, -8, -9
DIRICHLET, NEUMANN, CONNECT, PERIODIC = 1, 2, 3, 4
FP64, MIXED = 0, 1
PROJECT_RHS, WARM_START, RETIRE, AUTOTUNE = 1, 2, 4, 8


class BlockDesc(C.Structure):
    _fields_ = [("lo", C.c_int32 * 2), ("hi", C.c_int32 * 2), ("xf", C.POINTER(C.c_double)),
                ("yf", C.POINTER(C.c_double)), ("bc", C.c_int32 * 4)]


class SynthDesc(C.Structure):
    _fields_ = [("nz", C.c_int32), ("lz", C.c_double), ("bc_lo", C.c_int32), ("bc_hi", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("max_cycles", C.c_int32), ("flags", C.c_int32), ("etol", C.c_double), ("inner", C.c_int32),
                ("march", C.c_int32), ("smoother", C.c_int32), ("helmholtz", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("cycles", C.c_int32), ("rel_residual", C.c_double),
                ("removed_mean", C.c_double), ("cycles_per_mode", C.POINTER(C.c_int32)),
                ("t_ms", C.c_double * 4)]


class ProfileInfo(C.Structure):
    _fields_ = [("launches", C.c_int64 * 2), ("total_ms", C.c_double * 2), ("cells", C.c_double * 2)]


class Tuning(C.Structure):
    _fields_ = [("wg_target", C.c_int32), ("levels", C.c_int32), ("form", C.c_int32 * 16),
                ("ms_default", C.c_double), ("ms_tuned", C.c_double)]


class PlanSummary(C.Structure):
    _fields_ = [("ncells", C.c_int64), ("nlevels", C.c_int32), ("coarse_cells", C.c_int32),
                ("singular", C.c_int32), ("nblocks", C.c_int32), ("workspace_bytes", C.c_int64),
                ("nbr", (C.c_int32 * 4) * 64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libmbp.so not built at {LIB_PATH}; run python paper_2106_03583_amd/build.py")
    # torch carries its own HIP runtime under the same soname as the system
    # one libmbp.so links against.  Loaded first, it is the one runtime of the
    # process and libmbp.so binds to it; the other way round the process ends
    # up with the system runtime under torch, and the library finds no device.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, I, D, VP = C.c_void_p, C.c_int, C.c_double, C.c_void_p
    sig = {
        "mbp_status_string": (C.c_char_p, [I]),
        "mbp_version": (I, []),
        "mbp_grid_tanh": (I, [I, D, D, I, D, C.POINTER(D)]),
        "mbp_plan_check": (I, [C.POINTER(BlockDesc), I, C.POINTER(SynthDesc), C.POINTER(Options),
                               C.POINTER(PlanSummary)]),
        "mbp_plan_create": (I, [C.POINTER(BlockDesc), I, C.POINTER(SynthDesc), C.POINTER(Options),
                                C.POINTER(P)]),
        "mbp_plan_layout": (I, [P, C.POINTER(C.c_int64), C.POINTER(C.c_size_t), C.POINTER(I)]),
        "mbp_plan_set_helmholtz": (I, [P, D]),
        "mbp_solve": (I, [P, VP, VP, D, I, VP, C.POINTER(SolveInfo)]),
        "mbp_solve_batch": (I, [C.POINTER(P), C.POINTER(VP), C.POINTER(VP), I, D, I, VP,
                                C.POINTER(SolveInfo)]),
        "mbp_batch_schedule": (I, [C.POINTER(P), I, C.POINTER(I), C.POINTER(I)]),
        "mbp_forward_transform": (I, [P, VP, VP, VP]),
        "mbp_inverse_transform": (I, [P, VP, VP, VP]),
        "mbp_apply_operator": (I, [P, VP, VP, VP]),
        "mbp_residual_norm": (I, [P, VP, VP, D, VP, VP]),
        "mbp_velocity_layout": (I, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
        "mbp_divergence": (I, [P, VP, VP, VP, D, VP, VP]),
        "mbp_project": (I, [P, VP, VP, VP, D, VP, VP, D, I, VP, C.POINTER(SolveInfo)]),
        "mbp_residual_norm_noalloc": (I, [P, VP, VP, D, VP, VP]),
        "mbp_noalloc_scratch_bytes": (C.c_size_t, []),
        "mbp_modal_shift": (I, [P, C.POINTER(D)]),
        "mbp_plan_destroy": (None, [P]),
        "mbp_profile_enable": (I, [P, I]),
        "mbp_plan_autotune": (I, [P, VP, VP, C.POINTER(Tuning)]),
        "mbp_profile_read": (I, [P, C.POINTER(ProfileInfo)]),
        "mbp_server_create": (I, [C.c_size_t, I, C.POINTER(Options), C.POINTER(P)]),
        "mbp_server_submit": (I, [P, C.POINTER(BlockDesc), I, C.POINTER(SynthDesc), VP, VP, D, I,
                                  C.POINTER(C.c_uint64)]),
        "mbp_server_poll": (I, [P, C.c_uint64, C.POINTER(SolveInfo), C.POINTER(D)]),
        "mbp_server_wait": (I, [P, C.c_uint64, C.POINTER(SolveInfo), C.POINTER(D)]),
        "mbp_server_destroy": (None, [P]),
        "mbp3_plan_create": (I, [C.POINTER(BlockDesc), I, C.POINTER(SynthDesc), C.POINTER(Options),
                                 C.POINTER(P)]),
        "mbp3_plan_levels": (I, [P, C.POINTER(I), C.POINTER(I), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]),
        "mbp3_jacobi_sweep": (I, [P, VP, VP, VP, VP]),
        "mbp3_solve": (I, [P, VP, VP, D, I, VP, C.POINTER(SolveInfo)]),
        "mbp3_plan_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()

EXPORTED = [
    "mbp_status_string", "mbp_version", "mbp_grid_tanh", "mbp_plan_check", "mbp_plan_create",
    "mbp_plan_layout", "mbp_solve", "mbp_solve_batch", "mbp_forward_transform",
    "mbp_inverse_transform", "mbp_apply_operator", "mbp_residual_norm", "mbp_residual_norm_noalloc",
    "mbp_noalloc_scratch_bytes", "mbp_velocity_layout", "mbp_divergence", "mbp_project", "mbp_modal_shift", "mbp_plan_destroy",
    "mbp_server_create", "mbp_server_submit", "mbp_server_poll", "mbp_server_wait",
    "mbp_server_destroy", "mbp_profile_enable", "mbp_profile_read", "mbp_batch_schedule",
    "mbp_plan_autotune", "mbp_plan_set_helmholtz",
    "mbp3_plan_create", "mbp3_plan_levels", "mbp3_solve", "mbp3_plan_destroy", "mbp3_jacobi_sweep",
]


class MBPError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        msg = lib.mbp_status_string(status).decode()
        super().__init__(f"{where}: {msg} ({status})" if where else f"{msg} ({status})")


def _check(status: int, where: str):
    if status != OK:
        raise MBPError(status, where)


def status_string(status: int) -> str:
    return lib.mbp_status_string(status).decode()


def grid_tanh(n: int, lmin: float, lmax: float, gtype: int = 0, factor: float = 0.0) -> np.ndarray:
    out = np.empty(n + 1, dtype=np.float64)
    _check(lib.mbp_grid_tanh(n, lmin, lmax, gtype, factor, out.ctypes.data_as(C.POINTER(C.c_double))),
           "mbp_grid_tanh")
    return out


class _Desc:
    """ctypes descriptors of a problem; keeps the face arrays alive."""

    def __init__(self, problem):
        self.faces = []
        blocks = list(problem.blocks)
        self.blocks = (BlockDesc * len(blocks))()
        for i, b in enumerate(blocks):
            xf = np.ascontiguousarray(b.xf, dtype=np.float64)
            yf = np.ascontiguousarray(b.yf, dtype=np.float64)
            self.faces += [xf, yf]
            d = self.blocks[i]
            d.lo[0], d.lo[1] = int(b.lo[0]), int(b.lo[1])
            d.hi[0], d.hi[1] = int(b.hi[0]), int(b.hi[1])
            d.xf = xf.ctypes.data_as(C.POINTER(C.c_double))
            d.yf = yf.ctypes.data_as(C.POINTER(C.c_double))
            for f in range(4):
                d.bc[f] = int(b.bc[f])
        self.nblocks = len(blocks)
        self.z = SynthDesc(int(problem.nz), float(problem.lz), int(problem.zbc[0]), int(problem.zbc[1]))


SMOOTHER_DEFAULT, SMOOTHER_RBGS, SMOOTHER_JACOBI = 0, 1, 2


def _options(precision="fp64", nu1=1, nu2=1, max_cycles=100, flags=0, etol=0.0, inner=0, march=0,
             smoother=SMOOTHER_DEFAULT, helmholtz=0.0) -> Options:
    prec = {"fp64": FP64, "mixed": MIXED, FP64: FP64, MIXED: MIXED}[precision]
    return Options(prec, nu1, nu2, max_cycles, flags, etol, inner, march, smoother, float(helmholtz))


def plan_check(problem, **opts) -> dict:
    d = _Desc(problem)
    s = PlanSummary()
    o = _options(**opts)
    _check(lib.mbp_plan_check(d.blocks, d.nblocks, C.byref(d.z), C.byref(o), C.byref(s)), "mbp_plan_check")
    return {
        "ncells": s.ncells, "nlevels": s.nlevels, "coarse_cells": s.coarse_cells,
        "singular": bool(s.singular), "nblocks": s.nblocks, "workspace_bytes": s.workspace_bytes,
        "nbr": [[s.nbr[b][f] for f in range(4)] for b in range(min(s.nblocks, 64))],
    }


def plan_check_status(problem, **opts) -> int:
    d = _Desc(problem)
    o = _options(**opts)
    return lib.mbp_plan_check(d.blocks, d.nblocks, C.byref(d.z), C.byref(o), None)


def _ptr(t, numel=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"tensor has {t.numel()} elements, the plan needs {numel}")
    if t.device.type != "cuda":
        raise ValueError("tensor must live on the GPU")
    if t.dtype != torch.float64:
        raise ValueError("tensor must be float64")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Info:
    def __init__(self, si: SolveInfo, cycles_per_mode: Optional[np.ndarray]):
        self.status = si.status
        self.cycles = si.cycles
        self.rel_residual = si.rel_residual
        self.removed_mean = si.removed_mean
        self.cycles_per_mode = cycles_per_mode
        self.t_ms = list(si.t_ms)

    def __repr__(self):
        return (f"Info(status={self.status}, cycles={self.cycles}, rel_residual={self.rel_residual:.3e}, "
                f"t_ms={[round(t, 3) for t in self.t_ms]})")


class Plan:
    def __init__(self, problem, precision="fp64", nu1=1, nu2=1, max_cycles=100, flags=0, etol=0.0, inner=0,
                 march=0, smoother=SMOOTHER_DEFAULT, helmholtz=0.0):
        self.problem = problem
        self._desc = _Desc(problem)
        self._opt = _options(precision, nu1, nu2, max_cycles, flags, etol, inner, march, smoother, helmholtz)
        self._h = C.c_void_p()
        _check(lib.mbp_plan_create(self._desc.blocks, self._desc.nblocks, C.byref(self._desc.z),
                                   C.byref(self._opt), C.byref(self._h)), "mbp_plan_create")
        self.nz = int(problem.nz)
        nb = self._desc.nblocks
        off = (C.c_int64 * (nb + 1))()
        ws = C.c_size_t()
        sing = C.c_int()
        _check(lib.mbp_plan_layout(self._h, off, C.byref(ws), C.byref(sing)), "mbp_plan_layout")
        self.block_offsets = [off[i] for i in range(nb + 1)]
        self.ncells = self.block_offsets[-1]
        self.workspace_bytes = ws.value
        self.singular = bool(sing.value)

    @property
    def handle(self):
        return self._h

    def set_helmholtz(self, alpha: float):
        """Solve (L_h - alpha) p = f from now on (alpha >= 0)."""
        _check(lib.mbp_plan_set_helmholtz(self._h, float(alpha)), "mbp_plan_set_helmholtz")
        sing = C.c_int()
        _check(lib.mbp_plan_layout(self._h, None, None, C.byref(sing)), "mbp_plan_layout")
        self.singular = bool(sing.value)

    def solve(self, rhs, p, rtol=1e-10, flags=0, stream=None, raise_on_error=True) -> Info:
        cpm = np.zeros(self.nz, dtype=np.int32)
        si = SolveInfo()
        si.cycles_per_mode = cpm.ctypes.data_as(C.POINTER(C.c_int32))
        st = lib.mbp_solve(self._h, _ptr(rhs, self.ncells), _ptr(p, self.ncells), float(rtol),
                           int(flags), _stream(stream), C.byref(si))
        if raise_on_error and st != OK:
            raise MBPError(st, "mbp_solve")
        si.status = st if si.status == 0 else si.status
        return Info(si, cpm)

    def forward(self, f, fhat, stream=None):
        _check(lib.mbp_forward_transform(self._h, _ptr(f, self.ncells), _ptr(fhat, self.ncells),
                                         _stream(stream)), "forward")

    def inverse(self, phat, p, stream=None):
        _check(lib.mbp_inverse_transform(self._h, _ptr(phat, self.ncells), _ptr(p, self.ncells),
                                         _stream(stream)), "inverse")

    def apply(self, p, out, stream=None):
        _check(lib.mbp_apply_operator(self._h, _ptr(p, self.ncells), _ptr(out, self.ncells),
                                      _stream(stream)), "apply")

    def residual_norm(self, rhs, p, rhs_shift=0.0, out=None, stream=None):
        """(||f - s - L_h p||, ||f - s||) as a 2-element float64 device tensor."""
        import torch
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=rhs.device)
        _check(lib.mbp_residual_norm(self._h, _ptr(rhs, self.ncells), _ptr(p, self.ncells), float(rhs_shift),
                                     _ptr(out, 2), _stream(stream)), "mbp_residual_norm")
        return out

    def velocity_sizes(self):
        """Element counts of the packed face fields u, v, w."""
        nb = self._desc.nblocks
        uo, vo, wo = (C.c_int64 * (nb + 1))(), (C.c_int64 * (nb + 1))(), (C.c_int64 * (nb + 1))()
        _check(lib.mbp_velocity_layout(self._h, uo, vo, wo), "mbp_velocity_layout")
        return uo[nb], vo[nb], wo[nb]

    def divergence(self, u, v, w, out, scale=1.0, stream=None):
        nu, nv, nw = self.velocity_sizes()
        _check(lib.mbp_divergence(self._h, _ptr(u, nu), _ptr(v, nv), _ptr(w, nw), float(scale),
                                  _ptr(out, self.ncells), _stream(stream)), "mbp_divergence")

    def project(self, u, v, w, gamma_dt, phi, work, rtol=1e-10, flags=0, stream=None, raise_on_error=True) -> Info:
        """u, v, w -= gamma_dt G Phi with L_h Phi = D u / gamma_dt (in place)."""
        nu, nv, nw = self.velocity_sizes()
        cpm = np.zeros(self.nz, dtype=np.int32)
        si = SolveInfo()
        si.cycles_per_mode = cpm.ctypes.data_as(C.POINTER(C.c_int32))
        st = lib.mbp_project(self._h, _ptr(u, nu), _ptr(v, nv), _ptr(w, nw), float(gamma_dt),
                             _ptr(phi, self.ncells), _ptr(work, self.ncells), float(rtol), int(flags),
                             _stream(stream), C.byref(si))
        if raise_on_error and st != OK:
            raise MBPError(st, "mbp_project")
        si.status = st if si.status == 0 else si.status
        return Info(si, cpm)

    def modal_shift(self) -> np.ndarray:
        out = np.empty(self.nz, dtype=np.float64)
        _check(lib.mbp_modal_shift(self._h, out.ctypes.data_as(C.POINTER(C.c_double))), "modal_shift")
        return out

    def autotune(self, rhs, stream=None) -> dict:
        """Pick the fastest schedule for this plan by timing short runs on rhs."""
        t = Tuning()
        _check(lib.mbp_plan_autotune(self._h, _ptr(rhs, self.ncells), _stream(stream), C.byref(t)),
               "mbp_plan_autotune")
        return {"wg_target": t.wg_target, "form": list(t.form)[:t.levels], "ms_default": t.ms_default,
                "ms_tuned": t.ms_tuned}

    def profile(self, enable: bool = True):
        _check(lib.mbp_profile_enable(self._h, 1 if enable else 0), "mbp_profile_enable")

    def profile_read(self) -> dict:
        pi = ProfileInfo()
        _check(lib.mbp_profile_read(self._h, C.byref(pi)), "mbp_profile_read")
        return {"launches": list(pi.launches), "total_ms": list(pi.total_ms), "cells": list(pi.cells)}

    def close(self):
        if self._h:
            lib.mbp_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan3D:
    """The 3D multigrid solver without z synthesis (the comparison solver):
    weighted-Jacobi V-cycles on the whole 3D system, FP64."""

    def __init__(self, problem, nu1=2, nu2=2, max_cycles=100, flags=0, helmholtz=0.0, etol=0.0):
        self.problem = problem
        self._desc = _Desc(problem)
        self._opt = _options("fp64", nu1, nu2, max_cycles, flags, etol, 0, 0, SMOOTHER_JACOBI, helmholtz)
        self._h = C.c_void_p()
        _check(lib.mbp3_plan_create(self._desc.blocks, self._desc.nblocks, C.byref(self._desc.z),
                                    C.byref(self._opt), C.byref(self._h)), "mbp3_plan_create")
        self.nz = int(problem.nz)
        self.ncells = int(problem.ncells)
        n = C.c_int()
        _check(lib.mbp3_plan_levels(self._h, C.byref(n), None, None, None), "mbp3_plan_levels")
        nzl = (C.c_int * n.value)()
        cl = (C.c_int64 * n.value)()
        ws = C.c_size_t()
        _check(lib.mbp3_plan_levels(self._h, None, nzl, cl, C.byref(ws)), "mbp3_plan_levels")
        self.nlevels = n.value
        self.nz_per_level = list(nzl)
        self.cells_per_level = list(cl)
        self.workspace_bytes = ws.value

    def jacobi_sweep(self, pin, pout, f, stream=None):
        """One weighted-Jacobi sweep of the finest level (out of place)."""
        _check(lib.mbp3_jacobi_sweep(self._h, _ptr(pin, self.ncells), _ptr(pout, self.ncells),
                                     _ptr(f, self.ncells), _stream(stream)), "mbp3_jacobi_sweep")

    def solve(self, rhs, p, rtol=1e-10, flags=0, stream=None, raise_on_error=True) -> Info:
        si = SolveInfo()
        st = lib.mbp3_solve(self._h, _ptr(rhs, self.ncells), _ptr(p, self.ncells), float(rtol), int(flags),
                            _stream(stream), C.byref(si))
        if raise_on_error and st != OK:
            raise MBPError(st, "mbp3_solve")
        si.status = st if si.status == 0 else si.status
        return Info(si, None)

    def close(self):
        if self._h:
            lib.mbp3_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(plans: Sequence[Plan], rhs: Sequence, p: Sequence, rtol=1e-10, flags=0, stream=None,
                raise_on_error=True):
    n = len(plans)
    hs = (C.c_void_p * n)(*[pl.handle.value for pl in plans])
    rs = (C.c_void_p * n)(*[_ptr(t, pl.ncells).value for t, pl in zip(rhs, plans)])
    ps = (C.c_void_p * n)(*[_ptr(t, pl.ncells).value for t, pl in zip(p, plans)])
    infos = (SolveInfo * n)()
    cpms = []
    for i, pl in enumerate(plans):
        cpm = np.zeros(pl.nz, dtype=np.int32)
        cpms.append(cpm)
        infos[i].cycles_per_mode = cpm.ctypes.data_as(C.POINTER(C.c_int32))
    st = lib.mbp_solve_batch(hs, rs, ps, n, float(rtol), int(flags), _stream(stream), infos)
    if raise_on_error and st != OK:
        raise MBPError(st, "mbp_solve_batch")
    return [Info(infos[i], cpms[i]) for i in range(n)]


def batch_schedule(plans: Sequence[Plan]):
    """(streams, cycles per replay) the batch autotuner chose for this plan set, or None.
    streams is 0 when every replay of the set's last batch ran in the grouped form."""
    n = len(plans)
    hs = (C.c_void_p * n)(*[pl.handle.value for pl in plans])
    a, b = C.c_int(), C.c_int()
    st = lib.mbp_batch_schedule(hs, n, C.byref(a), C.byref(b))
    if st == PENDING:
        return None
    _check(st, "mbp_batch_schedule")
    return a.value, b.value


class Server:
    def __init__(self, hbm_budget: int, slots: int = 4, precision="mixed", nu1=1, nu2=1, max_cycles=100,
                 flags=0, etol=0.0, inner=0):
        self._opt = _options(precision, nu1, nu2, max_cycles, flags, etol, inner)
        self._h = C.c_void_p()
        _check(lib.mbp_server_create(int(hbm_budget), int(slots), C.byref(self._opt), C.byref(self._h)),
               "mbp_server_create")
        self._keep = {}

    def submit(self, problem, rhs, p, rtol=1e-10, flags=0) -> int:
        d = _Desc(problem)
        t = C.c_uint64()
        n = int(problem.nz) * sum((b.hi[0] - b.lo[0] + 1) * (b.hi[1] - b.lo[1] + 1) for b in problem.blocks)
        _check(lib.mbp_server_submit(self._h, d.blocks, d.nblocks, C.byref(d.z), _ptr(rhs, n), _ptr(p, n),
                                     float(rtol), int(flags), C.byref(t)), "mbp_server_submit")
        self._keep[t.value] = (d, rhs, p)
        return t.value

    def _info(self, ticket):
        si = SolveInfo()
        keep = self._keep.get(ticket)
        cpm = None
        if keep is not None:
            cpm = np.zeros(int(keep[0].z.nz), dtype=np.int32)
            si.cycles_per_mode = cpm.ctypes.data_as(C.POINTER(C.c_int32))
        return si, cpm

    def poll(self, ticket: int):
        si, cpm = self._info(ticket)
        lat = C.c_double()
        st = lib.mbp_server_poll(self._h, C.c_uint64(ticket), C.byref(si), C.byref(lat))
        if st == PENDING:
            return None
        self._keep.pop(ticket, None)
        return st, Info(si, cpm), lat.value

    def wait(self, ticket: int):
        si, cpm = self._info(ticket)
        lat = C.c_double()
        st = lib.mbp_server_wait(self._h, C.c_uint64(ticket), C.byref(si), C.byref(lat))
        self._keep.pop(ticket, None)
        return st, Info(si, cpm), lat.value

    def close(self):
        if self._h:
            lib.mbp_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
