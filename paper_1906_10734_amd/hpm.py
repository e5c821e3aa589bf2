"""ctypes binding of libhpm.so (include/hpm.h). Argument marshalling only: every step of the
method runs in the library's HIP kernels; torch provides device memory and the stream.

The library is loaded from this package's directory. If it is missing the import of this
module raises, so no caller can fall back to another implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhpm.so")

HPM_ABI_VERSION = 6
HPM_F64, HPM_F32 = 0, 1
HPM_KERNELS = {"newton": 0, "yukawa": 1}
HPM_M2L_MODES = {"grid": 0, "cells": 1, "shared": 2}
STATUS = {0: "HPM_OK", 1: "HPM_ERR_INVALID_ARG", 2: "HPM_ERR_OUT_OF_BOX", 3: "HPM_ERR_NONFINITE",
          4: "HPM_ERR_NO_MEMORY", 5: "HPM_ERR_DEVICE", 6: "HPM_ERR_UNSUPPORTED",
          7: "HPM_ERR_NOT_READY"}
HPM_ERR_NOT_READY = 7

# Entry points declared in include/hpm.h: name -> (restype, argtypes)
_vp, _i32, _i64, _d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double


class HpmProblem(ctypes.Structure):
    _fields_ = [("abi", ctypes.c_int32), ("ng", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("uniform_depth", ctypes.c_int32), ("leaf_capacity", ctypes.c_int32),
                ("max_depth", ctypes.c_int32), ("softening", ctypes.c_double),
                ("gconst", ctypes.c_double), ("box_lo", ctypes.c_double * 3),
                ("box_size", ctypes.c_double), ("kernel", ctypes.c_int32),
                ("m2l_mode", ctypes.c_int32), ("screening", ctypes.c_double),
                ("extended", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class HpmPlanInfo(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("ng", ctypes.c_int32),
                ("n_particles", ctypes.c_int64), ("n_cells", ctypes.c_int64),
                ("n_leaves", ctypes.c_int64), ("n_targets", ctypes.c_int64),
                ("cells_per_level", ctypes.c_int64 * 11), ("p2p_pairs", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64)]


class HpmServerConfig(ctypes.Structure):
    _fields_ = [("abi", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("hbm_budget", ctypes.c_int64), ("reserved", ctypes.c_int32 * 4)]


class HpmRequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slot", ctypes.c_int32), ("n", ctypes.c_int64),
                ("submit_ms", ctypes.c_double), ("start_ms", ctypes.c_double),
                ("done_ms", ctypes.c_double), ("plan_bytes", ctypes.c_int64),
                ("estimate_bytes", ctypes.c_int64)]


class HpmServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("queued", ctypes.c_int32),
                ("running", ctypes.c_int32), ("plans", ctypes.c_int64),
                ("held_bytes", ctypes.c_int64), ("peak_held_bytes", ctypes.c_int64),
                ("plans_created", ctypes.c_int64), ("plans_released", ctypes.c_int64)]


SIGNATURES = {
    "hpm_status_string": (ctypes.c_char_p, [_i32]),
    "hpm_last_error": (ctypes.c_char_p, []),
    "hpm_abi_version": (_i32, []),
    "hpm_plan_create": (_i32, [ctypes.POINTER(HpmProblem), _i64, _vp, _vp, _vp, _vp,
                               ctypes.POINTER(_vp)]),
    "hpm_plan_execute": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "hpm_plan_destroy": (None, [_vp]),
    "hpm_plan_rebuild": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp]),
    "hpm_plan_enable_timing": (_i32, [_vp, _i32]),
    "hpm_plan_stage_times": (_i32, [_vp, _vp, _vp, _vp]),
    "hpm_solve": (_i32, [ctypes.POINTER(HpmProblem), _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                         _vp]),
    "hpm_solve_noalloc": (_i32, [ctypes.POINTER(HpmProblem), _i64, _vp, _vp, _vp, _vp, _vp, _vp,
                                 _vp, _vp, _vp]),
    "hpm_plan_info_get": (_i32, [_vp, ctypes.POINTER(HpmPlanInfo)]),
    "hpm_plan_copy_perm": (_i32, [_vp, _vp]),
    "hpm_plan_copy_cells": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "hpm_plan_copy_gridlets": (_i32, [_vp, _i32, _vp]),
    "hpm_plan_copy_locals": (_i32, [_vp, _i32, _vp]),
    "hpm_plan_copy_local_offsets": (_i32, [_vp, _i32, _vp]),
    "hpm_direct_sum": (_i32, [_i32, _i64, _vp, _vp, _vp, _vp, _i64, _vp, _d, _d, _i32, _d, _vp,
                              _vp, _vp, _vp, _vp]),
    "hpm_plan_set_route": (_i32, [_vp, _i32]),
    "hpm_plan_set_overlap": (_i32, [_vp, _i32]),
    "hpm_plan_set_fp32_strict": (_i32, [_vp, _i32]),
    "hpm_plan_autotune": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, ctypes.POINTER(_i32),
                                 ctypes.POINTER(_d)]),
    "hpm_plan_bytes_estimate": (_i32, [ctypes.POINTER(HpmProblem), _i64,
                                       ctypes.POINTER(_i64)]),
    "hpm_server_create": (_i32, [ctypes.POINTER(HpmServerConfig), ctypes.POINTER(_vp)]),
    "hpm_server_submit": (_i32, [_vp, ctypes.POINTER(HpmProblem), _i64, _vp, _vp, _vp, _vp, _vp,
                                 _vp, _vp, _vp, ctypes.POINTER(ctypes.c_uint64)]),
    "hpm_server_poll": (_i32, [_vp, ctypes.c_uint64, ctypes.POINTER(HpmRequestInfo)]),
    "hpm_server_wait": (_i32, [_vp, ctypes.c_uint64, ctypes.POINTER(HpmRequestInfo)]),
    "hpm_server_run_batch": (_i32, [_vp, _i32, ctypes.POINTER(HpmProblem),
                                    ctypes.POINTER(_i64)] + [ctypes.POINTER(_vp)] * 8 +
                             [ctypes.POINTER(_i32)]),
    "hpm_server_stats_get": (_i32, [_vp, ctypes.POINTER(HpmServerStats)]),
    "hpm_server_destroy": (None, [_vp]),
}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1906_10734_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.hpm_abi_version() != HPM_ABI_VERSION:
        raise ImportError("libhpm.so ABI version mismatch")
    return lib


_lib = load_library()


class HpmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = STATUS.get(status, str(status))
        super().__init__(f"{where}: {self.status}: {_lib.hpm_last_error().decode()}")


def _check(status: int, where: str):
    if status != 0:
        raise HpmError(status, where)


@dataclass
class Problem:
    ng: int = 4
    precision: str = "f32"          # "f32" or "f64"
    uniform_depth: int = 0
    leaf_capacity: int = 64
    max_depth: int = 10
    softening: float = 1e-3
    gconst: float = 1.0
    box_lo: tuple = (0.0, 0.0, 0.0)
    box_size: float = 1.0
    kernel: str = "newton"          # "newton" or "yukawa" (screened, needs screening > 0)
    screening: float = 0.0
    m2l: str = "grid"               # "grid" (the method), "cells" (cell by cell) or "shared"
                                    # (one transform per parent for its children's common cubes)
    extended: bool = False          # target gridlets widened by one node per side (cells route)

    @property
    def nl(self) -> int:
        """Target (local) gridlet nodes per axis."""
        return self.ng + (2 if self.extended else 0)

    @property
    def dtype(self) -> torch.dtype:
        return torch.float32 if self.precision == "f32" else torch.float64

    def c(self) -> HpmProblem:
        p = HpmProblem()
        p.abi = HPM_ABI_VERSION
        p.ng = self.ng
        p.precision = HPM_F32 if self.precision == "f32" else HPM_F64
        p.uniform_depth = self.uniform_depth
        p.leaf_capacity = self.leaf_capacity
        p.max_depth = self.max_depth
        p.softening = self.softening
        p.gconst = self.gconst
        for k in range(3):
            p.box_lo[k] = self.box_lo[k]
        p.box_size = self.box_size
        p.kernel = HPM_KERNELS[self.kernel]
        p.m2l_mode = HPM_M2L_MODES[self.m2l]
        p.screening = self.screening
        p.extended = 1 if self.extended else 0
        p.reserved = 0
        return p


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return int(getattr(stream, "cuda_stream", stream))


def _dev(t: torch.Tensor, dtype: torch.dtype, n: int, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or t.numel() != n or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous {dtype} with {n} elements")
    return t.data_ptr()


class Plan:
    """Tree and buffers for one particle set (hpm_plan_create); execute() evaluates masses."""

    def __init__(self, problem: Problem, x, y, z, stream=None):
        self.problem = problem
        self.n = int(x.numel())
        dt = problem.dtype
        self._c = problem.c()
        h = _vp()
        _check(_lib.hpm_plan_create(ctypes.byref(self._c), self.n, _dev(x, dt, self.n, "x"),
                                    _dev(y, dt, self.n, "y"), _dev(z, dt, self.n, "z"),
                                    _stream(stream), ctypes.byref(h)), "hpm_plan_create")
        self._h = h

    STAGES = ("tree", "p2m", "m2m", "m2l", "l2l", "leaf", "p2p")

    def rebuild(self, x, y, z, stream=None):
        n, dt = int(x.numel()), self.problem.dtype
        _check(_lib.hpm_plan_rebuild(self._h, n, _dev(x, dt, n, "x"), _dev(y, dt, n, "y"),
                                     _dev(z, dt, n, "z"), _stream(stream)), "hpm_plan_rebuild")
        self.n = n

    def enable_timing(self, on: bool = True):
        _check(_lib.hpm_plan_enable_timing(self._h, 1 if on else 0), "hpm_plan_enable_timing")

    def stage_times(self) -> dict:
        ms = (ctypes.c_double * 7)()
        ne, nb = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.hpm_plan_stage_times(self._h, ms, ctypes.byref(ne), ctypes.byref(nb)),
               "hpm_plan_stage_times")
        out = dict(zip(self.STAGES, list(ms)))
        out["n_exec"], out["n_build"] = ne.value, nb.value
        return out

    def execute(self, m, phi, ax, ay, az, stream=None):
        dt, n = self.problem.dtype, self.n
        _check(_lib.hpm_plan_execute(self._h, _dev(m, dt, n, "m"), _dev(phi, dt, n, "phi"),
                                     _dev(ax, dt, n, "ax"), _dev(ay, dt, n, "ay"),
                                     _dev(az, dt, n, "az"), _stream(stream)), "hpm_plan_execute")

    def set_fp32_strict(self, on: bool):
        """hpm_plan_set_fp32_strict: float-float instead of double in the padded-grid route's
        inverse x sums, target means and L2L constants (FP32 plans, N_g 4 and 6)."""
        _check(_lib.hpm_plan_set_fp32_strict(self._h, 1 if on else 0), "hpm_plan_set_fp32_strict")

    def set_overlap(self, on: bool):
        """hpm_plan_set_overlap: near-zone sums beside the source-to-target step (True) or in
        line after it (False)."""
        _check(_lib.hpm_plan_set_overlap(self._h, 1 if on else 0), "hpm_plan_set_overlap")

    def set_route(self, route: str):
        """Source-to-target route of later evaluations: "grid", "cells" or "shared"."""
        _check(_lib.hpm_plan_set_route(self._h, HPM_M2L_MODES[route]), "hpm_plan_set_route")

    def autotune(self, m, reps: int = 3, stream=None):
        """Times every route the plan can use and keeps the fastest: (route, {route: ms})."""
        dt, n = self.problem.dtype, self.n
        out = [torch.empty(n, dtype=dt, device=m.device) for _ in range(4)]
        mode, ms = _i32(), (_d * 3)()
        _check(_lib.hpm_plan_autotune(self._h, _dev(m, dt, n, "m"), *(o.data_ptr() for o in out),
                                      int(reps), _stream(stream), ctypes.byref(mode), ms),
               "hpm_plan_autotune")
        names = {v: k for k, v in HPM_M2L_MODES.items()}
        return names[mode.value], {names[r]: ms[r] for r in range(3) if ms[r] >= 0}

    def __call__(self, m, stream=None):
        out = [torch.empty(self.n, dtype=self.problem.dtype, device=m.device) for _ in range(4)]
        self.execute(m, *out, stream=stream)
        return tuple(out)

    def info(self) -> dict:
        i = HpmPlanInfo()
        _check(_lib.hpm_plan_info_get(self._h, ctypes.byref(i)), "hpm_plan_info_get")
        return dict(n_levels=i.n_levels, ng=i.ng, n_particles=i.n_particles, n_cells=i.n_cells,
                    n_leaves=i.n_leaves, n_targets=i.n_targets,
                    cells_per_level=list(i.cells_per_level)[:i.n_levels],
                    p2p_pairs=i.p2p_pairs, device_bytes=i.device_bytes)

    def perm(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int32)
        _check(_lib.hpm_plan_copy_perm(self._h, out.ctypes.data), "hpm_plan_copy_perm")
        return out

    def cells(self, level: int) -> dict:
        cnt = self.info()["cells_per_level"][level]
        coords = np.empty((cnt, 3), np.int32)
        pb, pe, split, parent = (np.empty(cnt, np.int32) for _ in range(4))
        _check(_lib.hpm_plan_copy_cells(self._h, level, coords.ctypes.data, pb.ctypes.data,
                                        pe.ctypes.data, split.ctypes.data, parent.ctypes.data),
               "hpm_plan_copy_cells")
        return dict(coords=coords, pb=pb, pe=pe, split=split.astype(bool), parent=parent)

    def _rows(self, fn, level: int, per_axis: int | None = None) -> np.ndarray:
        cnt = self.info()["cells_per_level"][level]
        npdt = np.float32 if self.problem.precision == "f32" else np.float64
        out = np.empty((cnt, (per_axis or self.problem.ng) ** 3), npdt)
        _check(fn(self._h, level, out.ctypes.data), fn.__name__)
        return out

    def gridlets(self, level: int) -> np.ndarray:
        return self._rows(_lib.hpm_plan_copy_gridlets, level)

    def local_parts(self, level: int):
        """(c, dPhi): per-cell constant (float64) and gridlet part (plan dtype)."""
        d = self._rows(_lib.hpm_plan_copy_locals, level, self.problem.nl)
        c = np.empty(d.shape[0], np.float64)
        _check(_lib.hpm_plan_copy_local_offsets(self._h, level, c.ctypes.data),
               "hpm_plan_copy_local_offsets")
        return c, d

    def locals(self, level: int) -> np.ndarray:
        """Local potential c + dPhi of every cell of the level, in float64."""
        c, d = self.local_parts(level)
        return c[:, None] + d.astype(np.float64)

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hpm_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()


def solve(problem: Problem, x, y, z, m, stream=None):
    """One-shot solve (hpm_solve). Returns (phi, ax, ay, az) in input order."""
    n, dt = int(x.numel()), problem.dtype
    out = [torch.empty(n, dtype=dt, device=x.device) for _ in range(4)]
    c = problem.c()
    _check(_lib.hpm_solve(ctypes.byref(c), n, _dev(x, dt, n, "x"), _dev(y, dt, n, "y"),
                          _dev(z, dt, n, "z"), _dev(m, dt, n, "m"), *(o.data_ptr() for o in out),
                          _stream(stream)), "hpm_solve")
    return tuple(out)


def solve_noalloc(problem: Problem, x, y, z, m, out=None, stream=None):
    """One-shot solve without device allocation in the library (hpm_solve_noalloc); ``out``
    (optional) is the caller's (phi, ax, ay, az). Returns (phi, ax, ay, az) in input order."""
    n, dt = int(x.numel()), problem.dtype
    if out is None:
        out = [torch.empty(n, dtype=dt, device=x.device) for _ in range(4)]
    c = problem.c()
    _check(_lib.hpm_solve_noalloc(ctypes.byref(c), n, _dev(x, dt, n, "x"), _dev(y, dt, n, "y"),
                                  _dev(z, dt, n, "z"), _dev(m, dt, n, "m"),
                                  *(_dev(o, dt, n, "out") for o in out), _stream(stream)),
           "hpm_solve_noalloc")
    return tuple(out)


def direct_sum(x, y, z, m, targets, gconst: float = 1.0, softening: float = 0.0, stream=None,
               kernel: str = "newton", screening: float = 0.0):
    """Brute-force sum of the kernel on the device in FP64 at the given input indices."""
    n = int(x.numel())
    dt = x.dtype
    prec = HPM_F32 if dt == torch.float32 else HPM_F64
    tg = targets.to(device=x.device, dtype=torch.int32).contiguous()
    out = [torch.empty(tg.numel(), dtype=torch.float64, device=x.device) for _ in range(4)]
    _check(_lib.hpm_direct_sum(prec, n, _dev(x, dt, n, "x"), _dev(y, dt, n, "y"),
                               _dev(z, dt, n, "z"), _dev(m, dt, n, "m"), tg.numel(),
                               tg.data_ptr(), gconst, softening, HPM_KERNELS[kernel], screening,
                               *(o.data_ptr() for o in out),
                               _stream(stream)), "hpm_direct_sum")
    return tuple(out)


def plan_bytes_estimate(problem: Problem, n: int) -> int:
    """hpm_plan_bytes_estimate: the server's admission measure of one request."""
    out = _i64()
    c = problem.c()
    _check(_lib.hpm_plan_bytes_estimate(ctypes.byref(c), int(n), ctypes.byref(out)),
           "hpm_plan_bytes_estimate")
    return out.value


def _request_dict(i: HpmRequestInfo) -> dict:
    return dict(status=STATUS.get(i.status, str(i.status)), slot=i.slot, n=i.n,
                submit_ms=i.submit_ms, start_ms=i.start_ms, done_ms=i.done_ms,
                latency_ms=i.done_ms - i.submit_ms, plan_bytes=i.plan_bytes,
                estimate_bytes=i.estimate_bytes)


class Server:
    """hpm_server_*: independent solves in flight on the device at once, admitted by memory.

    submit() queues one solve and returns a ticket; wait()/poll() return (info, (phi, ax, ay, az)).
    The binding keeps the request's tensors alive until it has been reported. Inputs must be
    complete on the device when submitted: submit() synchronises the current stream first.
    """

    def __init__(self, slots: int = 4, hbm_budget: int = 0):
        cfg = HpmServerConfig()
        cfg.abi = HPM_ABI_VERSION
        cfg.slots = slots
        cfg.hbm_budget = int(hbm_budget)
        h = _vp()
        _check(_lib.hpm_server_create(ctypes.byref(cfg), ctypes.byref(h)), "hpm_server_create")
        self._h = h
        self._live = {}

    def submit(self, problem: Problem, x, y, z, m, out=None, sync: bool = True) -> int:
        n, dt = int(x.numel()), problem.dtype
        if out is None:
            out = tuple(torch.empty(n, dtype=dt, device=x.device) for _ in range(4))
        ptrs = [_dev(t, dt, n, nm) for t, nm in zip((x, y, z, m) + tuple(out),
                                                   ("x", "y", "z", "m", "phi", "ax", "ay", "az"))]
        if sync:
            torch.cuda.current_stream().synchronize()
        c = problem.c()
        t = ctypes.c_uint64()
        _check(_lib.hpm_server_submit(self._h, ctypes.byref(c), n, *ptrs, ctypes.byref(t)),
               "hpm_server_submit")
        self._live[t.value] = (x, y, z, m, tuple(out))
        return t.value

    def _call(self, fn, ticket: int):
        i = HpmRequestInfo()
        i.status = -1  # filled by the library only when it reports the request
        st = fn(self._h, ticket, ctypes.byref(i))
        if st == HPM_ERR_NOT_READY:
            return None
        if i.status == -1:
            raise HpmError(st, fn.__name__)
        keep = self._live.pop(ticket, None)
        return _request_dict(i), (keep[4] if keep else None)

    def wait(self, ticket: int):
        """Blocks until the request has finished: (info, (phi, ax, ay, az)); info["status"] is
        the solve's status."""
        return self._call(_lib.hpm_server_wait, ticket)

    def poll(self, ticket: int):
        """None while the request is queued or running, else as wait()."""
        return self._call(_lib.hpm_server_poll, ticket)

    def run_batch(self, problems, particles, outs=None):
        """hpm_server_run_batch over lists of problems and (x, y, z, m) tuples; returns
        (statuses, outputs)."""
        k = len(problems)
        torch.cuda.current_stream().synchronize()
        if outs is None:
            outs = [tuple(torch.empty(int(p[0].numel()), dtype=pr.dtype, device=p[0].device)
                          for _ in range(4)) for pr, p in zip(problems, particles)]
        cprobs = (HpmProblem * k)(*[pr.c() for pr in problems])
        ns = (_i64 * k)(*[int(p[0].numel()) for p in particles])
        cols = []
        for j in range(4):
            cols.append((_vp * k)(*[_dev(p[j], pr.dtype, int(p[0].numel()), "xyzm"[j])
                                    for pr, p in zip(problems, particles)]))
        for j in range(4):
            cols.append((_vp * k)(*[_dev(o[j], pr.dtype, int(p[0].numel()), "output")
                                    for pr, p, o in zip(problems, particles, outs)]))
        st = (_i32 * k)()
        _lib.hpm_server_run_batch(self._h, k, cprobs, ns, *cols, st)
        return [STATUS.get(v, str(v)) for v in st], outs

    def stats(self) -> dict:
        s = HpmServerStats()
        _check(_lib.hpm_server_stats_get(self._h, ctypes.byref(s)), "hpm_server_stats_get")
        return {f: getattr(s, f) for f, _ in HpmServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hpm_server_destroy(self._h)
        self._h = None
        self._live = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        self.close()
