"""Python binding of libcgks (the HIP implementation behind include/cgks.h).

Argument marshalling only: every step of the scheme runs in the library's
HIP kernels.  PyTorch supplies device memory (state tensors on the GPU) and
the stream the library queues its work on.  There is no fallback: without
the built library or without a GPU every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import build as _build

CGKS_OK, CGKS_EINVAL, CGKS_ENOMEM, CGKS_EDEVICE, CGKS_ENONPHYS, CGKS_EBUSY, CGKS_ESTATE = 0, -1, -2, -3, -4, -5, -6
PERIODIC, FREE, WALL, INFLOW, NOSLIP = 0, 1, 2, 3, 4
CGKS_FP64, CGKS_FP32_STORAGE = 0, 1


class cgks_config(C.Structure):
    _fields_ = [('dim', C.c_int), ('nx', C.c_int), ('ny', C.c_int),
                ('x0', C.c_double), ('x1', C.c_double), ('y0', C.c_double), ('y1', C.c_double),
                ('gamma', C.c_double), ('cfl', C.c_double),
                ('bc', C.c_int * 4), ('inflow_prim', (C.c_double * 4) * 4),
                ('weno_eps', C.c_double), ('tau_eps', C.c_double), ('tau_C', C.c_double),
                ('fixed_dt', C.c_double), ('storage', C.c_int), ('mu', C.c_double), ('gauss_points', C.c_int),
                ('recon_vars', C.c_int), ('side_slopes', C.c_int), ('tang_weno', C.c_int)]


class cgks_counters_t(C.Structure):
    _fields_ = [('steps', C.c_long), ('guard_w0', C.c_long), ('guard_weno', C.c_long),
                ('last_dt', C.c_double), ('t', C.c_double)]


class CgksError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        msg = _lib.cgks_strerror(code).decode() if _lib is not None else str(code)
        super().__init__('%s: %s (code %d)' % (what, msg, code))


_lib = None
_D = C.POINTER(C.c_double)


def library_path() -> str:
    """The in-tree library; CGKS_LIBRARY may name a tuning variant built from the same sources."""
    return os.environ.get('CGKS_LIBRARY') or _build.LIB


def load():
    """Load libcgks.so (building it first only if it does not exist)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        if path != _build.LIB:
            raise FileNotFoundError(path)
        _build.build()
    L = C.CDLL(path)
    L.cgks_create.argtypes = [C.POINTER(cgks_config), C.c_void_p, C.POINTER(C.c_void_p)]
    L.cgks_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_double]
    L.cgks_step.argtypes = [C.c_void_p, _D]
    L.cgks_step_dt.argtypes = [C.c_void_p, C.c_double, _D]
    L.cgks_advance_to.argtypes = [C.c_void_p, C.c_double, C.c_long, C.POINTER(C.c_long)]
    L.cgks_run_steps.argtypes = [C.c_void_p, C.c_long]
    L.cgks_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_int, _D, C.POINTER(C.c_long)]
    L.cgks_last_bad_cell.argtypes = [C.c_void_p, C.POINTER(C.c_long)]
    L.cgks_counters.argtypes = [C.c_void_p, C.POINTER(cgks_counters_t)]
    L.cgks_destroy.argtypes = [C.c_void_p]
    L.cgks_destroy.restype = None
    L.cgks_strerror.argtypes = [C.c_int]
    L.cgks_strerror.restype = C.c_char_p
    L.cgks_set_profiling.argtypes = [C.c_void_p, C.c_int]
    L.cgks_kernel_times.argtypes = [C.c_void_p, _D, C.POINTER(C.c_long), C.c_int]
    L.cgks_kernel_times.restype = C.c_int
    L.cgks_set_tiles.argtypes = [C.c_void_p, C.c_int, C.c_int]
    L.cgks_batch_create.argtypes = [C.c_size_t, C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]
    L.cgks_batch_admit.argtypes = [C.c_void_p, C.POINTER(cgks_config), C.c_void_p, C.c_int, C.c_double, C.c_long,
                                   C.POINTER(C.c_int)]
    L.cgks_batch_run.argtypes = [C.c_void_p, C.c_int]
    L.cgks_batch_poll.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), _D, C.POINTER(C.c_long)]
    L.cgks_batch_read.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int]
    L.cgks_batch_release.argtypes = [C.c_void_p, C.c_int]
    L.cgks_batch_set_tiles.argtypes = [C.c_void_p, C.c_int, C.c_int]
    L.cgks_batch_tuning.argtypes = [C.POINTER(C.c_int)] * 3
    L.cgks_batch_destroy.argtypes = [C.c_void_p]
    L.cgks_batch_destroy.restype = None
    L.cgks_step_noalloc.argtypes = [C.POINTER(cgks_config), C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, _D]
    _lib = L
    return L


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError('the HIP path needs a GPU (torch.cuda.is_available() is False)')
    return torch


def make_config(prob, storage: int = CGKS_FP64) -> cgks_config:
    d = prob.config_dict()
    cfg = cgks_config()
    for k in ('dim', 'nx', 'ny'):
        setattr(cfg, k, int(d[k]))
    for k in ('x0', 'x1', 'y0', 'y1', 'gamma', 'cfl', 'weno_eps', 'tau_eps', 'tau_C', 'fixed_dt', 'mu'):
        setattr(cfg, k, float(d[k]))
    for s in range(4):
        cfg.bc[s] = int(d['bc'][s])
        for q in range(4):
            cfg.inflow_prim[s][q] = float(d['inflow_prim'][s][q])
    cfg.storage = int(storage)
    cfg.gauss_points = int(d.get('gauss_points', 2))
    cfg.recon_vars = int(d.get('recon_vars', 0))
    cfg.side_slopes = int(d.get('side_slopes', 0))
    cfg.tang_weno = int(d.get('tang_weno', 0))
    return cfg


KERNEL_NAMES_2D = ['xfaces1', 'yfaces1', 'update1', 'xfaces2', 'yfaces2', 'update2']
KERNEL_NAMES_1D = ['faces1', 'update1', 'faces2', 'update2']


class Solver:
    """One simulation on the GPU (see paper_2001_01570_amd.inputs.Problem)."""

    def __init__(self, prob, stream=None, load_state: bool = True, storage: int = CGKS_FP64):
        torch = _torch()
        L = load()
        self.prob = prob
        self.dim = prob.dim
        self.shape = (6, prob.nx) if prob.dim == 1 else (12, prob.ny, prob.nx)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        rc = L.cgks_create(C.byref(make_config(prob, storage)), C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc:
            raise CgksError(rc, 'cgks_create')
        self.h = h
        if load_state:
            self.set_state(prob.fields, 0.0)

    def close(self):
        if getattr(self, 'h', None):
            load().cgks_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc:
            raise CgksError(rc, what)

    def set_state(self, fields, t0: float = 0.0):
        torch = _torch()
        if isinstance(fields, torch.Tensor) and fields.is_cuda:
            assert tuple(fields.shape) == self.shape and fields.dtype == torch.float64
            f = fields.contiguous()
            self._check(load().cgks_set_state(self.h, C.c_void_p(f.data_ptr()), 1, float(t0)), 'cgks_set_state')
        else:
            a = np.ascontiguousarray(np.asarray(fields, dtype=np.float64))
            assert a.shape == self.shape, (a.shape, self.shape)
            self._check(load().cgks_set_state(self.h, C.c_void_p(a.ctypes.data), 0, float(t0)), 'cgks_set_state')

    def step(self, dt: float = 0.0) -> float:
        used = C.c_double()
        self._check(load().cgks_step_dt(self.h, float(dt), C.byref(used)), 'cgks_step')
        return used.value

    def set_tiles(self, x_shape: int, y_shape: int):
        """Face tile shape per direction (see cgks_set_tiles); speed only."""
        self._check(load().cgks_set_tiles(self.h, int(x_shape), int(y_shape)), 'cgks_set_tiles')

    def run_steps(self, n: int):
        self._check(load().cgks_run_steps(self.h, int(n)), 'cgks_run_steps')

    def advance_to(self, t_end: float, max_steps: int = 0) -> int:
        n = C.c_long()
        self._check(load().cgks_advance_to(self.h, float(t_end), int(max_steps), C.byref(n)), 'cgks_advance_to')
        return n.value

    def get_state(self, device: bool = False):
        t = C.c_double()
        s = C.c_long()
        if device:
            torch = _torch()
            out = torch.empty(self.shape, dtype=torch.float64, device='cuda')
            self._check(load().cgks_get_state(self.h, C.c_void_p(out.data_ptr()), 1, C.byref(t), C.byref(s)),
                        'cgks_get_state')
        else:
            out = np.empty(self.shape)
            self._check(load().cgks_get_state(self.h, C.c_void_p(out.ctypes.data), 0, C.byref(t), C.byref(s)),
                        'cgks_get_state')
        return out, t.value, s.value

    @property
    def state(self):
        return self.get_state()[0]

    @property
    def t(self):
        return self.get_state()[1]

    def counters(self) -> dict:
        c = cgks_counters_t()
        self._check(load().cgks_counters(self.h, C.byref(c)), 'cgks_counters')
        return dict(steps=c.steps, guard_w0=c.guard_w0, guard_weno=c.guard_weno, last_dt=c.last_dt, t=c.t)

    def last_bad_cell(self) -> int:
        c = C.c_long()
        load().cgks_last_bad_cell(self.h, C.byref(c))
        return c.value

    def set_profiling(self, on=True, kinds=None):
        """Profile every kernel kind (on=True), none (False), or only the named kinds."""
        if not on:
            mask = 0
        elif kinds is None:
            mask = -1
        else:
            names = KERNEL_NAMES_2D if self.dim == 2 else KERNEL_NAMES_1D
            mask = sum(1 << names.index(k) for k in kinds)
        self._check(load().cgks_set_profiling(self.h, mask), 'cgks_set_profiling')

    def kernel_times(self) -> dict:
        """Per-kernel accumulated device time (ms) and launch counts recorded with
        HIP events on the solver's stream while profiling was on."""
        n = 8
        ms = (C.c_double * n)()
        calls = (C.c_long * n)()
        k = load().cgks_kernel_times(self.h, ms, calls, n)
        if k < 0:
            raise CgksError(k, 'cgks_kernel_times')
        names = KERNEL_NAMES_2D if self.dim == 2 else KERNEL_NAMES_1D
        return {names[i]: (ms[i], calls[i]) for i in range(min(k, len(names)))}


NOALLOC_MAX_CELLS = 65536


def step_noalloc(prob, fields_in, fields_out, dt: float = 0.0, stream=None, wait: bool = True):
    """One step with cgks_step_noalloc (no device allocation): fields_in and
    fields_out are distinct contiguous float64 CUDA tensors of the state
    shape.  wait=True: waits and returns the step size (raises on a
    non-physical result); wait=False: only queues the work, returns None."""
    torch = _torch()
    shape = (6, prob.nx) if prob.dim == 1 else (12, prob.ny, prob.nx)
    for f in (fields_in, fields_out):
        assert isinstance(f, torch.Tensor) and f.is_cuda and f.dtype == torch.float64
        assert tuple(f.shape) == shape and f.is_contiguous()
    if stream is None:
        stream = torch.cuda.current_stream()
    used = C.c_double()
    rc = load().cgks_step_noalloc(C.byref(make_config(prob)), C.c_void_p(fields_in.data_ptr()),
                                  C.c_void_p(fields_out.data_ptr()), float(dt), C.c_void_p(stream.cuda_stream),
                                  C.byref(used) if wait else None)
    if rc:
        raise CgksError(rc, 'cgks_step_noalloc')
    return used.value if wait else None


SLOT_FREE, SLOT_RUNNING, SLOT_DONE, SLOT_FAILED = 0, 1, 2, 3


def batch_tuning():
    """The library's tuned batch entry: (x tile shape, y tile shape, steps per run)."""
    x, y, n = C.c_int(), C.c_int(), C.c_int()
    load().cgks_batch_tuning(C.byref(x), C.byref(y), C.byref(n))
    return x.value, y.value, n.value


class Batch:
    """Many independent 2D problems advanced together (see cgks_batch_* in
    include/cgks.h).  Slots are admitted with a configuration (a Problem) and
    an initial state and run until their end time or step bound."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 256, stream=None):
        _torch()
        L = load()
        h = C.c_void_p()
        ptr = None if stream is None else C.c_void_p(stream.cuda_stream)
        rc = L.cgks_batch_create(int(hbm_budget_bytes), int(max_slots), ptr, C.byref(h))
        if rc:
            raise CgksError(rc, 'cgks_batch_create')
        self.h = h
        self.shapes = {}

    def close(self):
        if getattr(self, 'h', None):
            load().cgks_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, prob, fields=None, t_end: float = 0.0, max_steps: int = 0) -> int:
        """Returns the slot; raises CgksError (code CGKS_EBUSY when full)."""
        return self.admit_storage(prob, CGKS_FP64, fields, t_end, max_steps)

    def admit_storage(self, prob, storage: int, fields=None, t_end: float = 0.0, max_steps: int = 0) -> int:
        """admit with the gradient storage given (CGKS_FP64 or CGKS_FP32_STORAGE)."""
        torch = _torch()
        fields = prob.fields if fields is None else fields
        shape = (12, prob.ny, prob.nx) if prob.dim == 2 else (6, prob.nx)   # the library rejects dim 1
        slot = C.c_int()
        cfg = make_config(prob, storage)
        if isinstance(fields, torch.Tensor) and fields.is_cuda:
            assert tuple(fields.shape) == shape and fields.dtype == torch.float64
            f = fields.contiguous()
            rc = load().cgks_batch_admit(self.h, C.byref(cfg), C.c_void_p(f.data_ptr()), 1, float(t_end),
                                         int(max_steps), C.byref(slot))
        else:
            a = np.ascontiguousarray(np.asarray(fields, dtype=np.float64))
            assert a.shape == shape, (a.shape, shape)
            rc = load().cgks_batch_admit(self.h, C.byref(cfg), C.c_void_p(a.ctypes.data), 0, float(t_end),
                                         int(max_steps), C.byref(slot))
        if rc:
            raise CgksError(rc, 'cgks_batch_admit')
        self.shapes[slot.value] = shape
        return slot.value

    def run(self, steps: int):
        rc = load().cgks_batch_run(self.h, int(steps))
        if rc:
            raise CgksError(rc, 'cgks_batch_run')

    def poll(self, slot: int):
        st, t, n = C.c_int(), C.c_double(), C.c_long()
        rc = load().cgks_batch_poll(self.h, int(slot), C.byref(st), C.byref(t), C.byref(n))
        if rc:
            raise CgksError(rc, 'cgks_batch_poll')
        return st.value, t.value, n.value

    def read(self, slot: int, device: bool = False):
        shape = self.shapes[slot]
        if device:
            torch = _torch()
            out = torch.empty(shape, dtype=torch.float64, device='cuda')
            rc = load().cgks_batch_read(self.h, int(slot), C.c_void_p(out.data_ptr()), 1)
        else:
            out = np.empty(shape)
            rc = load().cgks_batch_read(self.h, int(slot), C.c_void_p(out.ctypes.data), 0)
        if rc:
            raise CgksError(rc, 'cgks_batch_read')
        return out

    def set_tiles(self, x_shape: int, y_shape: int):
        """Face tile shapes of the two-point FP64 slots (before any admit); speed only."""
        rc = load().cgks_batch_set_tiles(self.h, int(x_shape), int(y_shape))
        if rc:
            raise CgksError(rc, 'cgks_batch_set_tiles')

    def release(self, slot: int):
        rc = load().cgks_batch_release(self.h, int(slot))
        if rc:
            raise CgksError(rc, 'cgks_batch_release')
        self.shapes.pop(slot, None)
