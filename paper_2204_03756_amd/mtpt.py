"""Python binding of libmtpt.so (argument marshalling only).

Every function named ``mtpt_*`` here calls the C entry point of the same name
declared in ``include/mtpt.h``; all arithmetic of the step runs in the HIP
kernels of the library.  PyTorch is used only as a device-memory provider
(``TorchAllocator`` routes the library's allocations through torch's caching
allocator) and for the stream handle.  There is no fallback: if the library
is missing or cannot be loaded, the functions raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import build as _build

MTPT_ABI_VERSION = 4
MTPT_OK, MTPT_E_ARG, MTPT_E_NOMEM, MTPT_E_DEVICE, MTPT_E_NONFINITE, MTPT_E_ABI, MTPT_E_STATE = \
    0, -1, -2, -3, -4, -5, -6
MTPT_FP64, MTPT_FP32W_FP64ACC, MTPT_FP32_KAHAN = 0, 1, 2


class MtptError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mtpt error {code}: {msg}")
        self.code = code


class mtpt_params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("dim", C.c_int32), ("n", C.c_int64),
        ("n_species", C.c_int32), ("precision", C.c_int32),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("d_rw", C.c_double), ("d_mt", C.c_double), ("dt", C.c_double), ("beta", C.c_double),
        ("psi", C.c_double), ("k_react", C.c_double),
        ("seed", C.c_uint64), ("start_step", C.c_int64),
        ("vel", C.c_double * 3), ("disp", C.c_double * 9),
    ]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class mtpt_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class mtpt_stats_t(C.Structure):
    _fields_ = [
        ("steps_done", C.c_int64), ("pairs_last", C.c_int64), ("pairs_total", C.c_uint64),
        ("mass_total", C.c_double * 3), ("mass_initial", C.c_double * 3), ("drift", C.c_double),
        ("nonfinite", C.c_int32), ("n_cells", C.c_int32),
    ]


_LIB = None
_f64p = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)


def lib_path() -> str:
    """libmtpt.so next to this package, or the file named by MTPT_LIB."""
    return os.environ.get("MTPT_LIB") or _build.LIB


def load():
    """Load libmtpt.so (built by build()); raises if it is absent."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise ImportError(f"libmtpt.so not found at {path}: run __graft_entry__.build() "
                          "(or python paper_2204_03756_amd/build.py) first")
    lib = C.CDLL(path)
    P = C.POINTER
    sig = {
        "mtpt_create": (C.c_int, [P(mtpt_params), _f64p, _f64p, C.c_void_p, P(mtpt_allocator),
                                  P(C.c_void_p)]),
        "mtpt_step": (C.c_int, [C.c_void_p, C.c_int64]),
        "mtpt_masses": (C.c_int, [C.c_void_p, _f64p]),
        "mtpt_positions": (C.c_int, [C.c_void_p, _f64p]),
        "mtpt_stats": (C.c_int, [C.c_void_p, P(mtpt_stats_t)]),
        "mtpt_neighbors": (C.c_int, [C.c_void_p, _i64p, _i64p, C.c_int64, _i64p]),
        "mtpt_step_neighbors": (C.c_int, [C.c_void_p, C.c_int32, _i64p, _i64p, C.c_int64, _i64p]),
        "mtpt_neighbors_static": (C.c_int, [C.c_void_p, _i64p, _i64p, C.c_int64, _i64p]),
        "mtpt_destroy": (C.c_int, [C.c_void_p]),
        "mtpt_last_error": (C.c_char_p, []),
        "mtpt_abi_version": (C.c_int, []),
        "mtpt_set_profiling": (C.c_int, [C.c_void_p, C.c_int32]),
        "mtpt_phase_times": (C.c_int, [C.c_void_p, P(C.c_char_p), _f64p, _i64p, C.c_int32,
                                       P(C.c_int32)]),
        "mtpt_pool_create": (C.c_int, [C.c_size_t, C.c_int32, C.c_void_p, P(mtpt_allocator),
                                       P(C.c_void_p)]),
        "mtpt_pool_admit": (C.c_int, [C.c_void_p, P(mtpt_params), _f64p, _f64p, C.c_int64, _i64p]),
        "mtpt_pool_tick": (C.c_int, [C.c_void_p, P(C.c_int32)]),
        "mtpt_pool_done": (C.c_int, [C.c_void_p, C.c_int64, P(C.c_int32)]),
        "mtpt_pool_result": (C.c_int, [C.c_void_p, C.c_int64, _f64p]),
        "mtpt_pool_stats": (C.c_int, [C.c_void_p, C.c_int64, P(mtpt_stats_t)]),
        "mtpt_pool_usage": (C.c_int, [C.c_void_p, P(C.c_int32), P(C.c_size_t), P(C.c_size_t)]),
        "mtpt_sim_bytes": (C.c_int, [P(mtpt_params), P(C.c_size_t)]),
        "mtpt_pool_destroy": (C.c_int, [C.c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.mtpt_abi_version() != MTPT_ABI_VERSION:
        raise ImportError("libmtpt.so ABI version mismatch")
    _LIB = lib
    return lib


def _check(rc: int):
    if rc != MTPT_OK:
        raise MtptError(rc, load().mtpt_last_error().decode())


def make_params(p) -> mtpt_params:
    """mtpt_params from a workloads.Params (or any object with the same fields)."""
    q = mtpt_params()
    q.abi_version = MTPT_ABI_VERSION
    q.dim = int(p.dim)
    q.n = int(p.n)
    q.n_species = int(getattr(p, "n_species", 1))
    q.precision = int(getattr(p, "precision", 0))
    for k in range(3):
        q.lo[k] = float(p.lo[k]) if k < len(p.lo) else 0.0
        q.hi[k] = float(p.hi[k]) if k < len(p.hi) else 0.0
    q.d_rw = float(p.d_rw)
    q.d_mt = float(p.d_mt)
    q.dt = float(p.dt)
    q.beta = float(getattr(p, "beta", 0.5))
    q.psi = float(getattr(p, "psi", 0.0))
    q.k_react = float(getattr(p, "k_react", 0.0))
    q.seed = int(getattr(p, "seed", 0))
    q.start_step = int(getattr(p, "start_step", 0))
    vel = getattr(p, "vel", None) or (0.0, 0.0, 0.0)
    for k in range(3):
        q.vel[k] = float(vel[k]) if k < len(vel) else 0.0
    disp = getattr(p, "disp", None) or [0.0] * 9
    disp = [float(v) for v in np.asarray(disp, dtype=np.float64).reshape(-1)]
    if len(disp) == 4:                       # a 2-d tensor: embed in 3x3
        disp = [disp[0], disp[1], 0.0, disp[2], disp[3], 0.0, 0.0, 0.0, 1.0]
    if len(disp) != 9:
        raise ValueError("disp must hold 9 (or 4) values")
    for k in range(9):
        q.disp[k] = disp[k]
    return q


class TorchAllocator:
    """Routes the library's device allocations through torch's caching allocator."""

    def __init__(self, device: Optional[str] = None):
        import torch
        self._torch = torch
        self.device = torch.device(device or "cuda")
        self._blocks = {}
        self._alloc_cb = ALLOC_FN(self._alloc)
        self._free_cb = FREE_FN(self._free)
        self.struct = mtpt_allocator(self._alloc_cb, self._free_cb, None)

    def _alloc(self, nbytes, _ctx):
        try:
            t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=self.device)
        except RuntimeError:
            return None
        p = t.data_ptr()
        self._blocks[p] = t
        return p

    def _free(self, ptr, _ctx):
        self._blocks.pop(ptr, None)

    @property
    def held_bytes(self) -> int:
        return sum(t.numel() for t in self._blocks.values())


def current_stream_handle() -> int:
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------ C entry points
def mtpt_create(params, pos, mass, hip_stream=None, allocator: Optional[TorchAllocator] = None):
    lib = load()
    q = params if isinstance(params, mtpt_params) else make_params(params)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    h = C.c_void_p()
    rc = lib.mtpt_create(C.byref(q), pos.ctypes.data_as(_f64p), mass.ctypes.data_as(_f64p),
                         C.c_void_p(hip_stream) if hip_stream else None,
                         C.byref(allocator.struct) if allocator is not None else None, C.byref(h))
    _check(rc)
    return h


def mtpt_step(sim, n_steps: int):
    _check(load().mtpt_step(sim, int(n_steps)))


def mtpt_masses(sim, n: int, n_species: int) -> np.ndarray:
    out = np.empty((n_species, n), dtype=np.float64)
    _check(load().mtpt_masses(sim, out.ctypes.data_as(_f64p)))
    return out


def mtpt_positions(sim, n: int, dim: int) -> np.ndarray:
    out = np.empty((n, dim), dtype=np.float64)
    _check(load().mtpt_positions(sim, out.ctypes.data_as(_f64p)))
    return out


def _stats_dict(st) -> dict:
    return {
        "steps_done": st.steps_done, "pairs_last": st.pairs_last, "pairs_total": st.pairs_total,
        "mass_total": list(st.mass_total), "mass_initial": list(st.mass_initial),
        "drift": st.drift, "nonfinite": st.nonfinite, "n_cells": st.n_cells,
    }


def mtpt_stats(sim) -> dict:
    st = mtpt_stats_t()
    _check(load().mtpt_stats(sim, C.byref(st)))
    return _stats_dict(st)


def mtpt_pool_stats(pool, ticket: int) -> dict:
    st = mtpt_stats_t()
    _check(load().mtpt_pool_stats(pool, int(ticket), C.byref(st)))
    return _stats_dict(st)


def mtpt_neighbors(sim, n: int):
    lib = load()
    row = np.zeros(n + 1, dtype=np.int64)
    nnz = C.c_int64()
    _check(lib.mtpt_neighbors(sim, row.ctypes.data_as(_i64p), None, 0, C.byref(nnz)))
    col = np.zeros(max(nnz.value, 1), dtype=np.int64)
    _check(lib.mtpt_neighbors(sim, row.ctypes.data_as(_i64p), col.ctypes.data_as(_i64p),
                              nnz.value, C.byref(nnz)))
    return row, col[:nnz.value]


def mtpt_step_neighbors(sim, n: int, which: int):
    """Pairs the row-sum (which=0) or transfer (which=1) pass of the last step
    used, as CSR in pid order (self included)."""
    lib = load()
    row = np.zeros(n + 1, dtype=np.int64)
    nnz = C.c_int64()
    _check(lib.mtpt_step_neighbors(sim, int(which), row.ctypes.data_as(_i64p), None, 0, C.byref(nnz)))
    col = np.zeros(max(nnz.value, 1), dtype=np.int64)
    _check(lib.mtpt_step_neighbors(sim, int(which), row.ctypes.data_as(_i64p), col.ctypes.data_as(_i64p),
                                   nnz.value, C.byref(nnz)))
    return row, col[:nnz.value]


def mtpt_destroy(sim):
    _check(load().mtpt_destroy(sim))


def mtpt_set_profiling(sim, on: bool):
    _check(load().mtpt_set_profiling(sim, 1 if on else 0))


def mtpt_phase_times(sim) -> dict:
    lib = load()
    cap = 16
    names = (C.c_char_p * cap)()
    ms = np.zeros(cap)
    nl = np.zeros(cap, dtype=np.int64)
    cnt = C.c_int32()
    _check(lib.mtpt_phase_times(sim, names, ms.ctypes.data_as(_f64p), nl.ctypes.data_as(_i64p), cap,
                                C.byref(cnt)))
    return {names[k].decode(): (float(ms[k]), int(nl[k])) for k in range(cnt.value)}


def mtpt_sim_bytes(params) -> int:
    q = params if isinstance(params, mtpt_params) else make_params(params)
    b = C.c_size_t()
    _check(load().mtpt_sim_bytes(C.byref(q), C.byref(b)))
    return int(b.value)


def mtpt_pool_create(hbm_budget: int, max_slots: int, hip_stream=None,
                     allocator: Optional[TorchAllocator] = None):
    h = C.c_void_p()
    _check(load().mtpt_pool_create(int(hbm_budget), int(max_slots),
                                   C.c_void_p(hip_stream) if hip_stream else None,
                                   C.byref(allocator.struct) if allocator is not None else None,
                                   C.byref(h)))
    return h


def mtpt_pool_admit(pool, params, pos, mass, n_steps: int):
    """Returns the ticket, or None when the pool is full (MTPT_E_NOMEM)."""
    q = params if isinstance(params, mtpt_params) else make_params(params)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    t = C.c_int64()
    rc = load().mtpt_pool_admit(pool, C.byref(q), pos.ctypes.data_as(_f64p),
                                mass.ctypes.data_as(_f64p), int(n_steps), C.byref(t))
    if rc == MTPT_E_NOMEM:
        return None
    _check(rc)
    return int(t.value)


def mtpt_pool_tick(pool) -> int:
    c = C.c_int32()
    _check(load().mtpt_pool_tick(pool, C.byref(c)))
    return int(c.value)


def mtpt_pool_done(pool, ticket: int) -> bool:
    d = C.c_int32()
    _check(load().mtpt_pool_done(pool, int(ticket), C.byref(d)))
    return bool(d.value)


def mtpt_pool_result(pool, ticket: int, n: int, n_species: int) -> np.ndarray:
    out = np.empty((n_species, n), dtype=np.float64)
    _check(load().mtpt_pool_result(pool, int(ticket), out.ctypes.data_as(_f64p)))
    return out


def mtpt_pool_usage(pool):
    a, h, b = C.c_int32(), C.c_size_t(), C.c_size_t()
    _check(load().mtpt_pool_usage(pool, C.byref(a), C.byref(h), C.byref(b)))
    return int(a.value), int(h.value), int(b.value)


def mtpt_pool_destroy(pool):
    _check(load().mtpt_pool_destroy(pool))


# ------------------------------------------------------------ convenience
class Sim:
    """One simulation on the current torch stream (RAII around the C handle)."""

    def __init__(self, params, x0, m0, allocator: Optional[TorchAllocator] = None,
                 stream: Optional[int] = None):
        self.params = params
        self.n = int(params.n)
        self.dim = int(params.dim)
        self.ns = int(getattr(params, "n_species", 1))
        if stream is None:
            stream = current_stream_handle()
        self.allocator = allocator
        self.h = mtpt_create(params, np.asarray(x0).reshape(self.n, self.dim),
                             np.asarray(m0).reshape(self.ns, self.n), stream, allocator)

    def step(self, n_steps: int = 1):
        mtpt_step(self.h, n_steps)

    def masses(self) -> np.ndarray:
        return mtpt_masses(self.h, self.n, self.ns)

    def positions(self) -> np.ndarray:
        return mtpt_positions(self.h, self.n, self.dim)

    def stats(self) -> dict:
        return mtpt_stats(self.h)

    def neighbors(self):
        return mtpt_neighbors(self.h, self.n)

    def step_neighbors(self, which: int):
        """The pairs the last step's row-sum (0) or transfer (1) pass used."""
        return mtpt_step_neighbors(self.h, self.n, which)

    def close(self):
        if self.h:
            mtpt_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
