"""ctypes shim over the FP64 CPU oracle -- TEST INFRASTRUCTURE, NOT THE PRODUCT.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It loads ``libmtpt_oracle.so`` (built
from ``mtpt_oracle.c`` by ``build.py``) and shares nothing with the HIP path.

Every function takes and returns numpy arrays in original particle order:
positions ``[n][dim]`` float64, masses ``[S][n]`` float64.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_i64p = C.POINTER(C.c_int64)
_f64p = C.POINTER(C.c_double)
_u32p = C.POINTER(C.c_uint32)


def _load():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = _build.LIB
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build()
    lib = C.CDLL(path)
    lib.or_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    lib.or_philox4x32_10.restype = None
    lib.or_uniform52.argtypes = [C.c_uint32, C.c_uint32]
    lib.or_uniform52.restype = C.c_double
    lib.or_log.argtypes = [C.c_double]
    lib.or_log.restype = C.c_double
    lib.or_sincos_2pi.argtypes = [C.c_double, _f64p, _f64p]
    lib.or_sincos_2pi.restype = None
    lib.or_normal_pair.argtypes = [C.c_uint64, C.c_int64, C.c_uint32, C.c_uint32, _f64p]
    lib.or_normal_pair.restype = None
    lib.or_normals.argtypes = [C.c_uint64, C.c_int64, C.c_int, C.c_int64, _f64p]
    lib.or_normals.restype = None
    lib.or_rw_step.argtypes = [C.c_int, C.c_int64, _f64p, _f64p, C.c_double, _f64p, C.c_double,
                               C.c_uint64, C.c_int64, C.c_int, _f64p, _f64p]
    lib.or_rw_step.restype = None
    lib.or_neighbors.argtypes = [C.c_int, C.c_int64, _f64p, C.c_double, _f64p, C.c_int, _i64p, _i64p,
                                 C.c_int64]
    lib.or_neighbors.restype = C.c_int64
    lib.or_mt_weights.argtypes = [C.c_int, C.c_int64, _f64p, C.c_double, C.c_double, C.c_double,
                                  _f64p, _i64p, _i64p, _f64p, _f64p, _f64p]
    lib.or_mt_weights.restype = None
    lib.or_mt_step.argtypes = [C.c_int, C.c_int64, C.c_int, _f64p, _f64p, _f64p, C.c_double,
                               C.c_double, C.c_double, C.c_double, _f64p, C.c_int]
    lib.or_mt_step.restype = C.c_int64
    lib.or_react.argtypes = [C.c_int64, _f64p, C.c_double, C.c_double, C.c_double, C.c_double]
    lib.or_react.restype = None
    lib.or_total.argtypes = [C.c_int64, _f64p]
    lib.or_total.restype = C.c_double
    lib.or_run.argtypes = [C.c_int, C.c_int64, C.c_int, _f64p, _f64p, C.c_double, _f64p, C.c_double,
                           C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint64, C.c_int64,
                           C.c_int, _f64p, C.c_int, C.c_int64, _f64p, _f64p, _i64p, _f64p, C.c_int]
    lib.or_run.restype = C.c_int
    lib.or_pair_dist2.argtypes = [C.c_int, _f64p, _f64p, _f64p]
    lib.or_pair_dist2.restype = C.c_double
    lib.or_max_threads.argtypes = []
    lib.or_max_threads.restype = C.c_int
    lib.or_set_threads.argtypes = [C.c_int]
    lib.or_set_threads.restype = None
    _LIB = lib
    return lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- RNG -----
def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block: 4 counter words and 2 key words -> 4 words."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.or_philox4x32_10(_p(c, _u32p), _p(k, _u32p), _p(out, _u32p))
    return out


def uniform52(lo_word: int, hi_word: int) -> float:
    return _load().or_uniform52(lo_word, hi_word)


def log(u: float) -> float:
    return _load().or_log(u)


def sincos_2pi(u: float):
    s, c = C.c_double(), C.c_double()
    _load().or_sincos_2pi(u, C.byref(s), C.byref(c))
    return s.value, c.value


def normal_pair(seed: int, step: int, pid: int, call: int):
    z = np.zeros(2)
    _load().or_normal_pair(seed, step, pid, call, _p(z, _f64p))
    return z


def normals(seed: int, step: int, dim: int, n: int) -> np.ndarray:
    """Standard-normal jump components [n][dim] for pids 0..n-1 at one step."""
    xi = np.zeros((n, dim))
    _load().or_normals(seed, step, dim, n, _p(xi, _f64p))
    return xi


# ----------------------------------------------------- dispersion tensor --
def _tensor(tens):
    """None (isotropic) or a contiguous float64 [3][3] copy of a shape tensor
    given as 3x3, 9 values, or the 2x2 block of a 2-d one."""
    if tens is None:
        return None
    t = np.asarray(tens, dtype=np.float64)
    if t.size == 9:
        t = t.reshape(3, 3)
    elif t.size == 4:
        t3 = np.eye(3)
        t3[:2, :2] = t.reshape(2, 2)
        t = t3
    else:
        raise ValueError("tensor must be 2x2 or 3x3")
    if not np.any(t):
        return None
    return np.ascontiguousarray(t)


def _tp(t):
    return None if t is None else _p(t, _f64p)


def tensor_of(params):
    """The shape tensor T of a parameter set (D_RW = d_rw T, D_MT = d_mt T):
    ``disp`` (9 values, row-major; all zero = isotropic), None when isotropic."""
    g = params.get if isinstance(params, dict) else (lambda k, d=None: getattr(params, k, d))
    disp = g("disp", None)
    return _tensor(disp) if disp is not None else None


def pair_dist2(xi, xj, tens=None) -> float:
    """Squared distance of one pair in the cutoff's metric: Euclidean, or the
    Mahalanobis form dx^T T^-1 dx under shape tensor T."""
    xi = _f64(xi)
    xj = _f64(xj)
    t = _tensor(tens)
    v = _load().or_pair_dist2(xi.size, _tp(t), _p(xi, _f64p), _p(xj, _f64p))
    if v < 0:
        raise ValueError("tensor is not symmetric positive definite")
    return v


# ---------------------------------------------------------- random walk ---
def rw_step(x, lo, hi, d_rw, dt, seed, step, fp32=False, vel=None, tens=None) -> np.ndarray:
    """One random-walk step (drift vel*dt plus the jump, L xi with a shape
    tensor T = L L^T) with reflection; returns new positions [n][dim]."""
    x = _f64(x).copy()
    n, dim = x.shape
    lo3 = np.zeros(3); lo3[:dim] = lo
    hi3 = np.zeros(3); hi3[:dim] = hi
    v3 = np.zeros(3)
    if vel is not None:
        v3[:dim] = np.asarray(vel, dtype=np.float64)[:dim]
    t = _tensor(tens)
    _load().or_rw_step(dim, n, _p(lo3, _f64p), _p(hi3, _f64p), d_rw, _p(v3, _f64p), dt, seed, step,
                       1 if fp32 else 0, _tp(t), _p(x, _f64p))
    return x


# ---------------------------------------------------------- neighbours ----
def neighbors(x, psi: float, method: str = "kdtree", tens=None):
    """CSR of N(i) = {j : r2_ij <= psi*psi}, self included, rows ascending
    (r2 the Mahalanobis form under a shape tensor, when one is given).

    Returns (row_ptr[n+1] int64, col[nnz] int64)."""
    lib = _load()
    x = _f64(x)
    n, dim = x.shape
    meth = {"brute": 0, "kdtree": 1}[method]
    psi2 = psi * psi
    t = _tensor(tens)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    nnz = lib.or_neighbors(dim, n, _p(x, _f64p), psi2, _tp(t), meth, _p(row_ptr, _i64p), None, 0)
    if nnz < 0:
        raise MemoryError("oracle neighbour search")
    col = np.zeros(max(nnz, 1), dtype=np.int64)
    lib.or_neighbors(dim, n, _p(x, _f64p), psi2, _tp(t), meth, _p(row_ptr, _i64p), _p(col, _i64p), nnz)
    return row_ptr, col[:nnz]


def mt_weights(x, row_ptr, col, d_mt, dt, beta, tens=None):
    """Row sums s[n], kernel values K[nnz] and normalised weights W[nnz] per CSR entry."""
    lib = _load()
    x = _f64(x)
    n, dim = x.shape
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int64)
    s = np.zeros(n)
    kv = np.zeros(max(len(col), 1))
    wv = np.zeros(max(len(col), 1))
    t = _tensor(tens)
    lib.or_mt_weights(dim, n, _p(x, _f64p), d_mt, dt, beta, _tp(t), _p(row_ptr, _i64p), _p(col, _i64p),
                      _p(s, _f64p), _p(kv, _f64p), _p(wv, _f64p))
    return s, kv[:len(col)], wv[:len(col)]


def mt_step(x, m, d_mt, dt, beta, psi, method="kdtree", tens=None):
    """One mass-transfer step at fixed positions.  m is [S][n]; returns (m_new, pairs)."""
    lib = _load()
    x = _f64(x)
    m = _f64(np.atleast_2d(m))
    n, dim = x.shape
    S = m.shape[0]
    out = np.zeros_like(m)
    t = _tensor(tens)
    pairs = lib.or_mt_step(dim, n, S, _p(x, _f64p), _p(m, _f64p), _p(out, _f64p), d_mt, dt, beta,
                           psi, _tp(t), {"brute": 0, "kdtree": 1}[method])
    if pairs < 0:
        raise MemoryError("oracle mass transfer")
    return out, int(pairs)


def react(m, k_react, dt, volume) -> np.ndarray:
    """A+B->C reaction on masses [3][n]; returns the new masses."""
    m = _f64(m).copy()
    n = m.shape[1]
    _load().or_react(n, _p(m, _f64p), k_react, dt, float(n), volume)
    return m


def total(v) -> float:
    v = _f64(v)
    return _load().or_total(v.size, _p(v, _f64p))


def set_threads(n: int) -> None:
    _load().or_set_threads(int(n))


def max_threads() -> int:
    return int(_load().or_max_threads())


# ------------------------------------------------------------ the loop ----
@dataclass
class RunResult:
    x: np.ndarray          # [n][dim] positions after the last step
    m: np.ndarray          # [S][n] masses after the last step
    pairs: np.ndarray      # [steps] ordered pairs i != j within psi, per step
    totals: np.ndarray     # [steps][S] compensated mass totals after each step


def run(params, x0, m0, steps: int, method: str = "kdtree", threads: int = 0) -> RunResult:
    """Run ``steps`` MTPT steps from (x0, m0) with ``params`` (a mapping or
    object with dim, lo, hi, d_rw, vel (optional drift velocity), disp
    (optional shape tensor of the dispersion, 9 values row-major), d_mt, dt,
    beta, psi, k_react, seed, start_step, precision).  Everything runs in the
    caller's frame and box.  FP32 precisions keep FP32 position state: the
    inputs are rounded to float once here, as the library does at create."""
    g = params.get if isinstance(params, dict) else (lambda k, d=None: getattr(params, k, d))
    dim = int(g("dim"))
    x = _f64(x0).reshape(-1, dim).copy()
    n = x.shape[0]
    m = _f64(np.atleast_2d(m0)).copy()
    S = m.shape[0]
    t = tensor_of(params)
    fp32 = int(g("precision", 0)) != 0
    if fp32:
        x = x.astype(np.float32).astype(np.float64)
    lo3 = np.zeros(3); lo3[:dim] = np.asarray(g("lo")[:dim], dtype=np.float64)
    hi3 = np.zeros(3); hi3[:dim] = np.asarray(g("hi")[:dim], dtype=np.float64)
    psi = float(g("psi", 0.0) or 0.0)
    d_mt, dt = float(g("d_mt")), float(g("dt"))
    if psi <= 0.0:
        psi = 3.0 * math.sqrt(4.0 * d_mt * dt)
    v3 = np.zeros(3)
    vel = g("vel", None)
    if vel is not None:
        v3[:dim] = np.asarray(vel, dtype=np.float64)[:dim]
    pairs = np.zeros(steps, dtype=np.int64)
    totals = np.zeros((steps, S))
    rc = _load().or_run(dim, n, S, _p(lo3, _f64p), _p(hi3, _f64p), float(g("d_rw", 0.0)), _p(v3, _f64p),
                        d_mt, dt,
                        float(g("beta", 0.5)), psi, float(g("k_react", 0.0) or 0.0),
                        int(g("seed", 0)), int(g("start_step", 0)), 1 if fp32 else 0, _tp(t),
                        {"brute": 0, "kdtree": 1}[method], steps, _p(x, _f64p), _p(m, _f64p),
                        _p(pairs, _i64p), _p(totals, _f64p), int(threads))
    if rc != 0:
        raise MemoryError("oracle run (allocation, or a tensor that is not positive definite)")
    return RunResult(x=x, m=m, pairs=pairs, totals=totals)
