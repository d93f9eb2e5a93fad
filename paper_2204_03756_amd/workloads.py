"""Seeded synthetic inputs for the MTPT workloads.

This module only builds inputs: parameter sets, initial positions and initial
masses.  It holds none of the method's arithmetic, and both the HIP path's
tests and the CPU oracle draw their inputs from it.

The paper's workloads are uniformly scattered particles with a Heaviside
initial mass (Sec. 2.1, Sec. 2.2).  The five named workloads below follow that
recipe at the sizes the benchmark is quoted on:

* ``plain2d``   2-d, N=1e4 in [0,100]^2, pure mass transfer (no random walk),
                D_MT=1, dt=0.1, 50 steps, m=1 for x<50 else 0, FP64.
* ``rw2d``      2-d, N=4e6 in [0,2000]^2, D_RW=D_MT=0.5, dt=0.1, 100 steps,
                Gaussian mass blob (sigma 50) at the centre.
* ``rw3d``      3-d, N=2e6 in [0,126]^3, D_RW=D_MT=1, dt=0.1, 100 steps, mass
                1e-3 on the 1000 particles nearest the centre.
* ``serve``     a Poisson stream of independent 2-d/3-d sims (see requests()).
* ``react3d``   3-d, N=3.2e7 in [0,318]^3, D_RW=0.3, D_MT=0.7, dt=0.05, 200
                steps, species A=1 for x<159, B=1 for x>=159, C=0, A+B->C, k=1.

Every workload can be scaled down (``n=...``) at the same density, which keeps
the neighbour statistics of the full size; the parity tests use that.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

# precision codes (same values as the C-ABI's)
FP64 = 0
FP32W_FP64ACC = 1
FP32_KAHAN = 2
PRECISIONS = {"fp64": FP64, "fp32w": FP32W_FP64ACC, "kahan": FP32_KAHAN}


@dataclass
class Params:
    dim: int
    n: int
    lo: List[float]
    hi: List[float]
    d_rw: float
    d_mt: float
    dt: float
    beta: float = 0.5
    psi: float = 0.0          # <= 0: 3 * sqrt(4 * d_mt * dt)
    k_react: float = 0.0
    n_species: int = 1
    seed: int = 0             # random-walk key
    start_step: int = 0
    precision: int = FP64
    vel: List[float] = field(default_factory=lambda: [0.0, 0.0, 0.0])   # drift velocity
    # shape tensor T of the dispersion, row-major [3][3]: D_RW = d_rw T and
    # D_MT = d_mt T (all zero: isotropic, T = I)
    disp: List[float] = field(default_factory=lambda: [0.0] * 9)

    @property
    def psi_eff(self) -> float:
        return self.psi if self.psi > 0 else 3.0 * math.sqrt(4.0 * self.d_mt * self.dt)

    @property
    def volume(self) -> float:
        v = 1.0
        for k in range(self.dim):
            v *= self.hi[k] - self.lo[k]
        return v

    def as_dict(self) -> dict:
        return {
            "dim": self.dim, "n": self.n, "lo": list(self.lo), "hi": list(self.hi),
            "d_rw": self.d_rw, "d_mt": self.d_mt, "dt": self.dt, "beta": self.beta,
            "psi": self.psi, "k_react": self.k_react, "n_species": self.n_species,
            "seed": self.seed, "start_step": self.start_step, "precision": self.precision,
            "vel": list(self.vel), "disp": list(self.disp),
        }


@dataclass
class Workload:
    name: str
    params: Params
    x0: np.ndarray            # [n][dim] float64
    m0: np.ndarray            # [S][n] float64
    steps: int
    notes: dict = field(default_factory=dict)


def _uniform(rng_seed: int, n: int, dim: int, lo, hi) -> np.ndarray:
    rng = np.random.Generator(np.random.Philox(rng_seed))
    u = rng.random((n, dim))
    lo = np.asarray(lo[:dim], dtype=np.float64)
    hi = np.asarray(hi[:dim], dtype=np.float64)
    x = lo + u * (hi - lo)
    return np.minimum(np.maximum(x, lo), hi)


def plain2d(n: int = 10_000, steps: int = 50, precision: int = FP64) -> Workload:
    """2-d pure mass transfer, Heaviside m=1 for x < L/2 (density 1)."""
    L = 100.0 * math.sqrt(n / 10_000)
    p = Params(dim=2, n=n, lo=[0.0, 0.0, 0.0], hi=[L, L, 0.0], d_rw=0.0, d_mt=1.0, dt=0.1,
               beta=0.5, psi=0.0, seed=0x4D54505401, precision=precision)
    x = _uniform(20220401, n, 2, p.lo, p.hi)
    m = (x[:, 0] < L / 2).astype(np.float64)[None, :]
    return Workload("plain2d", p, x, m, steps, {"L": L})


def rw2d(n: int = 4_000_000, steps: int = 100, precision: int = FP32W_FP64ACC) -> Workload:
    """2-d random walk + mass transfer, Gaussian blob of sigma 50*(L/2000)."""
    L = 2000.0 * math.sqrt(n / 4_000_000)
    p = Params(dim=2, n=n, lo=[0.0, 0.0, 0.0], hi=[L, L, 0.0], d_rw=0.5, d_mt=0.5, dt=0.1,
               beta=0.5, psi=0.0, seed=0x4D54505402, precision=precision)
    x = _uniform(20220402, n, 2, p.lo, p.hi)
    sig = 50.0 * L / 2000.0
    c = L / 2
    r2 = (x[:, 0] - c) ** 2 + (x[:, 1] - c) ** 2
    m = np.exp(-r2 / (2.0 * sig * sig))[None, :]
    return Workload("rw2d", p, x, m, steps, {"L": L, "blob_sigma": sig})


def rw3d(n: int = 2_000_000, steps: int = 100, precision: int = FP32W_FP64ACC,
         n_src: Optional[int] = None) -> Workload:
    """3-d random walk + mass transfer, point-like source on the n_src particles
    nearest the centre (1000 at full size), 1e-3 each; ties broken by pid."""
    L = 126.0 * (n / 2_000_000) ** (1.0 / 3.0)
    p = Params(dim=3, n=n, lo=[0.0, 0.0, 0.0], hi=[L, L, L], d_rw=1.0, d_mt=1.0, dt=0.1,
               beta=0.5, psi=0.0, seed=0x4D54505403, precision=precision)
    x = _uniform(20220403, n, 3, p.lo, p.hi)
    if n_src is None:
        n_src = max(1, min(1000, n // 2000))
    c = L / 2
    d2 = ((x - c) ** 2).sum(axis=1)
    order = np.lexsort((np.arange(n), d2))[:n_src]
    m = np.zeros((1, n))
    m[0, order] = 1e-3
    return Workload("rw3d", p, x, m, steps, {"L": L, "n_src": n_src})


def react3d(n: int = 32_000_000, steps: int = 200, precision: int = FP32W_FP64ACC) -> Workload:
    """3-d random walk + mass transfer with A+B->C: A=1 for x<L/2, B=1 for x>=L/2."""
    L = 318.0 * (n / 32_000_000) ** (1.0 / 3.0)
    p = Params(dim=3, n=n, lo=[0.0, 0.0, 0.0], hi=[L, L, L], d_rw=0.3, d_mt=0.7, dt=0.05,
               beta=0.5, psi=0.0, k_react=1.0, n_species=3, seed=0x4D54505405,
               precision=precision)
    x = _uniform(20220405, n, 3, p.lo, p.hi)
    a = (x[:, 0] < L / 2).astype(np.float64)
    m = np.stack([a, 1.0 - a, np.zeros(n)])
    return Workload("react3d", p, x, m, steps, {"L": L})


def adv2d(n: int = 4_000_000, steps: int = 100, precision: int = FP32W_FP64ACC) -> Workload:
    """rw2d with a drift velocity v = (1, 0.5) (advection-dispersion): the
    Gaussian blob moves by v t while it spreads."""
    w = rw2d(n=n, steps=steps, precision=precision)
    p = replace(w.params, vel=[1.0, 0.5, 0.0], seed=0x4D54505406)
    return Workload("adv2d", p, w.x0, w.m0, steps, {**w.notes, "vel": [1.0, 0.5]})


def diag_tensor(a) -> List[float]:
    """Row-major [3][3] shape tensor diag(a) (unused diagonal entries 1)."""
    t = np.eye(3)
    for k, v in enumerate(a):
        t[k, k] = float(v)
    return t.reshape(-1).tolist()


def rotated_tensor(eigs, angles) -> List[float]:
    """Row-major [3][3] shape tensor R diag(eigs) R^T, R the rotation by the
    given angles (radians) about z, then y, then x; a 2-d tensor takes two
    eigenvalues and one angle (about z)."""
    e = list(eigs) + [1.0] * (3 - len(eigs))
    ang = list(angles) + [0.0] * (3 - len(angles))
    cz, sz = math.cos(ang[0]), math.sin(ang[0])
    cy, sy = math.cos(ang[1]), math.sin(ang[1])
    cx, sx = math.cos(ang[2]), math.sin(ang[2])
    rz = np.array([[cz, -sz, 0.0], [sz, cz, 0.0], [0.0, 0.0, 1.0]])
    ry = np.array([[cy, 0.0, sy], [0.0, 1.0, 0.0], [-sy, 0.0, cy]])
    rx = np.array([[1.0, 0.0, 0.0], [0.0, cx, -sx], [0.0, sx, cx]])
    r = rx @ ry @ rz
    t = r @ np.diag(e) @ r.T
    t = 0.5 * (t + t.T)            # exactly symmetric
    return t.reshape(-1).tolist()


def aniso2d(n: int = 4_000_000, steps: int = 100, precision: int = FP32W_FP64ACC) -> Workload:
    """rw2d with a rotated dispersion tensor (principal values 2 and 1/2, axes
    at 30 degrees; the walk and the mass transfer alike): the blob spreads
    into a tilted ellipse."""
    w = rw2d(n=n, steps=steps, precision=precision)
    p = replace(w.params, disp=rotated_tensor([2.0, 0.5], [math.pi / 6]), seed=0x4D54505407)
    return Workload("aniso2d", p, w.x0, w.m0, steps, {**w.notes, "disp_eigs": [2.0, 0.5], "angle_deg": 30})


WORKLOADS = {"plain2d": plain2d, "rw2d": rw2d, "rw3d": rw3d, "react3d": react3d, "adv2d": adv2d,
             "aniso2d": aniso2d}


def make(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)


def with_precision(w: Workload, precision: int) -> Workload:
    return replace(w, params=replace(w.params, precision=precision))


# ------------------------------------------------------------- serving ----
@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the stream starts
    params: Params
    x0: np.ndarray
    m0: np.ndarray
    steps: int


def request(rid: int, base_seed: int = 20220404, n_min: float = 1e4, n_max: float = 1e6,
            precision: int = FP32_KAHAN) -> Request:
    """One independent sim of the serving mix: d in {2,3} equiprobable,
    N = floor(10^U(log10 n_min, log10 n_max)), L = N^(1/d) (density 1),
    D in {0.5, 1, 2} with D_RW = D_MT = D/2, steps U{20..200}, dt = 0.1,
    Heaviside m = 1 for x < L/2.  Arrival time is filled by requests()."""
    rng = np.random.Generator(np.random.Philox(base_seed * 10_000 + rid))
    dim = int(rng.integers(2, 4))
    n = int(math.floor(10 ** rng.uniform(math.log10(n_min), math.log10(n_max))))
    D = float(rng.choice([0.5, 1.0, 2.0]))
    steps = int(rng.integers(20, 201))
    L = n ** (1.0 / dim)
    hi = [L] * dim + [0.0] * (3 - dim)
    p = Params(dim=dim, n=n, lo=[0.0, 0.0, 0.0], hi=hi, d_rw=D / 2, d_mt=D / 2, dt=0.1,
               beta=0.5, psi=0.0, seed=0x4D545054040000 + rid, precision=precision)
    u = rng.random((n, dim))
    x = np.minimum(u * L, L)
    m = (x[:, 0] < L / 2).astype(np.float64)[None, :]
    return Request(rid, 0.0, p, x, m, steps)


def arrivals(n_req: int, rate: float, seed: int = 20220404) -> np.ndarray:
    """Poisson arrival times (exponential gaps with the given rate per second)."""
    rng = np.random.Generator(np.random.Philox(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n_req))
