"""Planner utilities: the paper's host-side closed forms for choosing a time
step and the number of processors (here: GPUs) of a spatial decomposition.
Nothing here runs on a device, and the simulation never calls it.

* ``dt_min`` -- the time-step optimality condition of Sec. 2.2: the mean
  particle spacing L / N^(1/d) must be resolved by the mass-transfer kernel,
  dt >= beta (L / N^(1/d))^2 / (2 D).
* ``speedup`` / ``efficiency`` -- Sec. 7, Eq. (10) and Eq. (11): with
  square/cubic subdomains and a run time linear in the particles a processor
  holds, N_S of Eq. (8) (its subdomain plus a pad of width ``halo`` on every
  side), S_P = 1 / (P^(-1/d) + 2 halo / L)^d and E_P = S_P / P.
* ``max_processors`` -- Sec. 7, Eq. (12): the most processors that keep
  E_P >= E, P <= (1/E) ((1 - E^(1/d)) L / (2 halo))^d.
* ``slices_limit`` -- Sec. 7: slices of width L / P stop holding their whole
  pad once they are thinner than it, at P = L / halo.
* ``checkerboard_factors`` -- Sec. 4.2, Eq. (7): the factor pair of P whose
  ratio is closest to the domain's aspect ratio, the larger factor along
  the longer side.
* ``tiling_speedup`` -- Eq. (8) and Eq. (10) for a rectangular (or prism)
  tiling: N_S is the subdomain grown by the pad in every direction, so a
  square tiling gives Eq. (10) exactly and a P x 1 tiling gives the 1-d
  curve the paper compares slices with (Sec. 7), up to the factor
  1 / (1 + 2 halo / L) of the pad along the uncut side.

The pad of Sec. 6-7 is psi = 6 sqrt(D dt), the form that reproduces the
paper's printed bounds.  The multi-GPU layout of this library exchanges a
halo of 2 psi (so that every ghost's row sum is local): pass ``halo=2 psi``
to plan for it.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple


def pad(d: float, dt: float) -> float:
    """Pad (ghost-region) width psi = 6 sqrt(D dt) of Sec. 6."""
    if d <= 0.0 or dt <= 0.0:
        raise ValueError("D and dt must be positive")
    return 6.0 * math.sqrt(d * dt)


def dt_min(L: float, n: int, dim: int, d: float, beta: float = 1.0) -> float:
    """Smallest time step of the optimality condition (Sec. 2.2)."""
    if n < 1 or dim < 1 or d <= 0.0 or not 0.0 < beta <= 1.0:
        raise ValueError("need n >= 1, dim >= 1, D > 0 and beta in (0, 1]")
    spacing = L / n ** (1.0 / dim)
    return beta * spacing * spacing / (2.0 * d)


def speedup(p: float, L: float, halo: float, dim: int) -> float:
    """Predicted speedup on p processors with square/cubic subdomains, Eq. (10)."""
    return 1.0 / (p ** (-1.0 / dim) + 2.0 * halo / L) ** dim


def efficiency(p: float, L: float, halo: float, dim: int) -> float:
    """Predicted efficiency E_P = S_P / P, Eq. (11)."""
    return speedup(p, L, halo, dim) / p


def max_processors(e: float, L: float, halo: float, dim: int) -> float:
    """Most processors that keep the predicted efficiency >= e, Eq. (12)."""
    if not 0.0 < e < 1.0:
        raise ValueError("efficiency threshold must be in (0, 1)")
    if halo <= 0.0:
        raise ValueError("pad width must be positive")
    return (1.0 / e) * ((1.0 - e ** (1.0 / dim)) * L / (2.0 * halo)) ** dim


def slices_limit(L: float, halo: float) -> float:
    """Processor count at which a slice becomes thinner than the pad (Sec. 7)."""
    return L / halo


def largest_perfect_power(bound: float, dim: int) -> int:
    """Largest k^dim <= bound (at least 1): the checkerboard with
    square/cubic subdomains that the bound of Eq. (12) allows."""
    k = max(1, int(math.floor(bound ** (1.0 / dim))))
    while (k + 1) ** dim <= bound:
        k += 1
    while k > 1 and k ** dim > bound:
        k -= 1
    return k ** dim


def checkerboard_factors(p: int, width: float, height: float) -> Tuple[int, int]:
    """Tiles (along x, along y) of a 2-d checkerboard of p subdomains, Eq. (7).

    Among the factor pairs f1 <= f2 of p, the one whose ratio f2/f1 is
    closest to the aspect ratio A = max(W, H) / min(W, H); the larger factor
    goes along the longer side.  When two pairs are equally close, the more
    nearly square one is taken.  A prime p gives slices (p, 1)."""
    if p < 1 or width <= 0.0 or height <= 0.0:
        raise ValueError("need p >= 1 and a positive domain")
    a = max(width, height) / min(width, height)
    best = (1, p)
    for f1 in range(1, math.isqrt(p) + 1):
        if p % f1:
            continue
        f2 = p // f1
        # f2/f1 falls as f1 grows, so on a tie the later pair is the squarer one
        if abs(f2 / f1 - a) <= abs(best[1] / best[0] - a):
            best = (f1, f2)
    f1, f2 = best
    return (f2, f1) if width >= height else (f1, f2)


def tiling_speedup(tiles: Sequence[int], box: Sequence[float], halo: float) -> float:
    """Predicted speedup of a tiling with tiles[k] subdomains along axis k of
    a box of sides box[k]: N / N_S with N_S the subdomain grown by the pad on
    every side (Eq. (8) and Eq. (10) for a rectangular tiling)."""
    if len(tiles) != len(box) or not tiles:
        raise ValueError("one tile count per axis")
    s = 1.0
    for c, side in zip(tiles, box):
        if c < 1 or side <= 0.0:
            raise ValueError("tile counts >= 1 and positive sides")
        s *= side / (side / c + 2.0 * halo)
    return s
