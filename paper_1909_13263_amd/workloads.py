"""Seeded synthetic inputs shaped like the paper's test problems.

This module only generates initial data, grid coordinates and request streams;
it holds none of the scheme's arithmetic.  Both the GPU library's tests and the
oracle's tests draw their inputs from here.

Problems (Section 3 of Rathan & Biswas, arXiv:1909.13263, scaled up):
  burgers1d   Example 3.6's equation phi_t + (phi_x+1)^2/2 = 0, phi0 = -cos(pi x) on [-1,1)
  burgers2d   Example 3.3, phi_t + (phi_x+phi_y+1)^2/2 = 0, phi0 = -cos(pi(x+y)/2) on [-2,2)^2
  negcos2d    Example 3.4, phi_t - cos(phi_x+phi_y+1) = 0, same phi0 and domain
  levelset2d  phi_t + |grad phi| = 0 on [0,1]^2 (extrapolated boundaries), phi0 = signed
              distance to a union of 64 seeded circles (no paper example; closest is 3.12)
  advect1d    Example 3.1, phi_t + phi_x = 0, phi0 = -cos(pi x) on [-1,1)
  negcos1d    Example 3.2, phi_t - cos(phi_x+1) = 0, phi0 = -cos(pi x) on [-1,1)

Grid conventions: a periodic axis of n points on [lo, hi) has x_i = lo + i h,
h = (hi-lo)/n; an extrapolated axis is cell-centred, x_i = lo + (i+1/2) h.
Arrays are row-major with x fastest: phi[j, i] = phi(x_i, y_j).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

BC_PERIODIC, BC_EXTRAP = 0, 1
H_LINEAR, H_BURGERS, H_NEGCOS, H_NORM = 0, 1, 2, 3
CIRCLE_SEED = 13263
SERVE_SEED = 1909


@dataclass(frozen=True)
class Problem:
    name: str
    shape: tuple          # (n,) or (ny, nx)
    lo: tuple             # per axis, x first
    hi: tuple
    bc: int
    ham: int
    params: tuple         # Hamiltonian parameters (a, b, c) or (sigma, kappa)
    t_final: float
    cfl: float = 0.5
    seed: int = CIRCLE_SEED

    @property
    def dim(self) -> int:
        return len(self.shape)

    @property
    def spacing(self) -> tuple:
        n = self.shape[::-1]  # x first
        return tuple((self.hi[a] - self.lo[a]) / n[a] for a in range(self.dim))

    @property
    def cells(self) -> int:
        return int(np.prod(self.shape))

    def coords(self, axis: int) -> np.ndarray:
        n = self.shape[::-1][axis]
        h = self.spacing[axis]
        off = 0.5 if self.bc == BC_EXTRAP else 0.0
        return self.lo[axis] + (np.arange(n, dtype=np.float64) + off) * h

    def phi0(self) -> np.ndarray:
        return initial_data(self)


def burgers1d(n=160, t_final=0.5 / math.pi**2):
    return Problem("burgers1d", (n,), (-1.0,), (1.0,), BC_PERIODIC, H_BURGERS, (1.0, 0.0, 1.0),
                   t_final)


def advect1d(n=160, t_final=2.0):
    return Problem("advect1d", (n,), (-1.0,), (1.0,), BC_PERIODIC, H_LINEAR, (1.0, 0.0), t_final)


def negcos1d(n=160, t_final=0.5 / math.pi**2):
    return Problem("negcos1d", (n,), (-1.0,), (1.0,), BC_PERIODIC, H_NEGCOS, (1.0, 0.0, 1.0),
                   t_final)


def burgers2d(n=1024, t_final=0.5 / math.pi**2, ny=None):
    return Problem("burgers2d", (ny or n, n), (-2.0, -2.0), (2.0, 2.0), BC_PERIODIC, H_BURGERS,
                   (1.0, 1.0, 1.0), t_final)


def negcos2d(n=2048, t_final=1.0, ny=None):
    return Problem("negcos2d", (ny or n, n), (-2.0, -2.0), (2.0, 2.0), BC_PERIODIC, H_NEGCOS,
                   (1.0, 1.0, 1.0), t_final)


def levelset2d(n=4096, t_final=0.2, seed=CIRCLE_SEED, ny=None):
    return Problem("levelset2d", (ny or n, n), (0.0, 0.0), (1.0, 1.0), BC_EXTRAP, H_NORM,
                   (1.0, 0.0), t_final, seed=seed)


def circles(seed=CIRCLE_SEED, count=64):
    """Centres uniform in [0.1,0.9]^2 (drawn first), then radii uniform in [0.02,0.08]."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.1, 0.9, size=(count, 2))
    radii = rng.uniform(0.02, 0.08, size=count)
    return centres, radii


def initial_data(p: Problem) -> np.ndarray:
    if p.name in ("burgers1d", "advect1d", "negcos1d"):
        x = p.coords(0)
        return -np.cos(math.pi * x)
    if p.name in ("burgers2d", "negcos2d"):
        x = p.coords(0)
        y = p.coords(1)
        return -np.cos(math.pi * (x[None, :] + y[:, None]) / 2.0)
    if p.name == "levelset2d":
        centres, radii = circles(p.seed)
        return circle_distance(p.coords(0), p.coords(1), centres, radii)
    raise ValueError(p.name)


def circle_distance(x, y, centres, radii, tile=128, workers=None):
    """min over circles of (|(x, y) - c| - r) on the grid x (fastest) by y.

    Works tile by tile and skips, on each tile, the circles whose nearest possible
    distance exceeds the farthest distance to some other circle there; the minimum is
    exact, so the result does not depend on the skipping, the tiling or the threads."""
    from concurrent.futures import ThreadPoolExecutor
    cx, cy = centres[:, 0], centres[:, 1]
    out = np.empty((len(y), len(x)), dtype=np.float64)

    def work(j0, i0):
        xs, ys = x[i0:i0 + tile], y[j0:j0 + tile]
        near_x = np.maximum(0.0, np.maximum(xs[0] - cx, cx - xs[-1]))
        near_y = np.maximum(0.0, np.maximum(ys[0] - cy, cy - ys[-1]))
        far_x = np.maximum(np.abs(xs[0] - cx), np.abs(xs[-1] - cx))
        far_y = np.maximum(np.abs(ys[0] - cy), np.abs(ys[-1] - cy))
        lower = np.hypot(near_x, near_y) - radii
        upper = np.hypot(far_x, far_y) - radii
        keep = np.nonzero(lower <= upper.min() + 1e-9)[0]
        best = np.full((len(ys), len(xs)), np.inf)
        for k in keep:
            np.minimum(best, np.hypot(xs[None, :] - cx[k], ys[:, None] - cy[k]) - radii[k],
                       out=best)
        out[j0:j0 + tile, i0:i0 + tile] = best

    tiles = [(j0, i0) for j0 in range(0, len(y), tile) for i0 in range(0, len(x), tile)]
    workers = workers or min(16, os.cpu_count() or 1)
    if workers == 1 or len(tiles) < 4:
        for t in tiles:
            work(*t)
    else:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(lambda t: work(*t), tiles))
    return out


def random_smooth_periodic(shape, seed, modes=3):
    """A smooth periodic field (a few random Fourier modes), for tests."""
    rng = np.random.default_rng(seed)
    dims = len(shape)
    grids = np.meshgrid(*[np.arange(n) / n for n in shape], indexing="ij")
    out = np.zeros(shape)
    for _ in range(modes):
        k = rng.integers(1, 4, size=dims)
        ph = rng.uniform(0, 2 * math.pi)
        amp = rng.uniform(0.3, 1.0)
        arg = sum(2 * math.pi * k[a] * grids[a] for a in range(dims)) + ph
        out += amp * np.cos(arg)
    return out


@dataclass(frozen=True)
class Request:
    rid: int
    arrival: float        # seconds after the stream starts
    problem: Problem


def served_stream(count=2048, rate=200.0, seed=SERVE_SEED, n_min=64, n_max=1024):
    """Poisson arrivals at ``rate`` per second; square grids with side log-uniform in
    [n_min, n_max]; Hamiltonian uniform over the three 2-D families with their phi0;
    t_final uniform in [0.05, 0.5]."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    sides = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=count))).astype(int)
    kinds = rng.integers(0, 3, size=count)
    tfs = rng.uniform(0.05, 0.5, size=count)
    circle_seeds = rng.integers(0, 2**31 - 1, size=count)
    out = []
    for i in range(count):
        n = int(sides[i])
        if kinds[i] == 0:
            p = burgers2d(n, float(tfs[i]))
        elif kinds[i] == 1:
            p = negcos2d(n, float(tfs[i]))
        else:
            p = levelset2d(n, float(tfs[i]), seed=int(circle_seeds[i]))
        out.append(Request(i, float(arrivals[i]), p))
    return out
