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

Figure-only examples of Section 3 (no printed numbers; see ``figure_examples``):
  ex35_linear    Example 3.5, phi_t + phi_x = 0, the piecewise phi0(x - 0.5), to t = 2 or 8
  ex38_quartic   Example 3.8, phi_t + (phi_x^2-1)(phi_x^2-4)/4 = 0, phi0 = -2|x|, to t = 1
  ex310_sin2d    Example 3.10, phi_t + sin(phi_x+phi_y) = 0, phi0 = pi(|y|-|x|) on [-1,1)^2
  ex311_control  Example 3.11, the optimal-control equation on [-pi,pi)^2, phi0 = 0, t = 1
  ex312_eikonal  Example 3.12, phi_t + sqrt(phi_x^2+phi_y^2+1) = 0 on [0,1)^2, t = 0.6

The general form phi_t + H(x, t, phi, D phi) = 0 of eq. (1.1) (no example of the paper):
  timed1d, timed2d  H = cos(w t)(a phi_x + b phi_y) + lam phi on [-1,1) / [-1,1)^2,
                    phi0 = -cos(pi x) (+ sin(pi y)/2 in 2-D)

Grid conventions: a periodic axis of n points on [lo, hi) has x_i = lo + i h,
h = (hi-lo)/n; an extrapolated axis is cell-centred, x_i = lo + (i+1/2) h.
Arrays are row-major with x fastest: phi[j, i] = phi(x_i, y_j).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

BC_PERIODIC, BC_EXTRAP, BC_DIRICHLET = 0, 1, 2
H_LINEAR, H_BURGERS, H_NEGCOS, H_NORM, H_QUARTIC, H_CONTROL, H_CURVATURE, H_TIMED = range(8)
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


def ex35_linear(n=100, t_final=2.0):
    return Problem("ex35_linear", (n,), (-1.0,), (1.0,), BC_PERIODIC, H_LINEAR, (1.0, 0.0),
                   t_final)


def ex38_quartic(n=100, t_final=1.0):
    return Problem("ex38_quartic", (n,), (-1.0,), (1.0,), BC_PERIODIC, H_QUARTIC,
                   (1.0, 0.0, 0.0), t_final)


def ex310_sin2d(n=80, t_final=1.0):
    # sin(s) = -cos(s + pi/2)
    return Problem("ex310_sin2d", (n, n), (-1.0, -1.0), (1.0, 1.0), BC_DIRICHLET, H_NEGCOS,
                   (1.0, 1.0, 0.5 * math.pi), t_final)


def ex311_control(n=60, t_final=1.0):
    return Problem("ex311_control", (n, n), (-math.pi, -math.pi), (math.pi, math.pi),
                   BC_PERIODIC, H_CONTROL, (), t_final)


def ex312_eikonal(n=80, t_final=0.6):
    return Problem("ex312_eikonal", (n, n), (0.0, 0.0), (1.0, 1.0), BC_PERIODIC, H_NORM,
                   (1.0, 1.0), t_final)


def ex313_curvature(n=60, eps=0.1, t_final=0.6):
    """Example 3.13: phi_t - (1 - eps K) sqrt(|grad phi|^2 + 1) = 0 on the periodic unit
    square, eps = 0 (convection only) or 0.1.  The paper gives no final time; 0.6 is
    Example 3.12's, whose domain and data (up to sign and shift) it shares."""
    return Problem("ex313_curvature", (n, n), (0.0, 0.0), (1.0, 1.0), BC_PERIODIC,
                   H_CURVATURE, (-1.0, 1.0, float(eps)), t_final)


def timed1d(n=160, a=1.0, w=2.0 * math.pi, lam=0.5, t_final=1.0):
    """phi_t + cos(w t) a phi_x + lam phi = 0, phi0 = -cos(pi x) on [-1,1)."""
    return Problem("timed1d", (n,), (-1.0,), (1.0,), BC_PERIODIC, H_TIMED,
                   (float(a), 0.0, float(w), float(lam)), t_final)


def timed2d(n=128, a=1.0, b=-0.5, w=2.0 * math.pi, lam=0.5, t_final=1.0, ny=None):
    """phi_t + cos(w t)(a phi_x + b phi_y) + lam phi = 0, phi0 = -cos(pi x) + sin(pi y)/2
    on [-1,1)^2."""
    return Problem("timed2d", (ny or n, n), (-1.0, -1.0), (1.0, 1.0), BC_PERIODIC, H_TIMED,
                   (float(a), float(b), float(w), float(lam)), t_final)


def figure_examples():
    """The figure-only examples of Section 3 at the paper's grid sizes and times (with
    the 1-D Burgers and -cos runs past the kink time, Examples 3.6 and 3.7, and the 2-D
    Burgers run of Example 3.9)."""
    return [ex35_linear(100, 2.0), ex35_linear(100, 8.0), burgers1d(40, 3.5 / math.pi**2),
            negcos1d(80, 1.5 / math.pi**2), ex38_quartic(100, 1.0),
            burgers2d(40, 1.5 / math.pi**2), ex310_sin2d(80, 1.0), ex311_control(60, 1.0),
            ex312_eikonal(80, 0.6), ex313_curvature(60, 0.0), ex313_curvature(60, 0.1)]


def ex35_phi0(x):
    """The piecewise initial profile of Example 3.5 (before its shift by 0.5), on [-1,1).
    The third piece is 15/2 - 3 cos(2 pi x): with the printed 5/2 the profile would jump by
    5 at x = 0 and at x = 1/3, while 15/2 makes it continuous at both (and the linear part
    makes it periodic)."""
    x = np.asarray(x, dtype=np.float64)
    lin = -(math.sqrt(3) / 2 + 4.5 + 2 * math.pi / 3) * (x + 1)
    out = np.where(x < -1 / 3, 2 * np.cos(1.5 * math.pi * x**2) - math.sqrt(3),
          np.where(x < 0, 1.5 + 3 * np.cos(2 * math.pi * x),
          np.where(x < 1 / 3, 7.5 - 3 * np.cos(2 * math.pi * x),
                   (28 + 4 * math.pi + np.cos(3 * math.pi * x)) / 3 + 6 * math.pi * x * (x - 1))))
    return lin + out


def wrap_periodic(x, lo=-1.0, hi=1.0):
    return lo + np.mod(np.asarray(x) - lo, hi - lo)


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
    if p.name == "ex35_linear":
        return ex35_phi0(wrap_periodic(p.coords(0) - 0.5))
    if p.name == "ex38_quartic":
        return -2.0 * np.abs(p.coords(0))
    if p.name == "ex310_sin2d":
        x, y = p.coords(0), p.coords(1)
        return math.pi * (np.abs(y)[:, None] - np.abs(x)[None, :])
    if p.name == "ex311_control":
        return np.zeros(p.shape)
    if p.name == "ex312_eikonal":
        x, y = p.coords(0), p.coords(1)
        return 0.25 * (np.cos(2 * math.pi * x)[None, :] - 1) * (np.cos(2 * math.pi * y)[:, None] - 1) - 1
    if p.name == "ex313_curvature":
        x, y = p.coords(0), p.coords(1)
        return 1 - 0.25 * (np.cos(2 * math.pi * x)[None, :] - 1) * (np.cos(2 * math.pi * y)[:, None] - 1)
    if p.name == "timed1d":
        return -np.cos(math.pi * p.coords(0))
    if p.name == "timed2d":
        x, y = p.coords(0), p.coords(1)
        return -np.cos(math.pi * x)[None, :] + 0.5 * np.sin(math.pi * y)[:, None]
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
