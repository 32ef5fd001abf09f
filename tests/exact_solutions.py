"""Exact solutions of the paper's smooth test problems (test infrastructure).

phi_t + H(phi_x) = 0 with smooth phi0 is solved before characteristics cross by
  x = xi + H'(p0(xi)) t,   phi(x,t) = phi0(xi) + t (p0 H'(p0) - H(p0)),   p0 = phi0'(xi)
(method of characteristics; Hopf-Lax/Legendre form of the Hamilton-Jacobi solution).
The 2-D problems of Examples 3.3 and 3.4 depend on zeta = (x+y)/2 only: with
phi(x,y) = chi((x+y)/2), phi_x + phi_y = chi', so chi solves the 1-D equation with
chi0 = -cos(pi zeta).

The general form phi_t + H(x, t, phi, D phi) = 0 with H = cos(w t)(a phi_x + b phi_y) + lam phi
(a linear transport with a time-dependent speed and a decay) has the solution
phi(x, y, t) = exp(-lam t) phi0(x - a S(t), y - b S(t)), S(t) = sin(w t) / w (S = t for w = 0).
"""
from __future__ import annotations

import math

import numpy as np


def _solve_1d(x, t, ham, phi0, p0, dp0, iters=60):
    """Newton on x = xi + H'(p0(xi)) t, then phi = phi0(xi) + t (p0 H'(p0) - H(p0))."""
    H, H1, H2 = ham
    xi = np.array(x, dtype=np.float64, copy=True)
    for _ in range(iters):
        p = p0(xi)
        g = xi + H1(p) * t - x
        dg = 1.0 + H2(p) * dp0(xi) * t
        step = g / dg
        xi -= step
        if np.max(np.abs(step)) < 1e-15:
            break
    p = p0(xi)
    return phi0(xi) + t * (p * H1(p) - H(p))


def cos_phi0(z):
    return -np.cos(math.pi * z)


def cos_p0(z):
    return math.pi * np.sin(math.pi * z)


def cos_dp0(z):
    return math.pi**2 * np.cos(math.pi * z)


# (H, H', H'') of the 1-D Hamiltonians
BURGERS = (lambda p: 0.5 * (p + 1.0) ** 2, lambda p: p + 1.0, lambda p: np.ones_like(p))
NEGCOS = (lambda p: -np.cos(p + 1.0), lambda p: np.sin(p + 1.0), lambda p: np.cos(p + 1.0))


def burgers_1d(x, t):
    """phi_t + (phi_x+1)^2/2 = 0, phi0 = -cos(pi x); valid for t < 1/pi^2."""
    return _solve_1d(np.asarray(x, float), t, BURGERS, cos_phi0, cos_p0, cos_dp0)


def negcos_1d(x, t):
    """phi_t - cos(phi_x+1) = 0, phi0 = -cos(pi x); valid before characteristics cross."""
    return _solve_1d(np.asarray(x, float), t, NEGCOS, cos_phi0, cos_p0, cos_dp0)


def burgers_2d(x, y, t):
    return burgers_1d((np.asarray(x)[None, :] + np.asarray(y)[:, None]) / 2.0, t)


def negcos_2d(x, y, t):
    return negcos_1d((np.asarray(x)[None, :] + np.asarray(y)[:, None]) / 2.0, t)


def advect_1d(x, t):
    return -np.cos(math.pi * (np.asarray(x) - t))


def levelset_circles(x, y, t, centres, radii):
    """phi_t + |grad phi| = 0 with phi0 = min_k(|x-c_k| - r_k): by the Hopf-Lax formula
    phi(x,t) = min_{|z-x|<=t} phi0(z) = min_k(max(|x-c_k| - t, 0) - r_k)."""
    X = np.asarray(x)[None, :]
    Y = np.asarray(y)[:, None]
    best = np.full((Y.shape[0], X.shape[1]), np.inf)
    for (cx, cy), r in zip(centres, radii):
        d = np.hypot(X - cx, Y - cy)
        np.minimum(best, np.maximum(d - t, 0.0) - r, out=best)
    return best


def errors(num, exact, cell_volume):
    """(L_inf, L_1) with L_1 = cell volume * sum |e| (the domain integral)."""
    e = np.abs(np.asarray(num) - np.asarray(exact))
    return float(e.max()), float(cell_volume * e.sum())


def timed(pr, t):
    """The solution of the timed1d / timed2d problems (periodic axes) at time t."""
    a, b, w, lam = pr.params
    s = math.sin(w * t) / w if w != 0.0 else t
    lo, hi = pr.lo[0], pr.hi[0]
    x = lo + np.mod(pr.coords(0) - a * s - lo, hi - lo)
    if pr.dim == 1:
        return math.exp(-lam * t) * -np.cos(math.pi * x)
    lo, hi = pr.lo[1], pr.hi[1]
    y = lo + np.mod(pr.coords(1) - b * s - lo, hi - lo)
    return math.exp(-lam * t) * (-np.cos(math.pi * x)[None, :] +
                                 0.5 * np.sin(math.pi * y)[:, None])
