"""Brute-force WENO-L on tiny periodic grids, in mpmath (test infrastructure).

Built only from definitions, with no closed forms of the scheme:
  - the candidate on a sub-stencil is P_k'(x_i), P_k the cubic interpolating phi
    at the sub-stencil's four nodes (solved from a Vandermonde system);
  - the indicator is beta_k = (integral over the cell of sqrt(1 + P_k''(x)^2))^2,
    evaluated by adaptive quadrature;
  - omega_k = alpha_k / sum(alpha), alpha_k = d_k / (eps + beta_k)^2;
  - the right-biased derivative uses the right-biased sub-stencils
    {x_{i-2+k}, ..., x_{i+1+k}} and the cell [x_i, x_{i+1}] directly (the mirror
    image of the left-biased construction about x_i), with linear weights
    (3/10, 6/10, 1/10) in that left-to-right order.
The Lax-Friedrichs flux, the dissipation (box maximum of |H_p| sampled densely
is checked separately) and TVD-RK3 are written out as in Section 2 of the paper.
"""
from __future__ import annotations

import mpmath as mp

EPS = mp.mpf("1e-6")
D_MINUS = (mp.mpf(1) / 10, mp.mpf(6) / 10, mp.mpf(3) / 10)
D_PLUS = (mp.mpf(3) / 10, mp.mpf(6) / 10, mp.mpf(1) / 10)


def _cubic(nodes, values):
    """Coefficients c0..c3 of the cubic through (nodes, values), nodes relative to x_i."""
    A = mp.matrix([[z**p for p in range(4)] for z in nodes])
    return mp.lu_solve(A, mp.matrix(values))


def _length(coef, a, b):
    # P''(z) = 2 c2 + 6 c3 z; split the quadrature where P'' changes sign (the integrand
    # bends sharply there when the slope is large)
    f = lambda z: mp.sqrt(1 + (2 * coef[2] + 6 * coef[3] * z) ** 2)
    pts = [a, b]
    if coef[3] != 0:
        z0 = -coef[2] / (3 * coef[3])
        if a < z0 < b:
            pts = [a, z0, b]
    return mp.quad(f, pts)


def one_sided(phi, i, dx, side):
    """phi_x^- (side=-1) or phi_x^+ (side=+1) at node i of a periodic grid phi.
    Returns (u, betas, omegas, candidates) in mpmath."""
    n = len(phi)
    dx = mp.mpf(dx)
    if side < 0:
        starts = (-3, -2, -1)        # S_k = {x_{i-3+k}, ..., x_{i+k}}
        cell = (-dx, mp.mpf(0))      # [x_{i-1}, x_i]
        d = D_MINUS
    else:
        starts = (-2, -1, 0)         # T_k = {x_{i-2+k}, ..., x_{i+1+k}}
        cell = (mp.mpf(0), dx)       # [x_i, x_{i+1}]
        d = D_PLUS
    q, beta = [], []
    for s in starts:
        offs = [s + m for m in range(4)]
        nodes = [o * dx for o in offs]
        vals = [mp.mpf(phi[(i + o) % n]) for o in offs]
        c = _cubic(nodes, vals)
        q.append(c[1])                           # P'(x_i)
        L = _length(c, cell[0], cell[1])
        beta.append(L * L)
    alpha = [d[k] / (EPS + beta[k]) ** 2 for k in range(3)]
    s = sum(alpha)
    omega = [a / s for a in alpha]
    u = sum(omega[k] * q[k] for k in range(3))
    return u, beta, omega, q


def derivatives_1d(phi, dx):
    n = len(phi)
    um = [one_sided(phi, i, dx, -1)[0] for i in range(n)]
    up = [one_sided(phi, i, dx, +1)[0] for i in range(n)]
    return um, up


def derivatives_2d(phi, dx, dy):
    """phi as a list of rows (phi[j][i]); returns (um, up, vm, vp) as lists of rows."""
    ny, nx = len(phi), len(phi[0])
    um = [[None] * nx for _ in range(ny)]
    up = [[None] * nx for _ in range(ny)]
    vm = [[None] * nx for _ in range(ny)]
    vp = [[None] * nx for _ in range(ny)]
    for j in range(ny):
        a, b = derivatives_1d(phi[j], dx)
        for i in range(nx):
            um[j][i], up[j][i] = a[i], b[i]
    for i in range(nx):
        col = [phi[j][i] for j in range(ny)]
        a, b = derivatives_1d(col, dy)
        for j in range(ny):
            vm[j][i], vp[j][i] = a[j], b[j]
    return um, up, vm, vp


def burgers(u, v, a=1, b=1, c=1):
    s = a * u + b * v + c
    return s * s / 2


def rk3_step_2d_burgers(phi, dx, dy, t_final, cfl):
    """One TVD-RK3 step of phi_t + (phi_x + phi_y + 1)^2/2 = 0 on a periodic grid,
    with alpha = max |H_p| over the box of phi^n's derivative ranges (|H_u| = |H_v| = |s|,
    s linear, so the box maximum sits at a corner) and dt = cfl/(alpha_x/dx + alpha_y/dy)
    clamped to t_final.  Returns (phi_new, dt, alpha)."""
    ny, nx = len(phi), len(phi[0])
    dx, dy = mp.mpf(dx), mp.mpf(dy)

    def L(p, ax, ay):
        um, up, vm, vp = derivatives_2d(p, dx, dy)
        out = [[None] * nx for _ in range(ny)]
        for j in range(ny):
            for i in range(nx):
                ub = (um[j][i] + up[j][i]) / 2
                vb = (vm[j][i] + vp[j][i]) / 2
                H = burgers(ub, vb)
                out[j][i] = -(H - ax * (up[j][i] - um[j][i]) / 2 - ay * (vp[j][i] - vm[j][i]) / 2)
        return out, (um, up, vm, vp)

    um, up, vm, vp = derivatives_2d(phi, dx, dy)
    allu = [x for r in um + up for x in r]
    allv = [x for r in vm + vp for x in r]
    A, B, C, D = min(allu), max(allu), min(allv), max(allv)
    corners = [A + C + 1, A + D + 1, B + C + 1, B + D + 1]
    m = max(abs(s) for s in corners)
    ax = ay = m
    dt = mp.mpf(cfl) / (ax / dx + ay / dy)
    dt = min(dt, mp.mpf(t_final))
    p0 = [[mp.mpf(x) for x in r] for r in phi]
    L0, _ = L(p0, ax, ay)
    p1 = [[p0[j][i] + dt * L0[j][i] for i in range(nx)] for j in range(ny)]
    L1, _ = L(p1, ax, ay)
    p2 = [[mp.mpf(3) / 4 * p0[j][i] + (p1[j][i] + dt * L1[j][i]) / 4 for i in range(nx)]
          for j in range(ny)]
    L2, _ = L(p2, ax, ay)
    p3 = [[p0[j][i] / 3 + 2 * (p2[j][i] + dt * L2[j][i]) / 3 for i in range(nx)]
          for j in range(ny)]
    return p3, dt, ax
