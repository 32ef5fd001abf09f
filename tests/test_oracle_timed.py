"""Pins of the oracle's general form phi_t + H(x, t, phi, D phi) = 0 (eq. (1.1)): the family
H = cos(w t)(a phi_x + b phi_y) + lam phi, which no example of the paper uses, evaluated by
Step 5 at the stage times t_n, t_n + dt, t_n + dt/2 with each stage's own phi.

- Pure decay (a = b = 0): TVD-RK3 applied to phi' = -lam phi multiplies phi by its stability
  polynomial 1 - z + z^2/2 - z^3/6 (z = lam dt) every step: exact up to rounding.  Using
  phi^n instead of the stage values, or another combination of stages, changes the factor.
- A time-dependent speed (lam = 0): the closed form phi0(x - a S(t)), S(t) = sin(w t)/w, is
  approached at third order in time; evaluating every stage at t_n would make it first
  order.
- w = 0, lam = 0 reduces to the linear Hamiltonian (Example 3.1) bit for bit.
"""
import math

import numpy as np
import pytest

import oracle as O
from exact_solutions import timed as _exact
from paper_1909_13263_amd import workloads as W


def _prob(pr):
    return O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc)


@pytest.mark.parametrize("lam", [0.5, 3.0, -1.2])
@pytest.mark.parametrize("t0", [0.0, 0.7])
def test_pure_decay_follows_the_rk3_stability_polynomial(lam, t0):
    pr = W.timed2d(24, a=0.0, b=0.0, w=3.0, lam=lam, t_final=t0 + 1.0)
    prob = _prob(pr)
    phi = W.random_smooth_periodic(pr.shape, seed=5) + 2.0
    t = t0
    cur = phi.copy()
    dts = []
    while t < pr.t_final:
        prev = cur
        cur, info = O.rk3_step(prob, prev, t, pr.t_final, 0.5)
        t = info.t
        dts.append(info.last_dt)
        z = lam * info.last_dt
        factor = 1.0 - z + z * z / 2.0 - z ** 3 / 6.0
        assert np.allclose(cur, factor * prev, rtol=4e-15, atol=0.0)
    # dt = cfl / |lam| (the zero-order term sets the rate when a = b = 0), the last step
    # clamped to t_final
    assert all(dt == 0.5 / abs(lam) for dt in dts[:-1])
    assert 0.0 < dts[-1] <= 0.5 / abs(lam)


@pytest.mark.parametrize("dim", [1, 2])
def test_time_dependent_speed_converges_at_third_order(dim):
    errs = []
    # from 80 nodes per unit length on (coarser 2-D grids are not yet in the asymptotic range)
    for n in ((40, 80, 160) if dim == 1 else (80, 160, 320)):
        pr = (W.timed1d(n, a=1.0, w=2 * math.pi, lam=0.0, t_final=0.3) if dim == 1 else
              W.timed2d(n, a=1.0, b=-0.5, w=2 * math.pi, lam=0.0, t_final=0.3))
        # a fixed CFL couples dt to h: the temporal error O(dt^3) dominates WENO's O(h^5)
        phi, info = O.step_to(_prob(pr), pr.phi0(), pr.t_final, 0.5)
        assert info.t == pr.t_final
        errs.append(np.abs(phi - _exact(pr, pr.t_final)).max())
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert errs[-1] < 2e-6, errs
    assert min(orders) > 2.5, (errs, orders)


def test_speed_and_decay_together_match_the_closed_form():
    pr = W.timed2d(96, a=0.8, b=-0.6, w=5.0, lam=0.9, t_final=0.5)
    phi, info = O.step_to(_prob(pr), pr.phi0(), pr.t_final, 0.5)
    exact = _exact(pr, pr.t_final)
    assert np.abs(phi - exact).max() < 2e-5 * np.abs(exact).max()


def test_without_time_and_decay_it_is_the_linear_hamiltonian():
    pr = W.timed2d(40, a=0.7, b=-0.3, w=0.0, lam=0.0, t_final=0.25)
    lin = O.Problem(pr.shape, pr.spacing, O.H_LINEAR, (0.7, -0.3), pr.bc)
    got, gi = O.step_to(_prob(pr), pr.phi0(), pr.t_final, 0.5)
    ref, ri = O.step_to(lin, pr.phi0(), pr.t_final, 0.5)
    assert gi.steps == ri.steps
    assert np.array_equal(got, ref)


def test_dissipation_bounds_the_speed_at_every_time():
    pr = W.timed2d(16, a=-1.5, b=0.25, w=7.0, lam=2.0)
    ax, ay = O.dissipation(_prob(pr), -3.0, 4.0, -1.0, 2.0)
    assert (ax, ay) == (1.5, 0.25)
    ts = np.linspace(0.0, 2.0, 1001)
    assert np.abs(-1.5 * np.cos(7.0 * ts)).max() <= ax
