"""Pins of the oracle on the Hamiltonians and problems of the figure-only examples of
Section 3 of Rathan & Biswas (arXiv:1909.13263): Examples 3.5, 3.8, 3.10-3.12.  The paper
prints no numbers for them, so the references are the mathematics: the quartic's and the
control problem's Hamiltonians against finite differences and their closed-form
dissipation bounds, the exact solution of the linear Example 3.5, and the symmetries and
the comparison principle the exact solutions obey.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1909_13263_amd import workloads as W


def _problem(pr, scheme=O.WENO_L):
    origin = tuple(pr.coords(a)[0] for a in range(pr.dim))
    return O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc, scheme=scheme,
                     origin=origin + (0.0,) * (2 - len(origin)))


# --------------------------------------------------------------------------- Hamiltonians
@pytest.mark.parametrize("params", [(1.0, 0.0, 0.0), (1.0, 1.0, 0.0), (0.7, -1.3, 0.4)])
def test_quartic_dissipation_is_the_box_maximum(params):
    """(LF): alpha = max |H_u| over the box; the closed form (ends and the critical points
    +-sqrt(5/6) of s^3 - 5s/2) against dense sampling of central differences."""
    prob = O.Problem((8, 8), (0.1, 0.1), O.H_QUARTIC, params)
    rng = np.random.default_rng(3)
    for _ in range(12):
        A, B = sorted(rng.uniform(-2.5, 2.5, 2))
        C, D = sorted(rng.uniform(-2.5, 2.5, 2))
        ax, ay = O.dissipation(prob, A, B, C, D)
        U, V = np.meshgrid(np.linspace(A, B, 241), np.linspace(C, D, 241))
        h = 1e-6
        gx = (np.vectorize(lambda u, v: O.hamiltonian(prob, u + h, v))(U, V)
              - np.vectorize(lambda u, v: O.hamiltonian(prob, u - h, v))(U, V)) / (2 * h)
        gy = (np.vectorize(lambda u, v: O.hamiltonian(prob, u, v + h))(U, V)
              - np.vectorize(lambda u, v: O.hamiltonian(prob, u, v - h))(U, V)) / (2 * h)
        mx, my = np.abs(gx).max(), np.abs(gy).max()
        assert ax >= mx - 1e-5 and ay >= my - 1e-5
        assert ax <= mx * (1 + 1e-3) + 1e-5 and ay <= my * (1 + 1e-3) + 1e-5


def test_quartic_flux_is_consistent_and_monotone():
    prob = O.Problem((8,), (0.1,), O.H_QUARTIC, (1.0, 0.0, 0.0))
    rng = np.random.default_rng(5)
    for _ in range(200):
        u = rng.uniform(-2, 2)
        assert O.lax_friedrichs(prob, u, u, 0, 0, 3.0, 0.0) == pytest.approx(
            0.25 * (u * u - 1) * (u * u - 4), abs=1e-13)
    A, B = -2.0, 2.0
    ax, _ = O.dissipation(prob, A, B, 0, 0)
    for _ in range(200):
        um, up = rng.uniform(A, B, 2)
        d = 1e-4
        f = O.lax_friedrichs(prob, um, up, 0, 0, ax, 0)
        assert O.lax_friedrichs(prob, um, min(up + d, B), 0, 0, ax, 0) <= f + 1e-12
        assert O.lax_friedrichs(prob, min(um + d, B), up, 0, 0, ax, 0) >= f - 1e-12


def test_control_hamiltonian_derivatives_and_bounds():
    """Example 3.11: H is linear in u with slope sin y, has slope sin x + sign v in v, and
    the dissipation takes the bounds 1 and 2 of those slopes (attained on [-pi, pi)^2)."""
    prob = O.Problem((8, 8), (0.1, 0.1), O.H_CONTROL, ())
    rng = np.random.default_rng(11)
    h = 1e-6
    best = [0.0, 0.0]
    for _ in range(400):
        x, y = rng.uniform(-math.pi, math.pi, 2)
        u, v = rng.uniform(-3, 3, 2)
        if abs(v) < 1e-3:
            continue
        hu = (O.hamiltonian(prob, u + h, v, x, y) - O.hamiltonian(prob, u - h, v, x, y)) / (2 * h)
        hv = (O.hamiltonian(prob, u, v + h, x, y) - O.hamiltonian(prob, u, v - h, x, y)) / (2 * h)
        assert hu == pytest.approx(math.sin(y), abs=1e-7)
        assert hv == pytest.approx(math.sin(x) + math.copysign(1.0, v), abs=1e-7)
        best = [max(best[0], abs(hu)), max(best[1], abs(hv))]
    ax, ay = O.dissipation(prob, -1.0, 1.0, -1.0, 1.0)
    assert (ax, ay) == (1.0, 2.0)
    assert best[0] > 0.99 and best[1] > 1.98
    # at the origin, with phi = 0, H = 0 (no forcing there)
    assert O.hamiltonian(prob, 0.0, 0.0, 0.0, 0.0) == 0.0


# --------------------------------------------------------------------------- examples
def test_example35_against_the_exact_translate():
    """phi_t + phi_x = 0 carries the periodic profile: phi(x, t) = phi0(x - 0.5 - t).  The
    profile has kinks, so the grid-mean error falls at first order or better and the
    worst error sits at the kinks."""
    errs = []
    for n in (100, 200, 400):
        pr = W.ex35_linear(n, 2.0)
        phi, info = O.step_to(_problem(pr), pr.phi0(), pr.t_final, 0.5)
        ex = W.ex35_phi0(W.wrap_periodic(pr.coords(0) - 0.5 - pr.t_final))
        errs.append(float(np.abs(phi - ex).mean()))
    assert errs[0] < 0.04 and errs[1] < 0.6 * errs[0] and errs[2] < 0.7 * errs[1], errs


def test_example38_is_even():
    """phi0 = -2|x| and H(p) = H(-p): the solution stays even, x_i <-> x_{n-i}."""
    pr = W.ex38_quartic(100, 1.0)
    phi, _ = O.step_to(_problem(pr), pr.phi0(), 1.0, 0.5)
    assert np.abs(phi[1:] - phi[1:][::-1]).max() <= 1e-13
    assert phi.max() <= pr.phi0().max() + 1e-12          # H >= -9/16 ... bounded drift
    assert np.isfinite(phi).all()


def test_example311_point_symmetry():
    """H(-x, -y, u, v) = H(x, y, -u, -v) for the control problem, so with phi0 = 0 the
    solution is symmetric under (x, y) -> (-x, -y) on the periodic grid."""
    pr = W.ex311_control(60, 1.0)
    phi, _ = O.step_to(_problem(pr), pr.phi0(), 1.0, 0.5)
    sym = np.roll(np.roll(phi[::-1, ::-1], 1, 0), 1, 1)
    assert np.abs(phi - sym).max() <= 1e-13 * max(1.0, np.abs(phi).max())
    assert phi.max() > 1.0                                 # the forcing has acted


def test_example312_descends_at_unit_speed_or_faster():
    """H = sqrt(|grad phi|^2 + 1) >= 1, so phi(x, t) <= phi0(x) - t (comparison principle);
    the scheme keeps it to within its truncation error."""
    pr = W.ex312_eikonal(80, 0.6)
    phi, _ = O.step_to(_problem(pr), pr.phi0(), 0.6, 0.5)
    assert (phi - (pr.phi0() - 0.6)).max() <= 1e-5
