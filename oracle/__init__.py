"""Reference oracle for the arc-length WENO (WENO-L) Hamilton-Jacobi solver.

TEST INFRASTRUCTURE ONLY.  This package wraps ``weno_l_oracle.c``, a plain
scalar FP64 implementation written from Rathan & Biswas (arXiv:1909.13263),
Section 2.  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import it.  It shares no code with the GPU library.

Parity status of each routine (what pins it lives in ``tests/test_oracle_*``):
  weno_l_minus / weno_l_plus   pinned: brute force (Lagrange cubics + quadrature),
                               exactness on cubics, convergence orders
  weno_jp_minus / weno_jp_plus the comparison scheme (WENO-JP); pinned: its form equals
                               the weighted candidates, fifth-order rows with linear
                               weights, the WENO-JP columns of Tables 1-4
  arc_length                   pinned: adaptive quadrature, closed special cases
  derivatives                  pinned: brute force on 8-point grids, symmetries
  hamiltonian / lax_friedrichs pinned: consistency H_hat(u,u) = H(u), monotonicity
  dissipation                  closed forms pinned by brute-force box sampling;
                               the global-box reading itself is parity unpinned
  rk3_step / step_to           pinned: exact solutions (Examples 3.1-3.4), RK3 order;
                               the dt rule is a reading (parity unpinned); the stage
                               times of H(x, t, phi, Dphi) pinned by TVD-RK3's stability
                               polynomial and the closed form of H_TIMED
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "weno_l_oracle.c")
_LIB = os.path.join(_HERE, "libhjw_oracle.so")

BC_PERIODIC, BC_EXTRAP, BC_DIRICHLET = 0, 1, 2
H_LINEAR, H_BURGERS, H_NEGCOS, H_NORM, H_QUARTIC, H_CONTROL, H_CURVATURE, H_TIMED = range(8)
WENO_L, WENO_JP = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP over lines)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
             "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
                ("ham", ctypes.c_int32), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("hp", ctypes.c_double * 4),
                ("scheme", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("local_lf", ctypes.c_int32), ("pad2", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("t", ctypes.c_double), ("last_dt", ctypes.c_double),
                ("alpha_x", ctypes.c_double), ("alpha_y", ctypes.c_double),
                ("range", ctypes.c_double * 4)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_weno_l_minus.restype = ctypes.c_double
        lib.orc_weno_l_minus.argtypes = [dp, ctypes.c_double, dp, dp]
        lib.orc_weno_l_plus.restype = ctypes.c_double
        lib.orc_weno_l_plus.argtypes = [dp, ctypes.c_double, dp, dp]
        lib.orc_weno_jp_minus.restype = ctypes.c_double
        lib.orc_weno_jp_minus.argtypes = [dp, ctypes.c_double, dp, dp]
        lib.orc_weno_jp_plus.restype = ctypes.c_double
        lib.orc_weno_jp_plus.argtypes = [dp, ctypes.c_double, dp, dp]
        lib.orc_candidates.restype = None
        lib.orc_candidates.argtypes = [dp, dp]
        lib.orc_arc_length.restype = ctypes.c_double
        lib.orc_arc_length.argtypes = [ctypes.c_double] * 4
        lib.orc_derivatives.restype = ctypes.c_int
        lib.orc_derivatives.argtypes = [ctypes.POINTER(_Problem), dp, dp, dp, dp, dp]
        lib.orc_hamiltonian_at.restype = ctypes.c_double
        lib.orc_hamiltonian_at.argtypes = [ctypes.POINTER(_Problem)] + [ctypes.c_double] * 4
        lib.orc_hamiltonian_full.restype = ctypes.c_double
        lib.orc_hamiltonian_full.argtypes = [ctypes.POINTER(_Problem)] + [ctypes.c_double] * 6
        lib.orc_hamiltonian.restype = ctypes.c_double
        lib.orc_hamiltonian.argtypes = [ctypes.POINTER(_Problem), ctypes.c_double, ctypes.c_double]
        lib.orc_dissipation.restype = None
        lib.orc_dissipation.argtypes = [ctypes.POINTER(_Problem)] + [ctypes.c_double] * 4 + [dp, dp]
        lib.orc_lax_friedrichs.restype = ctypes.c_double
        lib.orc_lax_friedrichs.argtypes = [ctypes.POINTER(_Problem)] + [ctypes.c_double] * 6
        lib.orc_curvature_term.restype = ctypes.c_double
        lib.orc_curvature_term.argtypes = [ctypes.POINTER(_Problem), dp, ctypes.c_int64,
                                           ctypes.c_int64]
        lib.orc_rk3_step.restype = ctypes.c_int
        lib.orc_rk3_step.argtypes = [ctypes.POINTER(_Problem), dp, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.POINTER(_Info)]
        lib.orc_threads.restype = ctypes.c_int
        lib.orc_threads.argtypes = []
        lib.orc_step_to.restype = ctypes.c_int
        lib.orc_step_to.argtypes = [ctypes.POINTER(_Problem), dp, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int64, ctypes.POINTER(_Info)]
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Problem:
    """A uniform 1-D or 2-D grid with a built-in Hamiltonian.

    ``shape`` is (nx,) or (ny, nx) (row-major, x fastest); ``h`` is (dx,) or (dx, dy);
    ``bc`` is one code for all axes or a pair (bc_x, bc_y); ``params`` are the
    Hamiltonian parameters (see ``hamiltonian``); ``scheme`` is WENO_L or WENO_JP;
    ``origin`` is the (x, y) of node 0 (used by the position-dependent H_CONTROL)."""
    shape: tuple
    h: tuple
    ham: int
    params: tuple
    bc: object = BC_PERIODIC
    scheme: int = WENO_L
    origin: tuple = (0.0, 0.0)
    local_lf: bool = False   # alpha per node over its own pair: the reference for HJW_OPT_DISSIPATION = 1
    _c: _Problem = field(init=False, repr=False)

    def __post_init__(self):
        p = _Problem()
        p.dim = len(self.shape)
        if p.dim == 1:
            p.nx, p.ny = int(self.shape[0]), 1
            p.dx, p.dy = float(self.h[0]), 1.0
        else:
            p.ny, p.nx = int(self.shape[0]), int(self.shape[1])
            p.dx, p.dy = float(self.h[0]), float(self.h[1])
        bcs = self.bc if isinstance(self.bc, (tuple, list)) else (self.bc, self.bc)
        p.bc_x, p.bc_y = int(bcs[0]), int(bcs[1])
        p.ham = int(self.ham)
        p.scheme = int(self.scheme)
        p.x0 = float(self.origin[0])
        p.y0 = float(self.origin[1]) if len(self.origin) > 1 else 0.0
        p.local_lf = 1 if self.local_lf else 0
        hp = list(self.params) + [0.0] * (4 - len(self.params))
        for k in range(4):
            p.hp[k] = float(hp[k])
        self._c = p

    @property
    def dim(self):
        return len(self.shape)


@dataclass
class Info:
    steps: int
    t: float
    last_dt: float
    alpha_x: float
    alpha_y: float
    range: tuple


def _info(ci: _Info) -> Info:
    return Info(ci.steps, ci.t, ci.last_dt, ci.alpha_x, ci.alpha_y, tuple(ci.range))


def candidates(v):
    """The three third-order candidates of Step 2 from v = Delta^+ phi_{i-3..i+1}."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.shape == (5,)
    q = np.zeros(3)
    _load().orc_candidates(_dptr(v), _dptr(q))
    return q


def weno_l_minus(f, dx):
    """phi_x^- at x_i from phi_{i-3..i+2}; returns (u, beta[3], omega[3])."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert f.shape == (6,)
    beta = np.zeros(3)
    omega = np.zeros(3)
    u = lib.orc_weno_l_minus(_dptr(f), float(dx), _dptr(beta), _dptr(omega))
    return u, beta, omega


def weno_l_plus(g, dx):
    """phi_x^+ at x_i from phi_{i-2..i+3}; returns (u, beta[3], omega[3]) where
    index k refers to the reflected (left-biased) ordering of the sub-stencils."""
    lib = _load()
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert g.shape == (6,)
    beta = np.zeros(3)
    omega = np.zeros(3)
    u = lib.orc_weno_l_plus(_dptr(g), float(dx), _dptr(beta), _dptr(omega))
    return u, beta, omega


def weno_jp_minus(f, dx):
    """WENO-JP phi_x^- at x_i from phi_{i-3..i+2}; returns (u, IS[3], omega[3])."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert f.shape == (6,)
    ind = np.zeros(3)
    omega = np.zeros(3)
    u = lib.orc_weno_jp_minus(_dptr(f), float(dx), _dptr(ind), _dptr(omega))
    return u, ind, omega


def weno_jp_plus(g, dx):
    """WENO-JP phi_x^+ at x_i from phi_{i-2..i+3}; returns (u, IS[3], omega[3])."""
    lib = _load()
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert g.shape == (6,)
    ind = np.zeros(3)
    omega = np.zeros(3)
    u = lib.orc_weno_jp_plus(_dptr(g), float(dx), _dptr(ind), _dptr(omega))
    return u, ind, omega


def arc_length(b, c, x_lo, x_hi):
    """Length of a curve with slope b + 2 c x over [x_lo, x_hi]."""
    return _load().orc_arc_length(float(b), float(c), float(x_lo), float(x_hi))


def derivatives(prob: Problem, phi):
    """(u-, u+) in 1-D, (u-, u+, v-, v+) in 2-D, each shaped like phi."""
    lib = _load()
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    assert phi.shape == tuple(prob.shape)
    outs = [np.empty_like(phi) for _ in range(4)]
    rc = lib.orc_derivatives(ctypes.byref(prob._c), _dptr(phi), *[_dptr(o) for o in outs])
    if rc != 0:
        raise ValueError("orc_derivatives failed")
    return tuple(outs[:2]) if prob.dim == 1 else tuple(outs)


def hamiltonian(prob: Problem, u, v=0.0, x=0.0, y=0.0, t=0.0, phi=0.0):
    """H(x, t, phi, u, v): only H_CONTROL depends on the position (x, y), only H_TIMED on
    the time t and the node value phi."""
    return _load().orc_hamiltonian_full(ctypes.byref(prob._c), float(x), float(y), float(t),
                                        float(phi), float(u), float(v))


def dissipation(prob: Problem, A, B, C=0.0, D=0.0):
    ax = ctypes.c_double()
    ay = ctypes.c_double()
    _load().orc_dissipation(ctypes.byref(prob._c), float(A), float(B), float(C), float(D),
                            ctypes.byref(ax), ctypes.byref(ay))
    return ax.value, ay.value


def lax_friedrichs(prob: Problem, um, up, vm=0.0, vp=0.0, ax=0.0, ay=0.0):
    return _load().orc_lax_friedrichs(ctypes.byref(prob._c), float(um), float(up), float(vm),
                                      float(vp), float(ax), float(ay))


def curvature_term(prob: Problem, phi):
    """N / (1 + |grad phi|^2) at every node, from central differences (Example 3.13's
    term, without eps; see orc_curvature_term)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    lib = _load()
    ny, nx = phi.shape
    return np.array([[lib.orc_curvature_term(ctypes.byref(prob._c), _dptr(phi), i, j)
                      for i in range(nx)] for j in range(ny)])


def rk3_step(prob: Problem, phi, t, t_final, cfl):
    """One TVD-RK3 step; returns (phi_new, Info)."""
    lib = _load()
    out = np.array(phi, dtype=np.float64, copy=True, order="C")
    ci = _Info()
    ci.t = float(t)
    rc = lib.orc_rk3_step(ctypes.byref(prob._c), _dptr(out), float(t), float(t_final),
                          float(cfl), ctypes.byref(ci))
    if rc != 0:
        raise FloatingPointError(f"orc_rk3_step returned {rc}")
    return out, _info(ci)


def step_to(prob: Problem, phi, t_final, cfl, t0=0.0, max_steps=0):
    """Advance phi from t0 to t_final (at most max_steps steps if > 0); returns (phi, Info)."""
    lib = _load()
    out = np.array(phi, dtype=np.float64, copy=True, order="C")
    ci = _Info()
    ci.t = float(t0)
    rc = lib.orc_step_to(ctypes.byref(prob._c), _dptr(out), float(t_final), float(cfl),
                         int(max_steps), ctypes.byref(ci))
    if rc != 0:
        raise FloatingPointError(f"orc_step_to returned {rc}")
    return out, _info(ci)


def threads() -> int:
    """OpenMP threads the oracle's grid-line loops run on."""
    return int(_load().orc_threads())
