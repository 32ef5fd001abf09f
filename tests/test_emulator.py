"""The GPU tile code run on the CPU (libhjw_emu.so: the same phases of hjw_tile.h, with
NaN-filled LDS and guard zones) against the oracle.  This checks the kernels' indexing
(ragged tiles, halos, boundaries) and arithmetic before and independently of any GPU run."""
import math

import numpy as np
import pytest

import emulator as EM
import oracle as O
from paper_1909_13263_amd import workloads as W

# FP64 must match to rounding; the FP32 stencil to single-precision rounding of the
# derivative (relative to the largest derivative on the grid).
TOL = {0: 1e-13, 1: 2e-6, 2: 2e-5}

# (100, 200) and (135, 260) hold tiles whose halo is inside the grid (the direct-index
# load path); the others exercise edge tiles and ragged tails.
SHAPES = [(8,), (37,), (160,), (1030,), (8, 8), (33, 65), (40, 70), (64, 64), (96, 130),
          (100, 200), (135, 260)]


@pytest.fixture(params=[(32, 8), (16, 8), (16, 4)], ids=["tile64x32", "tile64x16", "tile64x16s4"])
def tile_rows(request):
    EM.set_tile(*request.param)
    yield request.param
    EM.set_tile(32, 8)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_emulated_derivatives_match_oracle(shape, bc, prec, tile_rows):
    rng = np.random.default_rng(len(shape) * 1000 + sum(shape))
    phi = W.random_smooth_periodic(shape, seed=sum(shape)) + 0.05 * rng.normal(size=shape)
    h = tuple(0.05 + 0.01 * a for a in range(len(shape)))
    ref = O.derivatives(O.Problem(shape, h, O.H_LINEAR, (1.0, 0.0), bc), phi)
    got = EM.derivatives(phi, h, bc, prec)
    for g, r in zip(got, ref):
        assert np.isfinite(g).all()
        assert np.abs(g - r).max() <= TOL[prec] * np.abs(r).max()


def _cases():
    return [W.burgers1d(160), W.advect1d(37), W.negcos1d(50), W.burgers2d(96, ny=70),
            W.negcos2d(65, ny=33), W.levelset2d(100, ny=72), W.burgers2d(200, ny=100),
            W.levelset2d(260, ny=135)]


@pytest.mark.parametrize("case", range(8))
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_emulated_rk3_step_matches_oracle(case, prec, tile_rows):
    pr = _cases()[case]
    phi = pr.phi0()
    prob = O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc)
    ref, info = O.rk3_step(prob, phi, 0.0, pr.t_final, 0.5)
    rc, got, ei = EM.rk3_step(phi, pr.spacing, pr.ham, pr.params, 0.0, pr.t_final, 0.5, pr.bc,
                              prec)
    assert rc == 0
    assert ei[1] == pytest.approx(info.last_dt, rel=1e-12 if prec == 0 else 1e-5)
    assert np.abs(got - ref).max() <= {0: 1e-14, 1: 1e-7, 2: 1e-6}[prec] * np.abs(ref).max()


def test_emulated_step_flags_non_finite():
    pr = W.burgers2d(64)
    phi = pr.phi0()
    phi[10, 20] = math.inf
    rc, _, info = EM.rk3_step(phi, pr.spacing, pr.ham, pr.params, 0.0, 0.01, 0.5, pr.bc, 0)
    assert rc == -5 and info[8] == 1.0


def test_emulated_transpose_is_bitwise():
    """x and y go through the same sweep, so transposing phi swaps (u, v) exactly, and with
    a symmetric Hamiltonian a whole step commutes with the transpose bit for bit."""
    pr = W.burgers2d(96)
    phi = pr.phi0() + 0.01 * W.random_smooth_periodic(pr.shape, seed=9)
    u = EM.derivatives(phi, pr.spacing, 0, 0)
    v = EM.derivatives(np.ascontiguousarray(phi.T), pr.spacing, 0, 0)
    assert np.array_equal(u[0], v[2].T) and np.array_equal(u[1], v[3].T)
    for prec in (0, 1):
        _, a, _ = EM.rk3_step(phi, pr.spacing, pr.ham, pr.params, 0.0, 1.0, 0.5, 0, prec)
        _, b, _ = EM.rk3_step(np.ascontiguousarray(phi.T), pr.spacing, pr.ham, pr.params, 0.0,
                              1.0, 0.5, 0, prec)
        assert np.array_equal(a, b.T)


# --------------------------------------------------------------------------- WENO-JP
@pytest.fixture
def weno_jp():
    EM.set_scheme(O.WENO_JP)
    yield
    EM.set_scheme(O.WENO_L)


@pytest.mark.parametrize("shape", [(37,), (1030,), (8, 8), (33, 65), (100, 200), (135, 260)])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_emulated_jp_derivatives_match_oracle(shape, bc, prec, weno_jp):
    """The comparison scheme's indicators in the same tile code: against the oracle's
    WENO-JP, element by element."""
    rng = np.random.default_rng(len(shape) * 1000 + sum(shape) + 7)
    phi = W.random_smooth_periodic(shape, seed=sum(shape)) + 0.05 * rng.normal(size=shape)
    h = tuple(0.05 + 0.01 * a for a in range(len(shape)))
    ref = O.derivatives(O.Problem(shape, h, O.H_LINEAR, (1.0, 0.0), bc, scheme=O.WENO_JP), phi)
    got = EM.derivatives(phi, h, bc, prec)
    for g, r in zip(got, ref):
        assert np.abs(g - r).max() <= TOL[prec] * np.abs(r).max()


@pytest.mark.parametrize("case", [0, 3, 5, 7])
@pytest.mark.parametrize("prec", [0, 1])
def test_emulated_jp_rk3_step_matches_oracle(case, prec, weno_jp):
    pr = _cases()[case]
    phi = pr.phi0()
    prob = O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc, scheme=O.WENO_JP)
    ref, info = O.rk3_step(prob, phi, 0.0, pr.t_final, 0.5)
    rc, got, ei = EM.rk3_step(phi, pr.spacing, pr.ham, pr.params, 0.0, pr.t_final, 0.5, pr.bc,
                              prec)
    assert rc == 0
    assert ei[1] == pytest.approx(info.last_dt, rel=1e-12 if prec == 0 else 1e-5)
    assert np.abs(got - ref).max() <= {0: 1e-14, 1: 1e-7}[prec] * np.abs(ref).max()


# --------------------------------------------------------------------------- figure examples
def _origin(pr):
    return tuple(pr.coords(a)[0] for a in range(pr.dim)) + (0.0,) * (2 - pr.dim)


@pytest.mark.parametrize("name", ["ex35", "ex38", "ex310", "ex311", "ex312", "ex313"])
@pytest.mark.parametrize("prec", [0, 1])
def test_emulated_figure_examples_match_oracle(name, prec, tile_rows):
    """The Hamiltonians of Examples 3.5 and 3.8-3.12 (the quartic, the position-dependent
    control problem with node coordinates, the sqrt form) in the tile code, one step
    from a state part way along the solve."""
    pr = {"ex35": lambda: W.ex35_linear(160, 0.5), "ex38": lambda: W.ex38_quartic(100, 0.2),
          "ex310": lambda: W.ex310_sin2d(70, 0.2), "ex311": lambda: W.ex311_control(66, 0.2),
          "ex312": lambda: W.ex312_eikonal(72, 0.2),
          "ex313": lambda: W.ex313_curvature(66, 0.1, 0.05)}[name]()
    x0, y0 = _origin(pr)
    EM.set_origin(x0, y0)
    try:
        prob = O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc, origin=(x0, y0))
        phi, _ = O.rk3_step(prob, pr.phi0(), 0.0, pr.t_final, 0.5)
        ref, info = O.rk3_step(prob, phi, 0.0, pr.t_final, 0.5)
        rc, got, ei = EM.rk3_step(phi, pr.spacing, pr.ham, pr.params, 0.0, pr.t_final, 0.5,
                                  pr.bc, prec)
    finally:
        EM.set_origin(0.0, 0.0)
    assert rc == 0
    assert ei[1] == pytest.approx(info.last_dt, rel=1e-12 if prec == 0 else 1e-5)
    assert np.abs(got - ref).max() <= {0: 1e-14, 1: 1e-7}[prec] * np.abs(ref).max()


@pytest.mark.parametrize("shape", [(37,), (8, 8), (33, 65), (100, 200), (135, 260)])
@pytest.mark.parametrize("bc", [(2, 2), (2, 0), (0, 2), (1, 2)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_emulated_dirichlet_step_matches_oracle(shape, bc, prec, tile_rows):
    """Held boundary layers on ragged grids, alone and beside the other boundaries."""
    if len(shape) == 1 and bc[1] != 2:
        return
    bcs = bc if len(shape) == 2 else (bc[0], bc[0])
    h = tuple(0.05 + 0.01 * a for a in range(len(shape)))
    phi = W.random_smooth_periodic(shape, seed=sum(shape) + 3)
    prob = O.Problem(shape, h, O.H_BURGERS, (1.0, 1.0, 1.0), bcs)
    ref, info = O.rk3_step(prob, phi, 0.0, 1.0, 0.5)
    rc, got, ei = EM.rk3_step(phi, h, O.H_BURGERS, (1.0, 1.0, 1.0), 0.0, 1.0, 0.5, bcs, prec)
    assert rc == 0
    assert ei[1] == pytest.approx(info.last_dt, rel=1e-12 if prec == 0 else 1e-5)
    assert list(ei[4:8]) == pytest.approx(list(info.range), rel=1e-12 if prec == 0 else 1e-5)
    assert np.abs(got - ref).max() <= {0: 1e-14, 1: 1e-7, 2: 1e-6}[prec] * np.abs(ref).max()
    held = np.zeros(phi.shape, bool)
    if bcs[0] == 2:
        held[..., :3] = held[..., -3:] = True
    if len(shape) == 2 and bcs[1] == 2:
        held[:3, :] = held[-3:, :] = True
    p_cast = phi if prec < 2 else phi.astype(np.float32).astype(np.float64)
    assert np.array_equal(got[held], p_cast[held])


@pytest.mark.parametrize("shape", [(8, 8), (33, 65), (100, 200), (135, 260)])
@pytest.mark.parametrize("bc", [(0, 0), (2, 2), (0, 2)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_emulated_curvature_step_matches_oracle(shape, bc, prec, tile_rows):
    """Example 3.13's term in the tile code: its 3 x 3 stencil reaches the four corner
    cells beyond the plus-shaped region (NaN in the emulated LDS unless loaded), on
    ragged tiles and across periodic wraps."""
    h = (1.0 / shape[1], 1.0 / shape[0])
    params = (-1.0, 1.0, 0.05)
    phi = 0.05 * W.random_smooth_periodic(shape, seed=sum(shape) + 11)
    prob = O.Problem(shape, h, O.H_CURVATURE, params, bc)
    ref, info = O.rk3_step(prob, phi, 0.0, 1.0, 0.5)
    rc, got, ei = EM.rk3_step(phi, h, O.H_CURVATURE, params, 0.0, 1.0, 0.5, bc, prec)
    assert rc == 0
    assert ei[1] == pytest.approx(info.last_dt, rel=1e-12 if prec == 0 else 1e-5)
    tol = {0: 1e-14, 1: 1e-7, 2: 1e-6}[prec]
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("shape", [(37,), (160,), (33, 65), (100, 200), (135, 260)])
@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (2, 2), (0, 2)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_emulated_timed_step_matches_oracle(shape, bc, prec, tile_rows):
    """H(x, t, phi, D phi) = cos(w t)(a u + b v) + lam phi: each stage at its own time (the
    step starts at t = 0.3) with its own value of phi at the node."""
    h = tuple(2.0 / n for n in shape[::-1])
    params = (0.9, -0.6, 5.0, 0.8)
    phi = W.random_smooth_periodic(shape, seed=sum(shape) + 29)
    prob = O.Problem(shape, h, O.H_TIMED, params, bc)
    ref, info = O.rk3_step(prob, phi, 0.3, 1.0, 0.5)
    rc, got, ei = EM.rk3_step(phi, h, O.H_TIMED, params, 0.3, 1.0, 0.5, bc, prec)
    assert rc == 0
    assert ei[0] == info.t
    assert ei[1] == pytest.approx(info.last_dt, rel=1e-12 if prec == 0 else 1e-5)
    tol = {0: 1e-14, 1: 1e-7, 2: 1e-6}[prec]
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


# --------------------------------------------------------------------------- random sweep
@pytest.mark.parametrize("seed", range(40))
def test_emulated_random_configurations_match_oracle(seed):
    """Seeded random shapes, boundaries per axis, Hamiltonians, parameters and schemes:
    one step of the tile code against the oracle."""
    import random_configs as RC
    cfg = RC.random_config(seed)
    h = RC.spacing(cfg)
    bcs = cfg["bcs"] if len(cfg["shape"]) == 2 else (cfg["bcs"][0], cfg["bcs"][0])
    prob = O.Problem(cfg["shape"], h, cfg["ham"], cfg["params"], bcs, scheme=cfg["scheme"],
                     origin=RC.origin(cfg))
    ref, info = O.rk3_step(prob, cfg["phi"], 0.0, 1.0, 0.5)
    EM.set_scheme(cfg["scheme"])
    EM.set_origin(*RC.origin(cfg))
    try:
        rc, got, ei = EM.rk3_step(cfg["phi"], h, cfg["ham"], cfg["params"], 0.0, 1.0, 0.5, bcs, 0)
    finally:
        EM.set_scheme(O.WENO_L)
        EM.set_origin(0.0, 0.0)
    assert rc == 0
    assert ei[1] == pytest.approx(info.last_dt, rel=1e-12)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), cfg


@pytest.mark.parametrize("seed", range(20))
def test_emulated_random_timed_configurations_match_oracle(seed):
    """Seeded random configurations of H(x, t, phi, D phi) (shape, boundaries, (a, b, w, lam),
    scheme, start time): one step of the tile code against the oracle."""
    import random_configs as RC
    cfg = RC.random_timed_config(seed)
    h = RC.spacing(cfg)
    bcs = cfg["bcs"] if len(cfg["shape"]) == 2 else (cfg["bcs"][0], cfg["bcs"][0])
    prob = O.Problem(cfg["shape"], h, cfg["ham"], cfg["params"], bcs, scheme=cfg["scheme"])
    ref, info = O.rk3_step(prob, cfg["phi"], cfg["t0"], cfg["t0"] + 1.0, 0.5)
    EM.set_scheme(cfg["scheme"])
    try:
        rc, got, ei = EM.rk3_step(cfg["phi"], h, cfg["ham"], cfg["params"], cfg["t0"],
                                  cfg["t0"] + 1.0, 0.5, bcs, 0)
    finally:
        EM.set_scheme(O.WENO_L)
    assert rc == 0
    assert ei[1] == pytest.approx(info.last_dt, rel=1e-12)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), cfg["shape"]


LLF_CASES = [((160,), O.H_NEGCOS, (1.0, 0.0, 1.0), 0), ((37,), O.H_BURGERS, (1.0, 0.0, 1.0), 1),
             ((33, 65), O.H_BURGERS, (1.0, 1.0, 1.0), (0, 0)),
             ((100, 200), O.H_NEGCOS, (1.0, -0.5, 1.0), (0, 2)),
             ((135, 260), O.H_NORM, (1.0, 0.0), (1, 1)),
             ((40, 70), O.H_QUARTIC, (0.7, 0.4, 0.1), (2, 2)),
             ((64, 64), O.H_CURVATURE, (-1.0, 1.0, 0.05), (0, 0)),
             ((96, 130), O.H_TIMED, (0.9, -0.6, 5.0, 0.8), (0, 1))]


@pytest.mark.parametrize("case", range(len(LLF_CASES)))
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_emulated_local_dissipation_matches_oracle(case, prec):
    """HJW_OPT_DISSIPATION = 1: alpha per node over its own pair (the reading the printed
    Table 2 follows), on several families, boundaries and ragged shapes."""
    shape, ham, params, bc = LLF_CASES[case]
    h = tuple(2.0 / n for n in shape[::-1])
    phi = 0.5 * W.random_smooth_periodic(shape, seed=sum(shape) + 41)
    prob = O.Problem(shape, h, ham, params, bc, local_lf=True)
    ref, info = O.rk3_step(prob, phi, 0.2, 1.0, 0.5)
    EM.set_dissipation(1)
    try:
        rc, got, ei = EM.rk3_step(phi, h, ham, params, 0.2, 1.0, 0.5, bc, prec)
    finally:
        EM.set_dissipation(0)
    assert rc == 0
    assert ei[1] == pytest.approx(info.last_dt, rel=1e-12 if prec == 0 else 1e-5)
    tol = {0: 1e-14, 1: 1e-7, 2: 1e-6}[prec]
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    if prec == 0:   # and it is not the global reading
        glob, _ = O.rk3_step(O.Problem(shape, h, ham, params, bc), phi, 0.2, 1.0, 0.5)
        if ham not in (O.H_TIMED,):
            assert np.abs(glob - ref).max() > 1e3 * tol * np.abs(ref).max()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_emulated_timed_without_time_and_decay_is_linear_bitwise(prec):
    """w = lam = 0: the tile code of the time- and phi-dependent family computes a u + b v and
    the RK stages exactly as the linear Hamiltonian's (no contraction in the emulator)."""
    base = W.timed2d(130, 0.7, -0.3, 0.0, 0.0, 0.1, ny=100)
    phi = base.phi0()
    a = EM.rk3_step(phi, base.spacing, O.H_TIMED, base.params, 0.0, 0.1, 0.5, 0, prec)
    b = EM.rk3_step(phi, base.spacing, O.H_LINEAR, (0.7, -0.3), 0.0, 0.1, 0.5, 0, prec)
    assert a[0] == b[0] == 0 and np.array_equal(a[1], b[1])
