"""Seeded random solver configurations for the randomized parity sweeps: shape (ragged,
partial tiles), boundary per axis, Hamiltonian family and parameters, scheme, data."""
import numpy as np

from paper_1909_13263_amd import workloads as W


def random_config(seed):
    rng = np.random.default_rng(seed)
    dim = 2 if rng.random() < 0.8 else 1
    shape = (int(rng.integers(8, 1200)),) if dim == 1 else \
        (int(rng.integers(8, 260)), int(rng.integers(8, 260)))
    ham = int(rng.integers(0, 7 if dim == 2 else 5))
    bcs = [int(rng.integers(0, 3)) for _ in range(dim)]
    if ham == W.H_CURVATURE:
        bcs = [b if b != W.BC_EXTRAP else W.BC_DIRICHLET for b in bcs]
    a, b, c = rng.uniform(-1.5, 1.5, 3)
    params = {W.H_LINEAR: (a, b), W.H_BURGERS: (a, b, c), W.H_NEGCOS: (a, b, c),
              W.H_NORM: (a, float(rng.choice([0.0, 1.0]))), W.H_QUARTIC: (a, b, 0.3 * c),
              W.H_CONTROL: (), W.H_CURVATURE: (-1.0, 1.0, float(rng.uniform(0.0, 0.05)))}[ham]
    if dim == 1 and ham in (W.H_LINEAR, W.H_BURGERS, W.H_NEGCOS, W.H_QUARTIC):
        params = (params[0], 0.0) + tuple(params[2:])
    scheme = int(rng.integers(0, 2))
    lo = tuple(float(v) for v in rng.uniform(-2.0, 0.0, dim))
    hi = tuple(l + float(rng.uniform(0.5, 3.0)) for l in lo)
    phi = 0.5 * W.random_smooth_periodic(shape, seed=seed) + 0.02 * rng.normal(size=shape)
    return dict(shape=shape, ham=ham, params=tuple(float(p) for p in params), bcs=tuple(bcs),
                scheme=scheme, lo=lo, hi=hi, phi=phi)


def spacing(cfg):
    n = cfg["shape"][::-1]
    return tuple((cfg["hi"][d] - cfg["lo"][d]) / n[d] for d in range(len(n)))


def origin(cfg):
    """Coordinates of node 0 per axis: cell-centred on an extrapolated axis."""
    h = spacing(cfg)
    o = tuple(cfg["lo"][d] + (0.5 * h[d] if cfg["bcs"][d] == W.BC_EXTRAP else 0.0)
              for d in range(len(h)))
    return o + (0.0,) * (2 - len(o))


def random_timed_config(seed):
    """A random configuration of the time- and phi-dependent family (the general form of
    eq. (1.1)): shape, boundary per axis, (a, b, w, lam), scheme, data and a start time."""
    rng = np.random.default_rng(10_000 + seed)
    dim = 2 if rng.random() < 0.75 else 1
    shape = (int(rng.integers(8, 1200)),) if dim == 1 else \
        (int(rng.integers(8, 260)), int(rng.integers(8, 260)))
    bcs = [int(rng.integers(0, 3)) for _ in range(dim)]
    a, b = rng.uniform(-1.5, 1.5, 2)
    params = (float(a), float(b) if dim == 2 else 0.0, float(rng.uniform(0.0, 20.0)),
              float(rng.uniform(-2.0, 2.0)))
    scheme = int(rng.integers(0, 2))
    lo = tuple(float(v) for v in rng.uniform(-2.0, 0.0, dim))
    hi = tuple(l + float(rng.uniform(0.5, 3.0)) for l in lo)
    phi = 0.5 * W.random_smooth_periodic(shape, seed=seed + 500) + 0.02 * rng.normal(size=shape)
    return dict(shape=shape, ham=W.H_TIMED, params=params, bcs=tuple(bcs), scheme=scheme,
                lo=lo, hi=hi, phi=phi, t0=float(rng.uniform(0.0, 3.0)))
