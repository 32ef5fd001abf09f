"""Grids at and beyond the width up to which a tile's loads take 32-bit offsets.

Tiles whose halo lies inside the grid address their loads as the tile's origin plus a
32-bit byte offset, which rows of at most 2^22 nodes allow; tiles of wider grids take
the general (boundary-resolving) path.  Bar: a periodic grid whose data repeat every 64
nodes along x gives, after RK3 steps, the 64-wide grid's result repeated, bit for bit
(every node sees the same values, and the ranges, hence alpha and dt, are the same).
The 64-wide grid itself is checked against the oracle elsewhere.
"""
import math
import os

import numpy as np
import pytest

from paper_1909_13263_amd import hjw
from paper_1909_13263_amd import workloads as W

pytestmark = pytest.mark.gpu

H = 1.0 / 64.0          # grid spacing in both axes (exact in binary)
NY = 48                 # three rows of 16-row tiles: the middle one is interior
PERIOD = 64


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    assert os.path.dirname(hjw.LIB_PATH).endswith("paper_1909_13263_amd")
    yield


def _pattern():
    """A smooth doubly periodic phi0 on the 64 x 48 block (x = i h, y = j h)."""
    x = np.arange(PERIOD) * H
    y = np.arange(NY) * H
    ly = NY * H
    X, Y = np.meshgrid(x, y)
    return (np.sin(2 * math.pi * X) + 0.5 * np.cos(2 * math.pi * Y / ly) +
            0.25 * np.sin(2 * math.pi * (X - Y / ly)))


def _solve(nx, prec, phi0, steps):
    g = hjw.Grid((NY, nx), (0.0, 0.0), (nx * H, NY * H), W.BC_PERIODIC, prec)
    g.set_hamiltonian(W.H_BURGERS, (1.0, 1.0, 1.0))
    g.set_phi(phi0)
    info = g.step_to(1.0, 0.5, max_steps=steps)
    phi = g.get_phi()
    g.close()
    return phi, info


@pytest.mark.parametrize("nx,prec", [(1 << 22, hjw.FP32_MIXED), (1 << 22, hjw.FP64),
                                     ((1 << 22) + PERIOD, hjw.FP32_MIXED)])
def test_wide_grid_repeats_the_narrow_result(nx, prec):
    steps = 3
    pat = _pattern()
    ref, ref_info = _solve(PERIOD, prec, pat, steps)
    assert ref_info.steps == steps
    wide = np.tile(pat, (1, nx // PERIOD))
    print(f"wide grid {NY} x {nx}, prec {prec}", flush=True)
    phi, info = _solve(nx, prec, wide, steps)
    del wide
    assert info.steps == steps and info.t == ref_info.t
    assert info.alpha_x == ref_info.alpha_x and info.alpha_y == ref_info.alpha_y
    # compare block by block of whole periods (the whole grid is 200 M values)
    periods = nx // PERIOD
    step = -(-periods // 16)
    for p0 in range(0, periods, step):
        p1 = min(periods, p0 + step)
        blk = phi[:, p0 * PERIOD:p1 * PERIOD].reshape(NY, p1 - p0, PERIOD)
        assert np.array_equal(blk, np.broadcast_to(ref[:, None, :], blk.shape)), p0
