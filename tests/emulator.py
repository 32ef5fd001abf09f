"""ctypes wrapper of libhjw_emu.so: the GPU tile code executed on the CPU (test support)."""
import ctypes
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU_PATH = os.path.join(ROOT, "paper_1909_13263_amd", "libhjw_emu.so")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(EMU_PATH):
            from paper_1909_13263_amd import build
            build.build_emulator()
        L = ctypes.CDLL(EMU_PATH)
        i64, d, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        L.hjw_emu_derivatives.restype = ctypes.c_int
        L.hjw_emu_derivatives.argtypes = [ctypes.c_int, i64, i64, d, d, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp]
        L.hjw_emu_set_tile_rows.restype = ctypes.c_int
        L.hjw_emu_set_tile_rows.argtypes = [ctypes.c_int]
        L.hjw_emu_set_segment.restype = ctypes.c_int
        L.hjw_emu_set_segment.argtypes = [ctypes.c_int]
        L.hjw_emu_set_dissipation.restype = ctypes.c_int
        L.hjw_emu_set_dissipation.argtypes = [ctypes.c_int]
        L.hjw_emu_set_scheme.restype = ctypes.c_int
        L.hjw_emu_set_scheme.argtypes = [ctypes.c_int]
        L.hjw_emu_set_origin.restype = None
        L.hjw_emu_set_origin.argtypes = [ctypes.c_double, ctypes.c_double]
        L.hjw_emu_step.restype = ctypes.c_int
        L.hjw_emu_step.argtypes = [ctypes.c_int, i64, i64, d, d, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, vp, vp, d, d, d, vp]
        _lib = L
    return _lib


def set_tile_rows(rows):
    assert lib().hjw_emu_set_tile_rows(int(rows)) == 0


def set_dissipation(local):
    """0: the step's global alpha; 1: alpha per node over its own pair (local LF)."""
    assert lib().hjw_emu_set_dissipation(int(local)) == 0


def set_scheme(scheme):
    """0 WENO-L, 1 WENO-JP for the emulated kernels."""
    assert lib().hjw_emu_set_scheme(int(scheme)) == 0


def set_origin(x0, y0=0.0):
    """Coordinates of node (0, 0) for the position-dependent Hamiltonians."""
    lib().hjw_emu_set_origin(float(x0), float(y0))


def set_tile(rows, segment):
    """2-D tile height and nodes per thread of the emulated kernels."""
    L = lib()
    assert L.hjw_emu_set_segment(8) == 0
    assert L.hjw_emu_set_tile_rows(int(rows)) == 0
    assert L.hjw_emu_set_segment(int(segment)) == 0


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _geom(shape, h, bc):
    bcs = bc if isinstance(bc, (tuple, list)) else (bc, bc)
    if len(shape) == 1:
        return 1, shape[0], 1, h[0], 1.0, bcs[0], 0
    return 2, shape[1], shape[0], h[0], h[1], bcs[0], bcs[1]


def derivatives(phi, h, bc=0, prec=0):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    dim, nx, ny, dx, dy, bx, by = _geom(phi.shape, h, bc)
    outs = [np.full(phi.shape, np.nan) for _ in range(4)]
    rc = lib().hjw_emu_derivatives(dim, nx, ny, dx, dy, bx, by, prec, _p(phi),
                                   *[_p(o) for o in outs])
    assert rc == 0, rc
    return tuple(outs[:2]) if dim == 1 else tuple(outs)


def rk3_step(phi, h, ham, params, t, t_final, cfl, bc=0, prec=0):
    out = np.array(phi, dtype=np.float64, copy=True, order="C")
    dim, nx, ny, dx, dy, bx, by = _geom(out.shape, h, bc)
    hp = np.zeros(4)
    hp[:len(params)] = params
    info = np.zeros(9)
    rc = lib().hjw_emu_step(dim, nx, ny, dx, dy, bx, by, prec, ham, _p(hp), _p(out), t,
                            t_final, cfl, _p(info))
    return rc, out, info
