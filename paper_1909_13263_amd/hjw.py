"""Thin ctypes binding of the C ABI in include/hjw.h.

Argument marshalling only: every step of the scheme runs in the HIP library
(libhjw.so).  PyTorch provides the device workspace; nothing here computes.
Raises if the library was not built -- there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhjw.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE, ENONFINITE, EBUSY = 0, -1, -2, -3, -4, -5, -6
BC_PERIODIC, BC_EXTRAP, BC_DIRICHLET = 0, 1, 2
FP64, FP32_MIXED, FP32 = 0, 1, 2
H_LINEAR, H_BURGERS, H_NEGCOS, H_NORM, H_QUARTIC, H_CONTROL, H_CURVATURE, H_TIMED = range(8)
WENO_L, WENO_JP = 0, 1
OPT_USE_GRAPH = 0
OPT_KERNEL_EVENTS = 1
OPT_TILE_ROWS = 2
OPT_SEGMENT = 3
OPT_PLAN = 4
OPT_DISSIPATION = 5
KERNEL_NAMES = ("pre", "plan", "mid", "last")

PREC_NAMES = {"fp64": FP64, "fp32_mixed": FP32_MIXED, "fp32": FP32}


class HJWError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hjw error {code}: {msg}")
        self.code = code


class _Info(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("t", ctypes.c_double), ("last_dt", ctypes.c_double),
                ("alpha_x", ctypes.c_double), ("alpha_y", ctypes.c_double),
                ("range", ctypes.c_double * 4)]


class _Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64 * 2), ("lo", ctypes.c_double * 2),
                ("hi", ctypes.c_double * 2), ("bc", ctypes.c_int * 2), ("ham", ctypes.c_int),
                ("params", ctypes.c_double * 4), ("t_final", ctypes.c_double),
                ("cfl", ctypes.c_double), ("scheme", ctypes.c_int), ("reserved", ctypes.c_int)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("active", ctypes.c_int64), ("done", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("batched_steps", ctypes.c_int64), ("node_stages", ctypes.c_double),
                ("pool_bytes", ctypes.c_size_t), ("pool_in_use", ctypes.c_size_t),
                ("pool_peak", ctypes.c_size_t)]


@dataclass
class Info:
    steps: int
    t: float
    last_dt: float
    alpha_x: float
    alpha_y: float
    range: tuple


_lib = None

# Grids and servers still open when the interpreter exits are closed by an exit hook,
# before the interpreter tears its modules down: their pinned host buffers, graphs and
# events are then released while the HIP runtime is certainly still up.
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


def lib():
    """Load libhjw.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        sig = {
            "hjw_grid_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(i64), dp, dp,
                                               ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                               ctypes.POINTER(vp)]),
            "hjw_workspace_bytes": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_size_t)]),
            "hjw_bind": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp]),
            "hjw_set_hamiltonian": (ctypes.c_int, [vp, ctypes.c_int, dp, ctypes.c_int]),
            "hjw_set_scheme": (ctypes.c_int, [vp, ctypes.c_int]),
            "hjw_set_phi": (ctypes.c_int, [vp, vp, ctypes.c_int]),
            "hjw_step_to": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_double, i64,
                                           ctypes.POINTER(_Info)]),
            "hjw_get_phi": (ctypes.c_int, [vp, vp, ctypes.c_int]),
            "hjw_derivatives": (ctypes.c_int, [vp, vp, vp, vp, vp]),
            "hjw_get_info": (ctypes.c_int, [vp, ctypes.POINTER(_Info)]),
            "hjw_set_option": (ctypes.c_int, [vp, ctypes.c_int, i64]),
            "hjw_kernel_times": (ctypes.c_int, [vp, dp, ctypes.POINTER(i64)]),
            "hjw_time_kernels": (ctypes.c_int, [vp, ctypes.c_int, dp]),
            "hjw_grid_destroy": (None, [vp]),
            "hjw_solve_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(i64), dp, dp,
                                                 ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                                 ctypes.c_int, dp, ctypes.c_int, vp,
                                                 ctypes.c_double, ctypes.c_double, i64,
                                                 ctypes.POINTER(_Info), vp]),
            "hjw_server_footprint": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_Request),
                                                    ctypes.POINTER(ctypes.c_size_t)]),
            "hjw_server_create": (ctypes.c_int, [ctypes.c_int, vp, ctypes.c_size_t, ctypes.c_int,
                                                 vp, ctypes.POINTER(vp)]),
            "hjw_server_submit": (ctypes.c_int, [vp, ctypes.POINTER(_Request), dp,
                                                 ctypes.POINTER(i64)]),
            "hjw_server_run": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(i64),
                                              ctypes.POINTER(i64)]),
            "hjw_server_completed": (ctypes.c_int, [vp, ctypes.POINTER(i64), ctypes.c_int,
                                                    ctypes.POINTER(ctypes.c_int)]),
            "hjw_server_result": (ctypes.c_int, [vp, i64, dp, ctypes.POINTER(_Info), dp, dp]),
            "hjw_server_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(_ServerStats)]),
            "hjw_server_clock": (ctypes.c_double, [vp]),
            "hjw_server_destroy": (None, [vp]),
            "hjw_last_error": (ctypes.c_char_p, []),
            "hjw_version": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code != OK:
        raise HJWError(code, lib().hjw_last_error().decode())


def _info(ci: _Info) -> Info:
    return Info(int(ci.steps), ci.t, ci.last_dt, ci.alpha_x, ci.alpha_y, tuple(ci.range))


class Grid:
    """One solve: a uniform grid, a Hamiltonian and phi, resident on the GPU.

    shape is (nx,) or (ny, nx); lo, hi and bc are per axis, x first."""

    def __init__(self, shape, lo, hi, bc=BC_PERIODIC, prec=FP64, stream=None, workspace=None):
        import torch
        L = lib()
        self.shape = tuple(int(s) for s in shape)
        self.dim = len(self.shape)
        n = self.shape[::-1]
        bcs = bc if isinstance(bc, (tuple, list)) else (bc,) * self.dim
        if isinstance(prec, str):
            prec = PREC_NAMES[prec]
        self.prec = prec
        arr_n = (ctypes.c_int64 * self.dim)(*n)
        arr_lo = (ctypes.c_double * self.dim)(*[float(v) for v in lo])
        arr_hi = (ctypes.c_double * self.dim)(*[float(v) for v in hi])
        arr_bc = (ctypes.c_int * self.dim)(*[int(b) for b in bcs])
        h = ctypes.c_void_p()
        _check(L.hjw_grid_create(self.dim, arr_n, arr_lo, arr_hi, arr_bc, int(prec),
                                 ctypes.byref(h)))
        self._h = h
        nb = ctypes.c_size_t()
        _check(L.hjw_workspace_bytes(self._h, ctypes.byref(nb)))
        self.workspace_bytes = int(nb.value)
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device="cuda")
        self._ws = workspace
        s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        _live.add(self)
        _check(L.hjw_bind(self._h, ctypes.c_void_p(workspace.data_ptr()),
                          ctypes.c_size_t(workspace.numel()), ctypes.c_void_p(s)))

    @property
    def cells(self):
        return int(np.prod(self.shape))

    def set_hamiltonian(self, kind, params):
        p = (ctypes.c_double * 4)(*([float(v) for v in params] + [0.0] * (4 - len(params))))
        _check(lib().hjw_set_hamiltonian(self._h, int(kind), p, len(params)))

    def set_scheme(self, scheme):
        """WENO_L (default) or WENO_JP."""
        _check(lib().hjw_set_scheme(self._h, int(scheme)))

    def set_phi(self, phi):
        import torch
        if isinstance(phi, torch.Tensor) and phi.is_cuda:
            t = phi.detach().to(torch.float64).contiguous()
            assert tuple(t.shape) == self.shape
            torch.cuda.current_stream().synchronize()
            _check(lib().hjw_set_phi(self._h, ctypes.c_void_p(t.data_ptr()), 1))
        else:
            a = np.ascontiguousarray(np.asarray(phi, dtype=np.float64))
            assert a.shape == self.shape, (a.shape, self.shape)
            _check(lib().hjw_set_phi(self._h, a.ctypes.data_as(ctypes.c_void_p), 0))

    def step_to(self, t_final, cfl=0.5, max_steps=0) -> Info:
        ci = _Info()
        _check(lib().hjw_step_to(self._h, float(t_final), float(cfl), int(max_steps),
                                 ctypes.byref(ci)))
        return _info(ci)

    def info(self) -> Info:
        ci = _Info()
        _check(lib().hjw_get_info(self._h, ctypes.byref(ci)))
        return _info(ci)

    def get_phi(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float64)
        _check(lib().hjw_get_phi(self._h, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def get_phi_device(self, out=None):
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        _check(lib().hjw_get_phi(self._h, ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def derivatives(self):
        """(u-, u+) or (u-, u+, v-, v+) as FP64 CUDA tensors."""
        import torch
        outs = [torch.empty(self.shape, dtype=torch.float64, device="cuda") for _ in range(4)]
        ptrs = [ctypes.c_void_p(o.data_ptr()) for o in outs]
        _check(lib().hjw_derivatives(self._h, *ptrs))
        return tuple(outs[:2]) if self.dim == 1 else tuple(outs)

    def set_option(self, option, value):
        _check(lib().hjw_set_option(self._h, int(option), int(value)))

    def kernel_times(self):
        """{kernel: (total_ms, launches)} recorded with OPT_KERNEL_EVENTS on."""
        ms = (ctypes.c_double * 4)()
        cnt = (ctypes.c_int64 * 4)()
        _check(lib().hjw_kernel_times(self._h, ms, cnt))
        return {KERNEL_NAMES[k]: (ms[k], int(cnt[k])) for k in range(4)}

    def time_kernels(self, reps=50):
        """Average ms per launch of the kernels of a step ({pre, plan, mid, last}; plan is
        0 where the second stage plans for itself), reps back-to-back launches each between
        HIP events.  Leaves phi undefined (set it again before stepping)."""
        ms = (ctypes.c_double * 4)()
        _check(lib().hjw_time_kernels(self._h, int(reps), ms))
        return {"pre": ms[0], "plan": ms[1], "mid": ms[2], "last": ms[3]}

    def close(self):
        if getattr(self, "_h", None):
            lib().hjw_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_noalloc(shape, lo, hi, bc, prec, ham, params, phi, t_final, cfl=0.5, max_steps=0,
                  stream=None) -> Info:
    """hjw_solve_noalloc: one whole solve on the library's fixed device array, nothing
    allocated.  phi is a contiguous FP64 CUDA tensor of `shape`: phi0 in, the result out."""
    import torch
    assert isinstance(phi, torch.Tensor) and phi.is_cuda and phi.dtype == torch.float64
    assert phi.is_contiguous() and tuple(phi.shape) == tuple(shape)
    dim = len(shape)
    n = tuple(int(v) for v in shape)[::-1]
    bcs = bc if isinstance(bc, (tuple, list)) else (bc,) * dim
    p = [float(v) for v in params]
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    ci = _Info()
    _check(lib().hjw_solve_noalloc(dim, (ctypes.c_int64 * dim)(*n),
                                   (ctypes.c_double * dim)(*[float(v) for v in lo]),
                                   (ctypes.c_double * dim)(*[float(v) for v in hi]),
                                   (ctypes.c_int * dim)(*[int(b) for b in bcs]), int(prec),
                                   int(ham), (ctypes.c_double * 4)(*(p + [0.0] * (4 - len(p)))),
                                   len(p), ctypes.c_void_p(phi.data_ptr()), float(t_final),
                                   float(cfl), int(max_steps), ctypes.byref(ci),
                                   ctypes.c_void_p(s)))
    return _info(ci)


def grid_for(problem, prec=FP64, scheme=WENO_L, **kw) -> Grid:
    """A Grid for a workloads.Problem, with its Hamiltonian (and scheme) set."""
    g = Grid(problem.shape, problem.lo, problem.hi, problem.bc, prec, **kw)
    g.set_hamiltonian(problem.ham, problem.params)
    if scheme != WENO_L:
        g.set_scheme(scheme)
    return g


def _request(problem, scheme=WENO_L) -> _Request:
    """The C request record of a 2-D workloads.Problem."""
    if len(problem.shape) != 2:
        raise ValueError("the server takes 2-D problems")
    r = _Request()
    ny, nx = problem.shape
    r.n[0], r.n[1] = nx, ny
    for d in range(2):
        r.lo[d] = float(problem.lo[d])
        r.hi[d] = float(problem.hi[d])
    bcs = problem.bc if isinstance(problem.bc, (tuple, list)) else (problem.bc,) * 2
    r.bc[0], r.bc[1] = int(bcs[0]), int(bcs[1])
    r.ham = int(problem.ham)
    params = [float(v) for v in problem.params] + [0.0] * (4 - len(problem.params))
    for k in range(4):
        r.params[k] = params[k]
    r.t_final = float(problem.t_final)
    r.cfl = float(problem.cfl)
    r.scheme = int(scheme)
    return r


@dataclass
class Result:
    rid: int
    status: int
    phi: np.ndarray | None
    info: Info
    t_submit: float
    t_finish: float

    @property
    def latency(self):
        return self.t_finish - self.t_submit


class Server:
    """Continuous batching of many 2-D solves over one device pool (hjw_server_*).

    pool: a CUDA uint8 tensor (allocated here when None, pool_bytes long)."""

    def __init__(self, prec=FP32_MIXED, pool_bytes=1 << 30, max_active=256, pool=None,
                 stream=None):
        import torch
        if isinstance(prec, str):
            prec = PREC_NAMES[prec]
        self.prec = prec
        if pool is None:
            pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device="cuda")
        self._pool = pool
        s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        torch.cuda.current_stream().synchronize()
        h = ctypes.c_void_p()
        _check(lib().hjw_server_create(int(prec), ctypes.c_void_p(pool.data_ptr()),
                                       ctypes.c_size_t(pool.numel()), int(max_active),
                                       ctypes.c_void_p(s), ctypes.byref(h)))
        self._h = h
        self._shapes = {}
        _live.add(self)

    @staticmethod
    def footprint(problem, prec=FP32_MIXED) -> int:
        if isinstance(prec, str):
            prec = PREC_NAMES[prec]
        r = _request(problem)
        out = ctypes.c_size_t()
        _check(lib().hjw_server_footprint(int(prec), ctypes.byref(r), ctypes.byref(out)))
        return int(out.value)

    def submit(self, problem, phi0=None, scheme=WENO_L) -> int:
        r = _request(problem, scheme)
        a = problem.phi0() if phi0 is None else phi0
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        if a.shape != tuple(problem.shape):
            raise ValueError(f"phi0 shape {a.shape} != {problem.shape}")
        rid = ctypes.c_int64()
        _check(lib().hjw_server_submit(self._h, ctypes.byref(r),
                                       a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       ctypes.byref(rid)))
        self._shapes[int(rid.value)] = tuple(problem.shape)
        return int(rid.value)

    def run(self, chunks=1):
        """Run up to `chunks` chunks of batched steps; returns (active, queued)."""
        act, que = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().hjw_server_run(self._h, int(chunks), ctypes.byref(act), ctypes.byref(que)))
        return int(act.value), int(que.value)

    def completed(self, cap=4096):
        ids = (ctypes.c_int64 * cap)()
        cnt = ctypes.c_int()
        _check(lib().hjw_server_completed(self._h, ids, cap, ctypes.byref(cnt)))
        return [int(ids[k]) for k in range(cnt.value)]

    def result(self, rid) -> Result:
        """Collect (and release) a finished request; a failed request has phi None."""
        shape = self._shapes.pop(rid)
        out = np.empty(shape, dtype=np.float64)
        ci = _Info()
        ts, tf = ctypes.c_double(), ctypes.c_double()
        code = lib().hjw_server_result(self._h, int(rid),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       ctypes.byref(ci), ctypes.byref(ts), ctypes.byref(tf))
        if code not in (OK, ENONFINITE):
            self._shapes[rid] = shape
            _check(code)
        return Result(rid, code, out if code == OK else None, _info(ci), ts.value, tf.value)

    def stats(self) -> dict:
        st = _ServerStats()
        _check(lib().hjw_server_get_stats(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in _ServerStats._fields_}

    def clock(self) -> float:
        return float(lib().hjw_server_clock(self._h))

    def drain(self, chunks=4):
        """Run until nothing is queued or admitted; returns the finished results."""
        results = []
        while True:
            act, que = self.run(chunks)
            for rid in self.completed():
                results.append(self.result(rid))
            if act == 0 and que == 0:
                break
        return results

    def close(self):
        if getattr(self, "_h", None):
            lib().hjw_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
