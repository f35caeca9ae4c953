"""Python access to the plain FP64 CPU oracle (``oracle/fpo.c``).

TEST INFRASTRUCTURE ONLY: the oracle exists to check the GPU library against
the paper.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this package; it shares no code with the GPU path.

Arrays are numpy float64 in the layout documented in ``fpo.h``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fpo.c")
_LIB_PATH = os.path.join(_HERE, "libfpo.so")

GCC_FLAGS = ["-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
             "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no intrinsics, no fast math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Grid(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("g", C.c_int), ("bc", C.c_int * 3)]


class _Scheme(C.Structure):
    _fields_ = [("recon", C.c_int), ("Y", C.c_int), ("reformulated", C.c_int),
                ("gamma", C.c_double), ("eps", C.c_double), ("splitting", C.c_int),
                ("mu", C.c_double), ("prandtl", C.c_double)]


class _Bcs(C.Structure):
    _fields_ = [("kind", (C.c_int * 2) * 3), ("mask", (C.c_void_p * 2) * 3), ("nodes", C.c_void_p),
                ("pre", C.c_double * 5), ("post", C.c_double * 5), ("normal", C.c_double * 3),
                ("offset", C.c_double), ("speed", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        gp = C.POINTER(_Grid)
        sp = C.POINTER(_Scheme)
        L.fpo_metrics.argtypes = [gp, C.c_int, dp, dp]
        L.fpo_metrics_at.argtypes = [gp, C.c_int, dp, C.c_int, ip, dp]
        L.fpo_face_fluxes.argtypes = [gp, sp, dp, dp, C.c_int, dp]
        L.fpo_residual.argtypes = [gp, sp, dp, dp, dp]
        L.fpo_residual_at.argtypes = [gp, sp, dp, dp, C.c_int, ip, dp]
        L.fpo_residual_at_xyz.argtypes = [gp, sp, dp, dp, C.c_int, ip, dp]
        L.fpo_rk3_step.argtypes = [gp, sp, dp, dp, C.c_double]
        L.fpo_solve.argtypes = [gp, sp, dp, dp, C.c_double, C.c_long]
        bp = C.POINTER(_Bcs)
        L.fpo_apply_bcs.argtypes = [gp, bp, dp, dp, C.c_double]
        L.fpo_solve_bcs.argtypes = [gp, sp, bp, dp, dp, C.c_double, C.c_double, C.c_long]
        L.fpo_glf_speeds.argtypes = [gp, sp, dp, dp, C.c_int, dp]
        L.fpo_max_dt.argtypes = [gp, sp, dp, dp, C.c_double]
        L.fpo_max_dt.restype = C.c_double
        L.fpo_weno5.argtypes = [dp, C.c_double]
        L.fpo_weno5.restype = C.c_double
        L.fpo_linear_upwind5.argtypes = [dp]
        L.fpo_linear_upwind5.restype = C.c_double
        L.fpo_weno7.argtypes = [dp, C.c_double]
        L.fpo_weno7.restype = C.c_double
        L.fpo_weno7_parts.argtypes = [dp, dp, dp]
        L.fpo_weno7_parts.restype = None
        L.fpo_wenocu6.argtypes = [dp, C.c_double]
        L.fpo_wenocu6.restype = C.c_double
        L.fpo_wenocu6_parts.argtypes = [dp, dp, dp]
        L.fpo_wenocu6_parts.restype = None
        L.fpo_face_interp.argtypes = [C.c_int, dp]
        L.fpo_face_interp.restype = C.c_double
        L.fpo_eigensystem.argtypes = [C.c_int, C.c_double, dp, dp, dp, C.c_double, dp, dp, dp]
        L.fpo_num_threads.restype = C.c_int
        L.fpo_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _chk(rc, name):
    if rc != 0:
        raise ValueError(f"oracle {name} rejected its arguments (rc={rc})")


class Grid:
    def __init__(self, ndim, n, g=3, bc=None):
        if np.isscalar(n):
            n = [int(n)] * ndim
        n = list(n) + [1] * (3 - len(n))
        self.ndim, self.n, self.g = ndim, [int(v) for v in n], int(g)
        self.bc = list(bc) if bc is not None else [0, 0, 0]
        self.bc = self.bc + [0] * (3 - len(self.bc))
        if ndim == 2:
            self.n[2] = 1

    @property
    def nv(self):
        return self.ndim + 2

    @property
    def nmet(self):
        return 10 if self.ndim == 3 else 5

    def c(self):
        s = _Grid()
        s.ndim = self.ndim
        for d in range(3):
            s.n[d] = self.n[d]
            s.bc[d] = self.bc[d]
        s.g = self.g
        return s

    def state_shape(self, nv=None):
        nv = self.nv if nv is None else nv
        ext = [self.n[d] + 2 * self.g for d in range(self.ndim)]
        return (nv,) + tuple(reversed(ext))

    def metric_shape(self):
        return self.state_shape(self.nmet)


class Scheme:
    def __init__(self, recon="weno5", Y=6, reformulated=True, gamma=1.4, eps=1e-6, splitting="llf",
                 mu=0.0, prandtl=0.72):
        self.recon = {"weno5": 0, "linup5": 1, "weno7": 2, "wenocu6": 3}[recon] if isinstance(recon, str) else int(recon)
        self.Y, self.reformulated, self.gamma, self.eps = int(Y), bool(reformulated), gamma, eps
        self.splitting = {"llf": 0, "glf": 1}[splitting] if isinstance(splitting, str) else int(splitting)
        self.mu, self.prandtl = float(mu), float(prandtl)

    def c(self):
        s = _Scheme()
        s.recon, s.Y, s.reformulated = self.recon, self.Y, int(self.reformulated)
        s.gamma, s.eps, s.splitting = self.gamma, self.eps, self.splitting
        s.mu, s.prandtl = self.mu, self.prandtl
        return s


HOLD, EXTRAP, WALL, SHOCK = 0, 1, 2, 3


class Bcs:
    """boundary faces: kind[axis][side] in HOLD / EXTRAP / WALL / SHOCK, an
    optional byte mask per face (1 = the kind applies, 0 = hold), the state
    nodes' coordinates for SHOCK, and the shock's states and plane"""

    def __init__(self, kind, mask=None, nodes=None, pre=None, post=None, normal=(1.0, 0.0, 0.0),
                 offset=0.0, speed=0.0):
        self.kind = [list(k) for k in kind] + [[0, 0]] * (3 - len(kind))
        self.mask = mask or {}
        self.nodes = None if nodes is None else np.ascontiguousarray(nodes, dtype=np.float64)
        self.pre = list(pre or [0.0] * 5) + [0.0] * (5 - len(pre or []))
        self.post = list(post or [0.0] * 5) + [0.0] * (5 - len(post or []))
        self.normal = list(normal) + [0.0] * (3 - len(normal))
        self.offset, self.speed = float(offset), float(speed)
        self._keep = []

    def c(self):
        b = _Bcs()
        self._keep = []
        for a in range(3):
            for sd in range(2):
                b.kind[a][sd] = int(self.kind[a][sd])
                m = self.mask.get((a, sd))
                if m is not None:
                    m = np.ascontiguousarray(m, dtype=np.uint8)
                    self._keep.append(m)
                    b.mask[a][sd] = m.ctypes.data
        if self.nodes is not None:
            b.nodes = self.nodes.ctypes.data
        for v in range(5):
            b.pre[v], b.post[v] = self.pre[v], self.post[v]
        for c in range(3):
            b.normal[c] = self.normal[c]
        b.offset, b.speed = self.offset, self.speed
        return b


def _arr(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def metrics(grid: Grid, Y: int, xyz) -> np.ndarray:
    xyz = _arr(xyz)
    out = np.zeros(grid.metric_shape())
    _chk(lib().fpo_metrics(C.byref(grid.c()), Y, _dp(xyz), _dp(out)), "metrics")
    return out


def metrics_at(grid: Grid, Y: int, xyz, ijk) -> np.ndarray:
    xyz = _arr(xyz)
    ijk = np.ascontiguousarray(np.asarray(ijk, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((ijk.shape[0], grid.nmet))
    _chk(lib().fpo_metrics_at(C.byref(grid.c()), Y, _dp(xyz), ijk.shape[0], _ip(ijk), _dp(out)),
         "metrics_at")
    return out


def face_fluxes(grid: Grid, scheme: Scheme, met, q, direction: int) -> np.ndarray:
    met, q = _arr(met), _arr(q)
    ext = list(grid.n[:grid.ndim])
    ext[direction] += 1
    out = np.zeros((grid.nv,) + tuple(reversed(ext)))
    _chk(lib().fpo_face_fluxes(C.byref(grid.c()), C.byref(scheme.c()), _dp(met), _dp(q),
                               direction, _dp(out)), "face_fluxes")
    return out


def residual(grid: Grid, scheme: Scheme, met, q) -> np.ndarray:
    met, q = _arr(met), _arr(q)
    out = np.zeros_like(q)
    _chk(lib().fpo_residual(C.byref(grid.c()), C.byref(scheme.c()), _dp(met), _dp(q), _dp(out)),
         "residual")
    return out


def residual_at(grid: Grid, scheme: Scheme, met, q, ijk) -> np.ndarray:
    met, q = _arr(met), _arr(q)
    ijk = np.ascontiguousarray(np.asarray(ijk, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((ijk.shape[0], grid.nv))
    _chk(lib().fpo_residual_at(C.byref(grid.c()), C.byref(scheme.c()), _dp(met), _dp(q),
                               ijk.shape[0], _ip(ijk), _dp(out)), "residual_at")
    return out


def residual_at_xyz(grid: Grid, scheme: Scheme, xyz, q, ijk) -> np.ndarray:
    """Residual at selected nodes with metrics computed from the coordinates."""
    xyz, q = _arr(xyz), _arr(q)
    ijk = np.ascontiguousarray(np.asarray(ijk, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((ijk.shape[0], grid.nv))
    _chk(lib().fpo_residual_at_xyz(C.byref(grid.c()), C.byref(scheme.c()), _dp(xyz), _dp(q),
                                   ijk.shape[0], _ip(ijk), _dp(out)), "residual_at_xyz")
    return out


def rk3_step(grid: Grid, scheme: Scheme, met, q, dt: float) -> np.ndarray:
    met = _arr(met)
    q = np.array(q, dtype=np.float64, order="C", copy=True)
    _chk(lib().fpo_rk3_step(C.byref(grid.c()), C.byref(scheme.c()), _dp(met), _dp(q), dt),
         "rk3_step")
    return q


def solve(grid: Grid, scheme: Scheme, met, q, dt: float, nsteps: int) -> np.ndarray:
    met = _arr(met)
    q = np.array(q, dtype=np.float64, order="C", copy=True)
    _chk(lib().fpo_solve(C.byref(grid.c()), C.byref(scheme.c()), _dp(met), _dp(q), dt,
                         int(nsteps)), "solve")
    return q


def apply_bcs(grid: Grid, bcs: Bcs, met, q, t: float) -> np.ndarray:
    met = _arr(met)
    q = np.array(q, dtype=np.float64, order="C", copy=True)
    cb = bcs.c()
    _chk(lib().fpo_apply_bcs(C.byref(grid.c()), C.byref(cb), _dp(met), _dp(q), float(t)), "apply_bcs")
    return q


def solve_bcs(grid: Grid, scheme: Scheme, bcs: Bcs, met, q, t0: float, dt: float, nsteps: int) -> np.ndarray:
    met = _arr(met)
    q = np.array(q, dtype=np.float64, order="C", copy=True)
    cb = bcs.c()
    _chk(lib().fpo_solve_bcs(C.byref(grid.c()), C.byref(scheme.c()), C.byref(cb), _dp(met), _dp(q),
                             float(t0), float(dt), int(nsteps)), "solve_bcs")
    return q


def glf_speeds(grid: Grid, scheme: Scheme, met, q, d: int) -> np.ndarray:
    met, q = _arr(met), _arr(q)
    out = np.zeros(3)
    _chk(lib().fpo_glf_speeds(C.byref(grid.c()), C.byref(scheme.c()), _dp(met), _dp(q), int(d), _dp(out)),
         "glf_speeds")
    return out


def max_dt(grid: Grid, scheme: Scheme, met, q, cfl: float) -> float:
    met, q = _arr(met), _arr(q)
    return float(lib().fpo_max_dt(C.byref(grid.c()), C.byref(scheme.c()), _dp(met), _dp(q), cfl))


def weno5(v, eps=1e-6) -> float:
    v = _arr(v)
    return float(lib().fpo_weno5(_dp(v), eps))


def linear_upwind5(v) -> float:
    v = _arr(v)
    return float(lib().fpo_linear_upwind5(_dp(v)))


def weno7(v, eps=1e-6) -> float:
    v = _arr(v)
    return float(lib().fpo_weno7(_dp(v), eps))


def weno7_parts(v):
    """(candidate face values q[4], smoothness indicators beta[4])"""
    v = _arr(v)
    q, b = np.zeros(4), np.zeros(4)
    lib().fpo_weno7_parts(_dp(v), _dp(q), _dp(b))
    return q, b


def wenocu6(v, eps=1e-6) -> float:
    v = _arr(v)
    return float(lib().fpo_wenocu6(_dp(v), eps))


def wenocu6_parts(v):
    """(candidate face values q[4], smoothness measures beta[4], beta[3] = beta6)"""
    v = _arr(v)
    q, b = np.zeros(4), np.zeros(4)
    lib().fpo_wenocu6_parts(_dp(v), _dp(q), _dp(b))
    return q, b


def face_interp(Y: int, w) -> float:
    w = _arr(w)
    return float(lib().fpo_face_interp(Y, _dp(w)))


def eigensystem(ndim, gamma, qL, qR, sf, Vf):
    nv = ndim + 2
    L = np.zeros((nv, nv))
    R = np.zeros((nv, nv))
    lam = np.zeros(nv)
    _chk(lib().fpo_eigensystem(ndim, gamma, _dp(_arr(qL)), _dp(_arr(qR)), _dp(_arr(sf)), Vf,
                               _dp(L), _dp(R), _dp(lam)), "eigensystem")
    return L, R, lam


def num_threads() -> int:
    return int(lib().fpo_num_threads())


def set_num_threads(n: int) -> None:
    lib().fpo_set_num_threads(int(n))
