"""Python binding of ``libfp.so`` (the C ABI declared in ``include/fp.h``).

Argument marshalling only: every array is a torch float64 tensor on the
current HIP device, passed by ``data_ptr()``; every computation runs in the
library's gfx950 kernels on torch's current stream.  If the library is not
built this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfp.so")

FP_OK, FP_EINVAL, FP_EUNSUPPORTED, FP_EHIP, FP_ENOMEM, FP_ENONPHYS = 0, -1, -2, -3, -4, -5
FP_WENO5JS, FP_LINUP5, FP_WENO7JS, FP_WENOCU6 = 0, 1, 2, 3
FP_FP64, FP_MIXED32 = 0, 1
FP_BC_PERIODIC, FP_BC_FROZEN = 0, 1
FP_LLF, FP_GLF = 0, 1
FP_FACE_HOLD, FP_FACE_EXTRAP, FP_FACE_WALL, FP_FACE_SHOCK = 0, 1, 2, 3

EXPORTS = ["fp_state_bytes", "fp_metric_bytes", "fp_coord_bytes", "fp_work_bytes", "fp_metrics",
           "fp_face_fluxes", "fp_residual", "fp_residual_dir", "fp_rk3_step", "fp_rk3_step_noalloc", "fp_solve",
           "fp_max_dt",
           "fp_check_state", "fp_batch_create", "fp_batch_set", "fp_batch_rk3_step", "fp_batch_solve",
           "fp_batch_set_links", "fp_batch_autotune", "fp_batch_get_tiles", "fp_batch_profile_step", "fp_batch_destroy", "fp_release_cache", "fp_last_error",
           "fp_apply_bcs", "fp_solve_bcs", "fp_viscous_work_bytes", "fp_viscous_residual", "fp_solve_ns",
           "fp_profile_step"]


class FPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class FPGrid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * 3), ("ghost", C.c_int32),
                ("bc", C.c_int32 * 3)]


class FPScheme(C.Structure):
    _fields_ = [("recon", C.c_int32), ("metric_order", C.c_int32), ("reformulated", C.c_int32),
                ("precision", C.c_int32), ("gamma", C.c_double), ("weno_eps", C.c_double),
                ("splitting", C.c_int32), ("reserved", C.c_int32), ("mu", C.c_double),
                ("prandtl", C.c_double)]


class FPBcs(C.Structure):
    _fields_ = [("kind", (C.c_int32 * 2) * 3), ("mask", (C.c_void_p * 2) * 3), ("nodes", C.c_void_p),
                ("pre", C.c_double * 5), ("post", C.c_double * 5), ("normal", C.c_double * 3),
                ("offset", C.c_double), ("speed", C.c_double)]


class FPBlock(C.Structure):
    _fields_ = [("grid", FPGrid), ("met", C.c_void_p), ("q", C.c_void_p), ("work", C.c_void_p),
                ("dt", C.c_double)]


class FPLink(C.Structure):
    _fields_ = [("block", C.c_int32), ("axis", C.c_int32), ("side", C.c_int32), ("nbr", C.c_int32)]


_lib = None


def lib():
    """Load the library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FPError(FP_EHIP, f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        gp, sp, vp, dp = C.POINTER(FPGrid), C.POINTER(FPScheme), C.c_void_p, C.c_void_p
        for name in ("fp_state_bytes", "fp_metric_bytes", "fp_work_bytes", "fp_viscous_work_bytes"):
            getattr(L, name).argtypes = [gp]
            getattr(L, name).restype = C.c_size_t
        L.fp_coord_bytes.argtypes = [gp, C.c_int32]
        L.fp_coord_bytes.restype = C.c_size_t
        L.fp_metrics.argtypes = [gp, C.c_int32, dp, dp, vp]
        L.fp_face_fluxes.argtypes = [gp, sp, dp, dp, C.c_int32, dp, vp]
        L.fp_residual.argtypes = [gp, sp, dp, dp, dp, vp]
        L.fp_residual_dir.argtypes = [gp, sp, dp, dp, C.c_int32, dp, C.c_int32, vp]
        L.fp_rk3_step.argtypes = [gp, sp, dp, dp, dp, C.c_double, vp]
        L.fp_rk3_step_noalloc.argtypes = [gp, sp, dp, dp, C.c_double, vp]
        L.fp_solve.argtypes = [gp, sp, dp, dp, dp, C.c_double, C.c_int64, vp]
        L.fp_max_dt.argtypes = [gp, sp, dp, dp, C.c_double, dp, vp]
        L.fp_apply_bcs.argtypes = [gp, C.POINTER(FPBcs), dp, dp, C.c_double, vp]
        L.fp_viscous_residual.argtypes = [gp, sp, dp, dp, dp, dp, vp]
        L.fp_solve_ns.argtypes = [gp, sp, dp, dp, dp, dp, C.c_double, C.c_int64, vp]
        L.fp_solve_bcs.argtypes = [gp, sp, C.POINTER(FPBcs), dp, dp, dp, C.c_double, C.c_double, C.c_int64, vp]
        L.fp_check_state.argtypes = [gp, sp, dp, dp, vp]
        L.fp_profile_step.argtypes = [gp, sp, C.POINTER(FPBcs), dp, dp, dp, dp, C.c_double, C.c_double,
                                      C.POINTER(C.c_float), C.POINTER(C.c_int32), C.c_int32,
                                      C.POINTER(C.c_int32), vp]
        bp = C.c_void_p
        L.fp_batch_create.argtypes = [sp, C.c_int32, C.POINTER(C.c_void_p)]
        L.fp_batch_set.argtypes = [bp, C.POINTER(FPBlock), C.c_int32, vp]
        L.fp_batch_rk3_step.argtypes = [bp, vp]
        L.fp_batch_set_links.argtypes = [bp, C.POINTER(FPLink), C.c_int32, vp]
        L.fp_batch_solve.argtypes = [bp, C.c_int64, vp]
        L.fp_batch_autotune.argtypes = [bp, C.POINTER(C.c_int32), vp]
        L.fp_batch_get_tiles.argtypes = [bp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.fp_batch_profile_step.argtypes = [bp, C.POINTER(C.c_float), C.POINTER(C.c_int32), C.c_int32,
                                            C.POINTER(C.c_int32), vp]
        L.fp_batch_destroy.argtypes = [bp]
        L.fp_batch_destroy.restype = None
        L.fp_release_cache.argtypes = []
        L.fp_release_cache.restype = None
        L.fp_last_error.restype = C.c_char_p
        for name in ("fp_metrics", "fp_face_fluxes", "fp_residual", "fp_residual_dir", "fp_rk3_step",
                     "fp_rk3_step_noalloc", "fp_solve",
                     "fp_max_dt", "fp_check_state", "fp_batch_create", "fp_batch_set", "fp_batch_rk3_step",
                     "fp_batch_solve", "fp_batch_autotune", "fp_batch_get_tiles", "fp_batch_profile_step",
                     "fp_batch_set_links",
                     "fp_apply_bcs", "fp_solve_bcs", "fp_viscous_residual", "fp_solve_ns", "fp_profile_step"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != FP_OK:
        raise FPError(rc, lib().fp_last_error().decode())


class Grid:
    """One structured block: ndim, interior nodes n, ghost width, boundary
    kind per axis (FP_BC_PERIODIC / FP_BC_FROZEN)."""

    def __init__(self, ndim, n, ghost=3, bc=None):
        if isinstance(n, int):
            n = [n] * ndim
        n = [int(v) for v in n] + [1] * (3 - len(n))
        if ndim == 2:
            n[2] = 1
        bc = list(bc) if bc is not None else [FP_BC_PERIODIC] * 3
        bc = [int(b) for b in bc] + [FP_BC_PERIODIC] * (3 - len(bc))
        self.ndim, self.n, self.ghost, self.bc = int(ndim), n, int(ghost), bc

    def c(self):
        g = FPGrid()
        g.ndim, g.ghost = self.ndim, self.ghost
        for d in range(3):
            g.n[d] = self.n[d]
            g.bc[d] = self.bc[d]
        return g

    @property
    def nv(self):
        return self.ndim + 2

    @property
    def nmet(self):
        return 10 if self.ndim == 3 else 5

    def state_shape(self, nv=None):
        ext = [self.n[d] + 2 * self.ghost for d in range(self.ndim)]
        return (self.nv if nv is None else nv,) + tuple(reversed(ext))

    def metric_shape(self):
        return self.state_shape(self.nmet)

    def coord_shape(self, Y):
        ext = [self.n[d] + 2 * (self.ghost + Y // 2) for d in range(self.ndim)]
        return (self.ndim,) + tuple(reversed(ext))

    def work_shape(self):
        """the RK3 workspace (see fp_work_bytes), flat: three state-sized
        arrays and a 256-double tail (the global LF speed sets and the
        device time of solve_bcs)"""
        vol = 1
        for e in self.state_shape():
            vol *= e
        return (3 * vol + 256,)


class Scheme:
    def __init__(self, recon="weno5", metric_order=6, reformulated=True, precision="fp64",
                 gamma=1.4, weno_eps=1e-6, splitting="llf", mu=0.0, prandtl=0.72):
        self.recon = {"weno5": FP_WENO5JS, "linup5": FP_LINUP5, "weno7": FP_WENO7JS,
                      "wenocu6": FP_WENOCU6}.get(recon, recon)
        self.splitting = {"llf": FP_LLF, "glf": FP_GLF}.get(splitting, splitting)
        self.mu, self.prandtl = float(mu), float(prandtl)
        self.precision = {"fp64": FP_FP64, "mixed": FP_MIXED32}.get(precision, precision)
        self.metric_order, self.reformulated = int(metric_order), int(bool(reformulated))
        self.gamma, self.weno_eps = float(gamma), float(weno_eps)

    def c(self):
        s = FPScheme()
        s.recon, s.metric_order, s.reformulated = int(self.recon), self.metric_order, self.reformulated
        s.precision, s.gamma, s.weno_eps = int(self.precision), self.gamma, self.weno_eps
        s.splitting, s.reserved = int(self.splitting), 0
        s.mu, s.prandtl = self.mu, self.prandtl
        return s


class Bcs:
    """Boundary faces (fp_apply_bcs): kind[axis][side] in FP_FACE_*, optional
    uint8 GPU masks per face {(axis, side): tensor} (1 = the kind applies),
    the state nodes' coordinates (float64 GPU tensor, ndim x state layout)
    for FP_FACE_SHOCK, and the shock's conservative states and plane."""

    def __init__(self, kind, mask=None, nodes=None, pre=None, post=None, normal=(1.0, 0.0, 0.0),
                 offset=0.0, speed=0.0):
        self.kind = [list(k) for k in kind] + [[FP_FACE_HOLD, FP_FACE_HOLD]] * (3 - len(kind))
        self.mask = dict(mask or {})
        for m in self.mask.values():
            if not isinstance(m, torch.Tensor) or not m.is_cuda or m.dtype != torch.uint8 or not m.is_contiguous():
                raise FPError(FP_EINVAL, "masks must be contiguous uint8 tensors on the GPU")
        if nodes is not None and (not nodes.is_cuda or nodes.dtype != torch.float64 or not nodes.is_contiguous()):
            raise FPError(FP_EINVAL, "nodes must be a contiguous float64 tensor on the GPU")
        self.nodes = nodes
        self.pre = list(pre or []) + [0.0] * (5 - len(pre or []))
        self.post = list(post or []) + [0.0] * (5 - len(post or []))
        self.normal = list(normal) + [0.0] * (3 - len(normal))
        self.offset, self.speed = float(offset), float(speed)

    def c(self, grid: "Grid"):
        b = FPBcs()
        for a in range(3):
            for sd in range(2):
                b.kind[a][sd] = int(self.kind[a][sd])
                m = self.mask.get((a, sd))
                if m is not None:
                    need = 1
                    for e in range(grid.ndim):
                        if e != a:
                            need *= grid.n[e]
                    if m.numel() < need:
                        raise FPError(FP_EINVAL, f"mask of face ({a}, {sd}) needs {need} bytes")
                    b.mask[a][sd] = m.data_ptr()
        if self.nodes is not None:
            if self.nodes.numel() * 8 < grid.ndim * state_bytes(grid) // grid.nv:
                raise FPError(FP_EINVAL, "nodes is smaller than ndim state-layout arrays")
            b.nodes = self.nodes.data_ptr()
        for v in range(5):
            b.pre[v], b.post[v] = float(self.pre[v]), float(self.post[v])
        for c in range(3):
            b.normal[c] = float(self.normal[c])
        b.offset, b.speed = self.offset, self.speed
        return b


def _dev(t: torch.Tensor, nbytes: int, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise FPError(FP_EINVAL, f"{name} must be a float64 tensor on the GPU")
    if not t.is_contiguous():
        raise FPError(FP_EINVAL, f"{name} must be contiguous")
    if t.numel() * 8 < nbytes:
        raise FPError(FP_EINVAL, f"{name} holds {t.numel() * 8} bytes, needs {nbytes}")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def state_bytes(grid: Grid) -> int:
    g = grid.c()
    return int(lib().fp_state_bytes(C.byref(g)))


def metric_bytes(grid: Grid) -> int:
    g = grid.c()
    return int(lib().fp_metric_bytes(C.byref(g)))


def coord_bytes(grid: Grid, Y: int) -> int:
    g = grid.c()
    return int(lib().fp_coord_bytes(C.byref(g), int(Y)))


def work_bytes(grid: Grid) -> int:
    g = grid.c()
    return int(lib().fp_work_bytes(C.byref(g)))


def metrics(grid: Grid, Y: int, xyz: torch.Tensor, met: torch.Tensor | None = None) -> torch.Tensor:
    if met is None:
        met = torch.zeros(grid.metric_shape(), dtype=torch.float64, device=xyz.device)
    g = grid.c()
    _check(lib().fp_metrics(C.byref(g), int(Y), _dev(xyz, coord_bytes(grid, Y), "xyz"),
                            _dev(met, metric_bytes(grid), "met"), _stream()))
    return met


def face_fluxes(grid: Grid, scheme: Scheme, met, q, direction: int, out=None) -> torch.Tensor:
    ext = list(grid.n[:grid.ndim])
    ext[direction] += 1
    shape = (grid.nv,) + tuple(reversed(ext))
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=q.device)
    g, s = grid.c(), scheme.c()
    nbytes = 8 * grid.nv
    for e in ext:
        nbytes *= e
    _check(lib().fp_face_fluxes(C.byref(g), C.byref(s), _dev(met, metric_bytes(grid), "met"),
                                _dev(q, state_bytes(grid), "q"), int(direction),
                                _dev(out, nbytes, "flux"), _stream()))
    return out


def residual(grid: Grid, scheme: Scheme, met, q, dqdt=None) -> torch.Tensor:
    if dqdt is None:
        dqdt = torch.zeros_like(q)
    g, s = grid.c(), scheme.c()
    _check(lib().fp_residual(C.byref(g), C.byref(s), _dev(met, metric_bytes(grid), "met"),
                             _dev(q, state_bytes(grid), "q"), _dev(dqdt, state_bytes(grid), "dqdt"),
                             _stream()))
    return dqdt


def residual_dir(grid: Grid, scheme: Scheme, met, q, direction: int, acc, accumulate=False):
    g, s = grid.c(), scheme.c()
    _check(lib().fp_residual_dir(C.byref(g), C.byref(s), _dev(met, metric_bytes(grid), "met"),
                                 _dev(q, state_bytes(grid), "q"), int(direction),
                                 _dev(acc, state_bytes(grid), "acc"), int(bool(accumulate)),
                                 _stream()))
    return acc


def rk3_step(grid: Grid, scheme: Scheme, met, q, work, dt: float) -> torch.Tensor:
    g, s = grid.c(), scheme.c()
    _check(lib().fp_rk3_step(C.byref(g), C.byref(s), _dev(met, metric_bytes(grid), "met"),
                             _dev(q, state_bytes(grid), "q"), _dev(work, work_bytes(grid), "work"),
                             float(dt), _stream()))
    return q


# the workspace limit of fp_rk3_step_noalloc (FP_NOALLOC_WORK_BYTES in fp.h)
NOALLOC_WORK_BYTES = 64 << 20


def rk3_step_noalloc(grid: Grid, scheme: Scheme, met, q, dt: float) -> torch.Tensor:
    """fp_rk3_step with the library's static per-GPU workspace (no device
    allocation by the caller or the library)."""
    g, s = grid.c(), scheme.c()
    _check(lib().fp_rk3_step_noalloc(C.byref(g), C.byref(s), _dev(met, metric_bytes(grid), "met"),
                                     _dev(q, state_bytes(grid), "q"), float(dt), _stream()))
    return q


def solve(grid: Grid, scheme: Scheme, met, q, work, dt: float, nsteps: int) -> torch.Tensor:
    g, s = grid.c(), scheme.c()
    _check(lib().fp_solve(C.byref(g), C.byref(s), _dev(met, metric_bytes(grid), "met"),
                          _dev(q, state_bytes(grid), "q"), _dev(work, work_bytes(grid), "work"),
                          float(dt), int(nsteps), _stream()))
    return q


def viscous_work_bytes(grid: Grid) -> int:
    g = grid.c()
    return int(lib().fp_viscous_work_bytes(C.byref(g)))


def viscous_work(grid: Grid, device="cuda") -> torch.Tensor:
    """the viscous node-flux workspace (fp_viscous_work_bytes), flat"""
    return torch.zeros(viscous_work_bytes(grid) // 8, dtype=torch.float64, device=device)


def viscous_residual(grid: Grid, scheme: Scheme, met, q, vwork, dqdt=None) -> torch.Tensor:
    if dqdt is None:
        dqdt = torch.zeros_like(q)
    g, s = grid.c(), scheme.c()
    _check(lib().fp_viscous_residual(C.byref(g), C.byref(s), _dev(met, metric_bytes(grid), "met"),
                                     _dev(q, state_bytes(grid), "q"), _dev(dqdt, state_bytes(grid), "dqdt"),
                                     _dev(vwork, viscous_work_bytes(grid), "vwork"), _stream()))
    return dqdt


def solve_ns(grid: Grid, scheme: Scheme, met, q, work, vwork, dt: float, nsteps: int) -> torch.Tensor:
    g, s = grid.c(), scheme.c()
    _check(lib().fp_solve_ns(C.byref(g), C.byref(s), _dev(met, metric_bytes(grid), "met"),
                             _dev(q, state_bytes(grid), "q"), _dev(work, work_bytes(grid), "work"),
                             _dev(vwork, viscous_work_bytes(grid), "vwork"), float(dt), int(nsteps), _stream()))
    return q


def apply_bcs(grid: Grid, bcs: Bcs, met, q, t: float) -> torch.Tensor:
    g, b = grid.c(), bcs.c(grid)
    _check(lib().fp_apply_bcs(C.byref(g), C.byref(b), _dev(met, metric_bytes(grid), "met"),
                              _dev(q, state_bytes(grid), "q"), float(t), _stream()))
    return q


def solve_bcs(grid: Grid, scheme: Scheme, bcs: Bcs, met, q, work, t0: float, dt: float,
              nsteps: int) -> torch.Tensor:
    g, s, b = grid.c(), scheme.c(), bcs.c(grid)
    _check(lib().fp_solve_bcs(C.byref(g), C.byref(s), C.byref(b), _dev(met, metric_bytes(grid), "met"),
                              _dev(q, state_bytes(grid), "q"), _dev(work, work_bytes(grid), "work"),
                              float(t0), float(dt), int(nsteps), _stream()))
    return q


# launch kinds of profile_step
PROFILE_KINDS = {0: "xi sweep", 1: "eta sweep", 2: "zeta sweep", 3: "frozen ghosts", 5: "GLF speeds",
                 6: "boundary faces", 7: "viscous fluxes", 8: "viscous divergence", 9: "speed-set reset"}


def profile_step(grid: Grid, scheme: Scheme, met, q, work, dt: float, bcs: "Bcs | None" = None, t: float = 0.0,
                 vwork=None):
    """One RK3 step of q with per-launch HIP-event timing (fp_profile_step):
    [(kind, ms)] in launch order (kinds: PROFILE_KINDS)."""
    g, s = grid.c(), scheme.c()
    b = C.byref(bcs.c(grid)) if bcs is not None else None
    vw = _dev(vwork, viscous_work_bytes(grid), "vwork") if vwork is not None else None
    ms = (C.c_float * 32)()
    kinds = (C.c_int32 * 32)()
    n = C.c_int32(0)
    _check(lib().fp_profile_step(C.byref(g), C.byref(s), b, _dev(met, metric_bytes(grid), "met"),
                                 _dev(q, state_bytes(grid), "q"), _dev(work, work_bytes(grid), "work"), vw,
                                 float(t), float(dt), ms, kinds, 32, C.byref(n), _stream()))
    return [(int(kinds[i]), float(ms[i])) for i in range(n.value)]


def max_dt(grid: Grid, scheme: Scheme, met, q, cfl: float, out=None) -> torch.Tensor:
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=q.device)
    g, s = grid.c(), scheme.c()
    _check(lib().fp_max_dt(C.byref(g), C.byref(s), _dev(met, metric_bytes(grid), "met"),
                           _dev(q, state_bytes(grid), "q"), float(cfl), _dev(out, 8, "dt"),
                           _stream()))
    return out


def check_state(grid: Grid, scheme: Scheme, q, flag=None) -> torch.Tensor:
    if flag is None:
        flag = torch.zeros(1, dtype=torch.int32, device=q.device)
    if not flag.is_cuda or flag.dtype != torch.int32:
        raise FPError(FP_EINVAL, "flag must be an int32 tensor on the GPU")
    g, s = grid.c(), scheme.c()
    _check(lib().fp_check_state(C.byref(g), C.byref(s), _dev(q, state_bytes(grid), "q"),
                                C.c_void_p(flag.data_ptr()), _stream()))
    return flag


class Batch:
    """Many independent blocks advanced by shared launches (fp_batch_*).

    set() takes (grid, met, q, work, dt) tuples of float64 GPU tensors; the
    tensors are kept referenced here until the next set() or close(), so the
    device memory the batch's work list points to stays alive."""

    def __init__(self, scheme: Scheme, max_blocks: int):
        self._sc = scheme.c()
        h = C.c_void_p()
        _check(lib().fp_batch_create(C.byref(self._sc), int(max_blocks), C.byref(h)))
        self._h = h
        self._keep = []
        self.max_blocks = int(max_blocks)

    def set(self, blocks):
        arr = (FPBlock * max(1, len(blocks)))()
        keep = []
        for i, (grid, met, q, work, dt) in enumerate(blocks):
            arr[i].grid = grid.c()
            arr[i].met = _dev(met, metric_bytes(grid), "met")
            arr[i].q = _dev(q, state_bytes(grid), "q")
            arr[i].work = _dev(work, work_bytes(grid), "work")
            arr[i].dt = float(dt)
            keep.append((met, q, work))
        _check(lib().fp_batch_set(self._h, arr, len(blocks), _stream()))
        self._keep = keep

    def set_links(self, links):
        """links: (block, axis, side, nbr) tuples (see fp_batch_set_links);
        interfaces shared both ways need both directions."""
        arr = (FPLink * max(1, len(links)))()
        for i, (blk, axis, side, nbr) in enumerate(links):
            arr[i].block, arr[i].axis, arr[i].side, arr[i].nbr = int(blk), int(axis), int(side), int(nbr)
        _check(lib().fp_batch_set_links(self._h, arr, len(links), _stream()))

    def rk3_step(self):
        _check(lib().fp_batch_rk3_step(self._h, _stream()))

    def solve(self, nsteps: int):
        _check(lib().fp_batch_solve(self._h, int(nsteps), _stream()))

    def autotune(self) -> int:
        """tune the eta and zeta segment targets; returns the eta target"""
        seg = C.c_int32(0)
        _check(lib().fp_batch_autotune(self._h, C.byref(seg), _stream()))
        return int(seg.value)

    def tiles(self) -> dict:
        """the current segment targets and whether the last autotune reused
        the process-wide cache"""
        e, z, c = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        _check(lib().fp_batch_get_tiles(self._h, C.byref(e), C.byref(z), C.byref(c)))
        return {"seg_eta": int(e.value), "seg_zeta": int(z.value), "from_cache": bool(c.value)}

    def profile_step(self):
        """One RK3 step with per-launch HIP-event timing: [(ndim, kind, ms)]
        in launch order, kind 0/1/2 = xi/eta/zeta sweep, 3 = ghost copy,
        4 = interface exchange."""
        ms = (C.c_float * 32)()
        kinds = (C.c_int32 * 32)()
        n = C.c_int32(0)
        _check(lib().fp_batch_profile_step(self._h, ms, kinds, 32, C.byref(n), _stream()))
        return [(kinds[i] // 16, kinds[i] % 16, float(ms[i])) for i in range(n.value)]

    def close(self):
        if self._h:
            lib().fp_batch_destroy(self._h)
            self._h = None
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def release_cache() -> None:
    lib().fp_release_cache()
