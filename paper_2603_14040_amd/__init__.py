"""tephra: MI355X-native matrix-free multigrid Stokes solver (Python binding).

Thin wrapper over the C ABI of ``include/tephra.h``: torch tensors provide
device memory and the stream, every step of the solve runs in the HIP
library.  Field arrays are float64 CUDA tensors of shape (ny + 2, nx + 2) in
the staggered-grid convention documented in the header.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import (ACCEL_ANDERSON, ACCEL_FGMRES, ACCEL_GCR, FP64, FREE_SLIP, MEAN_ARITHMETIC,
                   MEAN_GEOMETRIC, MIXED, NO_SLIP, SMOOTH_GS, SMOOTH_JACOBI, SMOOTH_RAS, SMOOTH_RAS_MIXED,
                   TephraError)

__all__ = ["Solver", "Batch", "SolveInfo", "StokesFunction", "solve", "FP64", "MIXED", "FREE_SLIP",
           "NO_SLIP", "SMOOTH_GS", "SMOOTH_JACOBI", "SMOOTH_RAS", "SMOOTH_RAS_MIXED", "MEAN_ARITHMETIC",
           "MEAN_GEOMETRIC",
           "ACCEL_FGMRES", "ACCEL_GCR", "ACCEL_ANDERSON", "Markers", "TephraError", "library", "set_allocator"]


def library():
    """The loaded libtephra.so (raises if it has not been built)."""
    return _lib.load()


# ---------------------------------------------------------------- allocator
# The library's device workspace is taken from torch's caching allocator
# (tph_set_allocator with the process-wide default), so that torch accounts
# for it and reuses its blocks; TEPHRA_ALLOCATOR=hip keeps hipMalloc.
def _torch_alloc(nbytes, ctx):
    try:
        dev = torch.cuda.current_device()
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev, stream=torch.cuda.current_stream(dev))
    except Exception:
        return None                      # NULL: the library reports TPH_ERR_OOM


def _torch_free(ptr, ctx):
    try:
        torch.cuda.caching_allocator_delete(ptr)
    except Exception:
        pass


_ALLOC_CB = _lib.ALLOC_FN(_torch_alloc)
_FREE_CB = _lib.FREE_FN(_torch_free)
_allocator = None
_live = weakref.WeakSet()                # handles closed before the interpreter tears torch down


def set_allocator(kind: str = "torch", alloc=None, free=None):
    """Process-wide device allocator of handles created from now on.

    kind "torch": torch's caching allocator; "hip": hipMalloc / hipFree;
    "custom": the ctypes callbacks ``alloc`` (_lib.ALLOC_FN) and ``free``
    (_lib.FREE_FN), which the caller keeps alive.
    """
    global _allocator
    lib = _lib.load()
    if kind == "torch":
        a, f = _ALLOC_CB, _FREE_CB
    elif kind == "hip":
        a, f = _lib.ALLOC_FN(), _lib.FREE_FN()
    elif kind == "custom":
        a, f = alloc, free
    else:
        raise ValueError("kind must be 'torch', 'hip' or 'custom'")
    _lib.check("tph_set_allocator", lib.tph_set_allocator(None, a, f, None))
    _allocator = kind


def _ensure_allocator():
    if _allocator is None:
        set_allocator("hip" if os.environ.get("TEPHRA_ALLOCATOR", "torch") == "hip" else "torch")


@atexit.register
def _close_live_handles():
    for h in list(_live):
        try:
            h.close()
        except Exception:
            pass


@dataclass
class SolveInfo:
    status: str
    iters: int
    restarts: int
    res_energy: float
    res_estimate: float
    t_setup_ms: float
    t_solve_ms: float
    history: list = field(default_factory=list)
    vcycles: int = 0
    res_l2: float = float("nan")


def _ptr(t: Optional[torch.Tensor], shape, name: str):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape {shape}, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One problem size with its device workspace (tph_create)."""

    def __init__(self, nx: int, ny: int, lx: float = 1.0, ly: float = 1.0,
                 bc: Sequence[int] = (FREE_SLIP,) * 4, precision: int = MIXED,
                 levels: int = 0, smoother: int = SMOOTH_GS, nu_pre: int = 2, nu_post: int = 2,
                 nu_growth: float = 1.0, omega: float = 1.0, alpha: float = 1.0,
                 eta_mean: int = MEAN_ARITHMETIC, rtol: float = 1e-8, restart: int = 20,
                 max_iters: int = 500, uzawa_steps: int = 2, fused: bool = True,
                 msweep: int = -1, tile_shape: int = -1, coarse_level: int = -1,
                 accel="fgmres", beta: float = 1.0, ras_tile: int = 32, ras_inner: int = 4, seed: int = 0,
                 graph: bool = False, coarsen: float = 2.0,
                 device: Optional[torch.device] = None,
                 stream: Optional[torch.cuda.Stream] = None):
        lib = _lib.load()
        _ensure_allocator()
        d = _desc(lib, nx, ny, lx=lx, ly=ly, bc=bc, precision=precision, levels=levels, smoother=smoother,
                  nu_pre=nu_pre, nu_post=nu_post, nu_growth=nu_growth, omega=omega, alpha=alpha,
                  eta_mean=eta_mean, rtol=rtol, restart=restart, max_iters=max_iters, uzawa_steps=uzawa_steps,
                  fused=fused, msweep=msweep, tile_shape=tile_shape, coarse_level=coarse_level,
                  accel=accel, beta=beta, ras_tile=ras_tile, ras_inner=ras_inner, seed=seed, graph=graph,
                  coarsen=coarsen)
        self.desc = d
        self.nx, self.ny = nx, ny
        self.shape = (ny + 2, nx + 2)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            _lib.check("tph_create", lib.tph_create(ctypes.byref(d), ctypes.c_void_p(self.stream.cuda_stream),
                                                    ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self.generation = 0           # bumped whenever the solver's coefficients change
        _live.add(self)

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.tph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- helpers --------------------------------------------------------------
    def zeros(self) -> torch.Tensor:
        return torch.zeros(self.shape, dtype=torch.float64, device=self.device)

    def _p(self, t, name):
        return _ptr(t, self.shape, name)

    def _sync_in(self):
        # work queued by torch on another stream must be visible to the library
        if self.stream != torch.cuda.current_stream(self.device):
            self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _info(self, info: _lib.Info, status: int, hist) -> SolveInfo:
        n = min(info.iters, len(hist))
        return SolveInfo(_lib.STATUS_NAMES.get(status, str(status)), info.iters, info.restarts,
                         info.res_energy, info.res_estimate, info.t_setup_ms, info.t_solve_ms,
                         [hist[k] for k in range(n)], vcycles=info.vcycles, res_l2=info.res_l2)

    # -- entry points ---------------------------------------------------------
    @property
    def levels(self) -> int:
        n = 0
        while True:
            nx = ctypes.c_int32()
            st = self._lib.tph_level_shape(self._h, n, ctypes.byref(nx), None)
            if st != 0:
                return n
            n += 1

    def level_shape(self, level: int) -> Tuple[int, int]:
        nx, ny = ctypes.c_int32(), ctypes.c_int32()
        _lib.check("tph_level_shape", self._lib.tph_level_shape(self._h, level, ctypes.byref(nx), ctypes.byref(ny)))
        return nx.value, ny.value

    LEVEL_KINDS = ("tiles", "multisweep", "coarse_tail", "dense", "ras")

    def level_plan(self, level: int) -> Tuple[str, int]:
        """(kernel kind, tile shape) of one level: see tph_level_plan."""
        k, s = ctypes.c_int32(), ctypes.c_int32()
        _lib.check("tph_level_plan", self._lib.tph_level_plan(self._h, level, ctypes.byref(k), ctypes.byref(s)))
        return self.LEVEL_KINDS[k.value], s.value

    def set_coefficients(self, eta_b, eta_p, rho_b, gx: float = 0.0, gy: float = -1.0,
                         fx_extra=None, fy_extra=None):
        self.generation += 1
        self._sync_in()
        _lib.check("tph_set_coefficients", self._lib.tph_set_coefficients(
            self._h, self._p(eta_b, "eta_b"), self._p(eta_p, "eta_p"), self._p(rho_b, "rho_b"),
            float(gx), float(gy), self._p(fx_extra, "fx_extra"), self._p(fy_extra, "fy_extra")))

    def solve(self, vx=None, vy=None, p=None, history: int = 0, raise_on_fail: bool = False):
        vx = self.zeros() if vx is None else vx
        vy = self.zeros() if vy is None else vy
        p = self.zeros() if p is None else p
        info = _lib.Info()
        hist = (ctypes.c_double * max(history, 1))()
        if history:
            info.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
            info.history_len = history
        self._sync_in()
        st = self._lib.tph_solve(self._h, self._p(vx, "vx"), self._p(vy, "vy"), self._p(p, "p"), ctypes.byref(info))
        _lib.check("tph_solve", st, allow_not_converged=not raise_on_fail)
        return vx, vy, p, self._info(info, st, hist if history else [])

    def lithostatic_pressure(self, rho_b, gy: float = -1.0):
        """Zero-mean lithostatic pressure (tph_lithostatic_pressure)."""
        p = self.zeros()
        self._sync_in()
        _lib.check("tph_lithostatic_pressure", self._lib.tph_lithostatic_pressure(
            self._h, self._p(rho_b, "rho_b"), float(gy), self._p(p, "p")))
        return p

    def solve_continuation(self, eta_b, eta_p, rho_b, gx: float = 0.0, gy: float = -1.0,
                           thetas=(0.0, 0.25, 0.5, 0.75, 1.0), stage_rtol: float = 1e-3, lithostatic: bool = True,
                           vx=None, vy=None, p=None, history: int = 0):
        """Viscosity-rescaling continuation solve (tph_solve_continuation); sets the coefficients."""
        vx = self.zeros() if vx is None else vx
        vy = self.zeros() if vy is None else vy
        p = self.zeros() if p is None else p
        self.generation += 1           # the stages load blended coefficients
        th = (ctypes.c_double * len(thetas))(*[float(t) for t in thetas])
        info = _lib.Info()
        hist = (ctypes.c_double * max(history, 1))()
        if history:
            info.history = hist
            info.history_len = history
        self._sync_in()
        st = self._lib.tph_solve_continuation(self._h, self._p(eta_b, "eta_b"), self._p(eta_p, "eta_p"),
                                              self._p(rho_b, "rho_b"), float(gx), float(gy), th, len(thetas),
                                              float(stage_rtol), 1 if lithostatic else 0, self._p(vx, "vx"),
                                              self._p(vy, "vy"), self._p(p, "p"), ctypes.byref(info))
        _lib.check("tph_solve_continuation", st, allow_not_converged=True)
        return vx, vy, p, self._info(info, st, list(hist[:min(info.iters, history)]) if history else [])

    def solve_rhs(self, fx, fy, fp=None, vx=None, vy=None, p=None):
        vx = self.zeros() if vx is None else vx
        vy = self.zeros() if vy is None else vy
        p = self.zeros() if p is None else p
        fp = self.zeros() if fp is None else fp
        info = _lib.Info()
        self._sync_in()
        st = self._lib.tph_solve_rhs(self._h, self._p(fx, "fx"), self._p(fy, "fy"), self._p(fp, "fp"),
                                     self._p(vx, "vx"), self._p(vy, "vy"), self._p(p, "p"), ctypes.byref(info))
        _lib.check("tph_solve_rhs", st, allow_not_converged=True)
        return vx, vy, p, self._info(info, st, [])

    def apply(self, vx, vy, p):
        ax, ay, ap = self.zeros(), self.zeros(), self.zeros()
        self._sync_in()
        _lib.check("tph_apply", self._lib.tph_apply(self._h, self._p(vx, "vx"), self._p(vy, "vy"), self._p(p, "p"),
                                                    self._p(ax, "ax"), self._p(ay, "ay"), self._p(ap, "ap")))
        return ax, ay, ap

    def precondition_apply(self, rx, ry, rp):
        """(z, w) with z = M^{-1} r and w = A z (tph_precondition_apply)."""
        z = (self.zeros(), self.zeros(), self.zeros())
        w = (self.zeros(), self.zeros(), self.zeros())
        self._sync_in()
        _lib.check("tph_precondition_apply", self._lib.tph_precondition_apply(
            self._h, self._p(rx, "rx"), self._p(ry, "ry"), self._p(rp, "rp"), *[self._p(t, "z") for t in z],
            *[self._p(t, "w") for t in w]))
        return z, w

    def precondition(self, rx, ry, rp):
        zx, zy, zp = self.zeros(), self.zeros(), self.zeros()
        self._sync_in()
        _lib.check("tph_precondition", self._lib.tph_precondition(
            self._h, self._p(rx, "rx"), self._p(ry, "ry"), self._p(rp, "rp"),
            self._p(zx, "zx"), self._p(zy, "zy"), self._p(zp, "zp")))
        return zx, zy, zp

    def energy_residual(self, vx, vy, p) -> float:
        out = ctypes.c_double()
        self._sync_in()
        _lib.check("tph_energy_residual", self._lib.tph_energy_residual(
            self._h, self._p(vx, "vx"), self._p(vy, "vy"), self._p(p, "p"), ctypes.byref(out)))
        return out.value

    def level_viscosity(self, level: int):
        nx, ny = self.level_shape(level)
        eb = torch.zeros((ny + 2, nx + 2), dtype=torch.float64, device=self.device)
        ep = torch.zeros_like(eb)
        self._sync_in()
        _lib.check("tph_level_viscosity", self._lib.tph_level_viscosity(
            self._h, level, ctypes.c_void_p(eb.data_ptr()), ctypes.c_void_p(ep.data_ptr())))
        return eb, ep

    def solve_adjoint(self, gvx=None, gvy=None, gp=None):
        lx, ly, lp = self.zeros(), self.zeros(), self.zeros()
        info = _lib.Info()
        self._sync_in()
        st = self._lib.tph_solve_adjoint(self._h, self._p(gvx, "gvx"), self._p(gvy, "gvy"), self._p(gp, "gp"),
                                         self._p(lx, "lvx"), self._p(ly, "lvy"), self._p(lp, "lp"),
                                         ctypes.byref(info))
        _lib.check("tph_solve_adjoint", st, allow_not_converged=True)
        return lx, ly, lp, self._info(info, st, [])

    def time_kernel(self, kind: int, reps: int = 50):
        """(ms per launch, algorithmic bytes per launch) of one hot-path kernel."""
        ms, by = ctypes.c_double(), ctypes.c_double()
        self._sync_in()
        _lib.check("tph_time_kernel", self._lib.tph_time_kernel(self._h, int(kind), int(reps), ctypes.byref(ms),
                                                                ctypes.byref(by)))
        return ms.value, by.value

    def kernel_timing(self, stride: int = 1, target: Optional[int] = None):
        """Time every stride-th launch of the target kernel class of later
        solves (0: off): the finest-level smoother (default) or, with
        target=_lib.KERNEL_LINK, the Uzawa link passes."""
        if target is not None:
            _lib.check("tph_kernel_timing_target", self._lib.tph_kernel_timing_target(self._h, int(target)))
        _lib.check("tph_kernel_timing", self._lib.tph_kernel_timing(self._h, int(stride)))

    def kernel_timing_read(self):
        """(launches, total ms, total algorithmic bytes, dropped) since the last read; resets."""
        n, ms, by, dr = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        _lib.check("tph_kernel_timing_read", self._lib.tph_kernel_timing_read(
            self._h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by), ctypes.byref(dr)))
        return n.value, ms.value, by.value, dr.value

    def coeff_gradient(self, vx, vy, p, lvx, lvy, lp):
        gb, gp, gr = self.zeros(), self.zeros(), self.zeros()
        self._sync_in()
        _lib.check("tph_coeff_gradient", self._lib.tph_coeff_gradient(
            self._h, self._p(vx, "vx"), self._p(vy, "vy"), self._p(p, "p"),
            self._p(lvx, "lvx"), self._p(lvy, "lvy"), self._p(lp, "lp"),
            self._p(gb, "g_eta_b"), self._p(gp, "g_eta_p"), self._p(gr, "g_rho_b")))
        return gb, gp, gr


def _desc(lib, nx, ny, lx=1.0, ly=1.0, bc=(FREE_SLIP,) * 4, precision=MIXED, levels=0, smoother=SMOOTH_GS,
          nu_pre=2, nu_post=2, nu_growth=1.0, omega=1.0, alpha=1.0, eta_mean=MEAN_ARITHMETIC, rtol=1e-8,
          restart=20, max_iters=500, uzawa_steps=2, fused=True, msweep=-1, tile_shape=-1, coarse_level=-1,
          accel="fgmres", beta=1.0, ras_tile=32, ras_inner=4, seed=0, graph=False, coarsen=2.0):
    d = _lib.Desc()
    lib.tph_desc_default(ctypes.byref(d), nx, ny)
    d.lx, d.ly = float(lx), float(ly)
    for w in range(4):
        d.bc[w] = int(bc[w])
    d.precision, d.levels, d.smoother = int(precision), int(levels), int(smoother)
    d.nu_pre, d.nu_post, d.nu_growth = int(nu_pre), int(nu_post), float(nu_growth)
    d.omega, d.alpha, d.eta_mean, d.rtol = float(omega), float(alpha), int(eta_mean), float(rtol)
    d.restart, d.max_iters, d.uzawa_steps, d.fused = int(restart), int(max_iters), int(uzawa_steps), int(bool(fused))
    d.msweep, d.tile_shape, d.coarse_level = int(msweep), int(tile_shape), int(coarse_level)
    d.accel = _lib.ACCEL_NAMES[accel.lower()] if isinstance(accel, str) else int(accel)
    d.beta = float(beta)
    d.ras_tile, d.ras_inner, d.seed = int(ras_tile), int(ras_inner), int(seed)
    d.graph = int(bool(graph))
    d.coarsen = float(coarsen)
    return d


class Batch:
    """Independent problems of uneven sizes solved together (tph_batch_*).

    ``shapes`` is a list of (nx, ny), (nx, ny, lx, ly) or (nx, ny, lx, ly,
    bc); the keyword parameters are shared by every problem (see
    tph_batch_create).
    """

    def __init__(self, shapes, device: Optional[torch.device] = None,
                 stream: Optional[torch.cuda.Stream] = None, **params):
        lib = _lib.load()
        _ensure_allocator()
        self._lib = lib
        self.count = len(shapes)
        self.rtol = float(params.get("rtol", 1e-8))
        descs = (_lib.Desc * self.count)()
        self.shapes = []
        for k, sh in enumerate(shapes):
            nx, ny = int(sh[0]), int(sh[1])
            lx, ly = (float(sh[2]), float(sh[3])) if len(sh) > 2 else (1.0, 1.0)
            kw = dict(params)
            if len(sh) > 4:
                kw["bc"] = tuple(sh[4])          # per-problem boundary conditions
            descs[k] = _desc(lib, nx, ny, lx, ly, **kw)
            self.shapes.append((ny + 2, nx + 2))
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            _lib.check("tph_batch_create", lib.tph_batch_create(self.count, descs,
                                                                ctypes.c_void_p(self.stream.cuda_stream),
                                                                ctypes.byref(h)))
        self._h = h
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.tph_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, tensors, name):
        if len(tensors) != self.count:
            raise ValueError(f"{name}: expected {self.count} tensors")
        arr = (ctypes.c_void_p * self.count)()
        for k, t in enumerate(tensors):
            arr[k] = _ptr(t, self.shapes[k], f"{name}[{k}]")
        return arr

    def _sync_in(self):
        if self.stream != torch.cuda.current_stream(self.device):
            self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def set_coefficients(self, eta_b, eta_p, rho_b, gxy):
        g = (ctypes.c_double * (2 * self.count))()
        for k, (gx, gy) in enumerate(gxy):
            g[2 * k], g[2 * k + 1] = float(gx), float(gy)
        self._sync_in()
        _lib.check("tph_batch_set_coefficients", self._lib.tph_batch_set_coefficients(
            self._h, self._ptrs(eta_b, "eta_b"), self._ptrs(eta_p, "eta_p"), self._ptrs(rho_b, "rho_b"), g))

    def zeros(self):
        return [torch.zeros(s, dtype=torch.float64, device=self.device) for s in self.shapes]

    def solve(self, vx=None, vy=None, p=None):
        vx = self.zeros() if vx is None else vx
        vy = self.zeros() if vy is None else vy
        p = self.zeros() if p is None else p
        infos = (_lib.Info * self.count)()
        self._sync_in()
        st = self._lib.tph_batch_solve(self._h, self._ptrs(vx, "vx"), self._ptrs(vy, "vy"), self._ptrs(p, "p"), infos)
        _lib.check("tph_batch_solve", st, allow_not_converged=True)
        out = [SolveInfo("TPH_OK" if infos[k].res_energy <= self.rtol else "TPH_NOT_CONVERGED", infos[k].iters,
                         infos[k].restarts, infos[k].res_energy, infos[k].res_estimate, infos[k].t_setup_ms,
                         infos[k].t_solve_ms, vcycles=infos[k].vcycles, res_l2=infos[k].res_l2)
               for k in range(self.count)]
        return vx, vy, p, out


def _mptr(t, n, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() \
            or t.dim() != 1 or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of {n} entries")
    return ctypes.c_void_p(t.data_ptr())


class Markers:
    """Marker <-> grid transfers and RK4 advection (tph_markers_*).

    Marker positions and values are 1D float64 CUDA tensors of n entries;
    grids are (ny + 2, nx + 2) float64 tensors.  Node kinds: "basic",
    "cell", "vx", "vy" (see the header).
    """

    def __init__(self, nx: int, ny: int, lx: float = 1.0, ly: float = 1.0, capacity: int = 1 << 20,
                 device: Optional[torch.device] = None, stream: Optional[torch.cuda.Stream] = None):
        lib = _lib.load()
        _ensure_allocator()
        self._lib = lib
        self.nx, self.ny = nx, ny
        self.shape = (ny + 2, nx + 2)
        self.capacity = int(capacity)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            _lib.check("tph_markers_create", lib.tph_markers_create(nx, ny, float(lx), float(ly), self.capacity,
                                                                    ctypes.c_void_p(self.stream.cuda_stream),
                                                                    ctypes.byref(h)))
        self._h = h
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.tph_markers_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_in(self):
        if self.stream != torch.cuda.current_stream(self.device):
            self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _sync_out(self):
        if self.stream != torch.cuda.current_stream(self.device):
            torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def to_grid(self, kind: str, xm, ym, fields, fill: float = 0.0):
        """Normalised bilinear averages of each marker field on the `kind` nodes (one binning)."""
        n = xm.numel()
        self._sync_in()
        _lib.check("tph_markers_bin", self._lib.tph_markers_bin(self._h, _lib.NODE_KINDS[kind], n,
                                                                _mptr(xm, n, "xm"), _mptr(ym, n, "ym")))
        outs = []
        for k, f in enumerate(fields):
            g = torch.zeros(self.shape, dtype=torch.float64, device=self.device)
            _lib.check("tph_markers_to_grid", self._lib.tph_markers_to_grid(self._h, _mptr(f, n, f"fields[{k}]"),
                                                                            float(fill), _ptr(g, self.shape, "grid")))
            outs.append(g)
        self._sync_out()
        return outs

    def from_grid(self, kind: str, xm, ym, grid):
        n = xm.numel()
        out = torch.empty(n, dtype=torch.float64, device=self.device)
        self._sync_in()
        _lib.check("tph_markers_from_grid", self._lib.tph_markers_from_grid(
            self._h, _lib.NODE_KINDS[kind], n, _mptr(xm, n, "xm"), _mptr(ym, n, "ym"), _ptr(grid, self.shape, "grid"),
            _mptr(out, n, "out")))
        self._sync_out()
        return out

    def advect_rk4(self, xm, ym, vx, vy, dt: float):
        """One RK4 step in place."""
        n = xm.numel()
        self._sync_in()
        _lib.check("tph_markers_advect_rk4", self._lib.tph_markers_advect_rk4(
            self._h, n, _mptr(xm, n, "xm"), _mptr(ym, n, "ym"), _ptr(vx, self.shape, "vx"), _ptr(vy, self.shape, "vy"),
            float(dt)))
        self._sync_out()

    def sync(self):
        _lib.check("tph_markers_sync", self._lib.tph_markers_sync(self._h))


def solve(eta_b, eta_p, rho_b, gx: float = 0.0, gy: float = -1.0, lx: float = 1.0, ly: float = 1.0,
          **params):
    """One-shot solve: returns (vx, vy, p, info)."""
    ny, nx = eta_b.shape[0] - 2, eta_b.shape[1] - 2
    with Solver(nx, ny, lx, ly, device=eta_b.device, **params) as s:
        s.set_coefficients(eta_b, eta_p, rho_b, gx, gy)
        return s.solve()


def energy_residual_noalloc(eta_b, eta_p, rho_b, vx, vy, p, out, gx: float = 0.0, gy: float = -1.0,
                            lx: float = 1.0, ly: float = 1.0, bc: Sequence[int] = (FREE_SLIP,) * 4,
                            stream: Optional[torch.cuda.Stream] = None) -> None:
    """tph_energy_residual_noalloc: writes (relative energy residual, plain
    relative l2 residual) of (vx, vy, p) into the 2-element float64 device
    tensor ``out`` on ``stream`` (default: the current stream); no solver,
    no allocation, no synchronisation."""
    lib = _lib.load()
    ny, nx = eta_b.shape[0] - 2, eta_b.shape[1] - 2
    d = _desc(lib, nx, ny, lx=lx, ly=ly, bc=bc)
    shape = (ny + 2, nx + 2)
    if not (isinstance(out, torch.Tensor) and out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
            and out.numel() >= 2):
        raise ValueError("out must be a contiguous float64 CUDA tensor of at least 2 elements")
    st = stream if stream is not None else torch.cuda.current_stream(eta_b.device)
    _lib.check("tph_energy_residual_noalloc", lib.tph_energy_residual_noalloc(
        ctypes.byref(d), _ptr(eta_b, shape, "eta_b"), _ptr(eta_p, shape, "eta_p"), _ptr(rho_b, shape, "rho_b"),
        float(gx), float(gy), _ptr(vx, shape, "vx"), _ptr(vy, shape, "vy"), _ptr(p, shape, "p"),
        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream)))


class StokesFunction(torch.autograd.Function):
    """(eta_b, eta_p, rho_b) -> (vx, vy, p) with a hand-written adjoint backward.

    Forward: tph_set_coefficients + tph_solve on the given solver.  Backward:
    the adjoint solve (A is symmetric) with right-hand side (dJ/dvx, dJ/dvy,
    dJ/dp), then the coefficient-gradient kernel.  The adjoint needs the
    operator of the forward solve: when the solver's coefficients have
    changed in between (another forward on the same solver, a continuation),
    backward loads the saved forward coefficients again.  A forward or
    adjoint solve that does not reach the solver's rtol raises TephraError
    (a gradient of an unconverged state is not the gradient of J).
    """

    @staticmethod
    def forward(ctx, eta_b, eta_p, rho_b, solver: Solver, gx: float = 0.0, gy: float = -1.0):
        eb, ep, rb = eta_b.detach().contiguous(), eta_p.detach().contiguous(), rho_b.detach().contiguous()
        solver.set_coefficients(eb, ep, rb, gx, gy)
        vx, vy, p, info = solver.solve()
        if info.status != "TPH_OK":
            raise TephraError("tph_solve", _lib.TPH_NOT_CONVERGED,
                              f"forward solve of StokesFunction did not converge: relative energy residual "
                              f"{info.res_energy:.3e} after {info.iters} iterations (rtol {solver.desc.rtol:g})")
        ctx.solver = solver
        ctx.info = info
        ctx.generation = solver.generation
        ctx.gravity = (float(gx), float(gy))
        ctx.save_for_backward(vx, vy, p, eb, ep, rb)
        return vx, vy, p

    @staticmethod
    def backward(ctx, gvx, gvy, gp):
        s: Solver = ctx.solver
        vx, vy, p, eb, ep, rb = ctx.saved_tensors
        if s.generation != ctx.generation:
            s.set_coefficients(eb, ep, rb, *ctx.gravity)     # the forward operator again
            ctx.generation = s.generation
        z = lambda g: s.zeros() if g is None else g.contiguous()
        lx, ly, lp, info = s.solve_adjoint(z(gvx), z(gvy), z(gp))
        if info.status != "TPH_OK":
            raise TephraError("tph_solve_adjoint", _lib.TPH_NOT_CONVERGED,
                              f"adjoint solve of StokesFunction did not converge: relative energy residual "
                              f"{info.res_energy:.3e} after {info.iters} iterations (rtol {s.desc.rtol:g})")
        gb, gpp, gr = s.coeff_gradient(vx, vy, p, lx, ly, lp)
        return gb, gpp, gr, None, None, None
